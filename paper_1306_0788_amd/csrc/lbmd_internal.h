// Internal declarations of the lbmd HIP library (gfx950).  Device helpers,
// the context structure and the kernel launchers shared by the translation
// units of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbmd.h"

namespace lbmd {

// ---------------------------------------------------------------- D3Q19
// Velocities (Appendix, Eq. velo) with opposite pairs adjacent; weights
// (Eq. weights).  The order is the exported population order.
struct D3Q19 {
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
};
template <class C>
__host__ __device__ constexpr C weight(int i) {
  return i == 0 ? C(1) / C(3) : (i <= 6 ? C(1) / C(18) : C(1) / C(36));
}

// ------------------------------------------------------------ storage types
// Population storage.  float and double hold f itself and are also the
// arithmetic type.  dev16<IEEE> holds the deviation f_i - w_i rho0 in 16 bits
// (IEEE binary16 or bfloat16, round to nearest even) with float arithmetic:
// near the rest state the deviation is a few per cent of w_i rho0, so the
// 16-bit mantissa is spent on the part of f that changes.
template <bool IEEE>
struct dev16 {
  uint16_t bits;
};
using half_dev = dev16<true>;
using bf16_dev = dev16<false>;

template <class S>
struct Storage {
  using C = S;  // arithmetic type
  static constexpr bool deviation = false;
};
template <bool IEEE>
struct Storage<dev16<IEEE>> {
  using C = float;
  static constexpr bool deviation = true;
};
template <class S>
using arith_t = typename Storage<S>::C;

__device__ __forceinline__ float dev_decode(uint16_t b, dev16<true>*) {
  return float(__builtin_bit_cast(_Float16, b));
}
__device__ __forceinline__ float dev_decode(uint16_t b, dev16<false>*) {
  return float(__builtin_bit_cast(__bf16, b));
}
__device__ __forceinline__ uint16_t dev_encode(float v, dev16<true>*) {
  return __builtin_bit_cast(uint16_t, _Float16(v));
}
__device__ __forceinline__ uint16_t dev_encode(float v, dev16<false>*) {
  return __builtin_bit_cast(uint16_t, __bf16(v));
}

// 32-bit integer mixer (the "lowbias32" hash of C. Wellons' hash-prospector
// search: xor-shift / multiply rounds, a bijection with low avalanche bias).
__host__ __device__ constexpr uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// xorshift32 (Marsaglia, "Xorshift RNGs", 2003): one step of the 13/17/5
// shift triple, a bijection on the nonzero 32-bit words.
__host__ __device__ constexpr uint32_t xorshift32(uint32_t x) {
  x ^= x << 13;
  x ^= x >> 17;
  x ^= x << 5;
  return x;
}

// Stochastic rounding of a stored deviation: r (16 random bits) is added
// below the kept mantissa bits of |v| and the rest truncated, so the stored
// value rounds up with probability equal to the discarded fraction and is
// unbiased per value.  Round-to-nearest would err the same way at every
// site of a nearly uniform phase (the deviations there all sit near one
// value) and drift the mass coherently.  Non-finite values round to nearest.
__device__ __forceinline__ uint16_t dev_encode_sr(float v, uint32_t r, dev16<false>*) {
  const uint32_t b = __builtin_bit_cast(uint32_t, v);
  if ((b & 0x7f800000u) == 0x7f800000u) return dev_encode(v, (dev16<false>*)nullptr);
  return uint16_t((b + (r & 0xffffu)) >> 16);  // bfloat16 keeps the top 16 bits
}
__device__ __forceinline__ uint16_t dev_encode_sr(float v, uint32_t r, dev16<true>*) {
  const uint32_t b = __builtin_bit_cast(uint32_t, v);
  if ((b & 0x7f800000u) == 0x7f800000u) return dev_encode(v, (dev16<true>*)nullptr);
  // binary16 keeps 10 of the 23 mantissa bits: randomise the low 13 and
  // truncate; the conversion of the truncated float is then exact in the
  // normal range of binary16 (below it, about 6e-5, it rounds to nearest)
  const uint32_t t = (b + (r & 0x1fffu)) & ~0x1fffu;
  return dev_encode(__builtin_bit_cast(float, t), (dev16<true>*)nullptr);
}

// ------------------------------------------------------------ particle positions
// Position wrapped into [0, L).  Far outside the box (only after a numerical
// failure: velocities diverge before they turn non-finite) x - L floor(x/L)
// is inexact, so such values are folded with the exact fmod; NaN stays NaN
// (the failure check sees it).
__host__ __device__ inline double wrapd(double x, double L) {
  x -= L * std::floor(x / L);
  if (x >= L) x -= L;
  if (x < 0.0) x += L;
  if (!(x >= 0.0 && x < L) && std::isfinite(x)) {
    x = std::fmod(x, L);
    if (x < 0.0) x += L;
    if (!(x < L)) x = 0.0;
  }
  return x;
}

// Lattice cell of a coordinate floor(x) for a box of n sites: 0 <= f < n
// for every position the integrator produces; anything else (non-finite or
// out of range after a numerical failure, which is flagged on its own) is
// mapped into the box so that no node index leaves the lattice.
__host__ __device__ inline int cell_coord(double f, int n) {
  if (f >= 0.0 && f < double(n)) return int(f);
  if (!std::isfinite(f)) return 0;
  double g = std::fmod(f, double(n));
  if (g < 0.0) g += double(n);
  return (g >= 0.0 && g < double(n)) ? int(g) : 0;
}

// ------------------------------------------------------------ Philox4x32-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds; each round
// multiplies words 0 and 2 by fixed 32-bit constants, xors the high halves
// with the other two words and the round key, and bumps the key by two Weyl
// constants.  Counter layout used by the library: (index, step low word,
// draw block | stream tag << 16, step high word); key = seed.
struct U4 {
  uint32_t x, y, z, w;
};
__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = uint64_t(0xD2511F53u) * c.x;
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c.z;
    U4 n;
    // three-input exclusive or in one instruction (truth table 0x96: set
    // where an odd number of the inputs is set)
    n.x = __builtin_amdgcn_bitop3_b32(uint32_t(p1 >> 32), c.y, k0, 0x96);
    n.y = uint32_t(p1);
    n.z = __builtin_amdgcn_bitop3_b32(uint32_t(p0 >> 32), c.w, k1, 0x96);
    n.w = uint32_t(p0);
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Box-Muller pair from two words; u = (word + 1/2) / 2^32 in (0, 1).
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1) {
  const double u1 = (double(a) + 0.5) * 2.3283064365386963e-10;
  const double u2 = (double(b) + 0.5) * 2.3283064365386963e-10;
  const double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  z0 = r * c;
  z1 = r * s;
}
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
  const float u1 = (float(a) + 0.5f) * 2.3283064365386963e-10f;
  const float u2 = (float(b) + 0.5f) * 2.3283064365386963e-10f;
  // -2 ln u1 = -2 ln(2) log2(u1) with the hardware base-2 logarithm and
  // square root: u1 >= 2^-33 and -2 ln u1 >= 2.3e-10 are normal numbers, so
  // the instructions need none of the library's denormal scaling
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
  // hardware sine/cosine take the angle in turns
  z0 = r * __builtin_amdgcn_cosf(u2);
  z1 = r * __builtin_amdgcn_sinf(u2);
}

template <class C>
__device__ __forceinline__ void normals4(uint64_t seed, int64_t step, uint32_t index, uint32_t block,
                                         uint32_t tag, C* z) {
  U4 c{index, uint32_t(step), block | (tag << 16), uint32_t(uint64_t(step) >> 32)};
  U4 o = philox4x32_10(c, uint32_t(seed), uint32_t(seed >> 32));
  box_muller(o.x, o.y, z[0], z[1]);
  box_muller(o.z, o.w, z[2], z[3]);
}

// --------------------------------------------------------------- context
struct ParticleTypes {
  double kappa[LBMD_MAX_TYPES][2];
  double mass[LBMD_MAX_TYPES];
  double charge[LBMD_MAX_TYPES];
  double lambda[LBMD_MAX_TYPES][2];  // fluid solvation lambda_A, lambda_B
  int32_t ntypes;
  int32_t lambda_on;  // any lambda != 0
};

struct PairParams {
  int32_t wca_on, dh_on, fene_on;
  double wca_sigma, wca_eps, wca_rc2;
  double dh_kappa, dh_rc, dh_lB;
  double fene_k, fene_R0;
};

// Scalar parameters of the particle kernels, passed by value.
struct PartArgs {
  int64_t np;
  int nx, ny, nz;
  int64_t N;
  double gamma, kT;
  double G[2][2];        // Shan-Chen coupling matrix (node records formed in the coupling kernel)
  uint64_t seed;
  const int64_t* stepp;  // device step counter
  ParticleTypes T;
  PairParams pp;
  int ncell[3];
  double rcut;  // largest non-bonded cut-off (cells farther than it are skipped)
  int use_cells;  // particles sorted by cell (perm, xs) this step
  int build_list;  // compact the touched nodes into a list after the marks (fused organisation)
  int mark_in_couple;  // the coupling kernel marks the touched nodes (push organisation)
  int mark_in_begin;   // the half kick marks them (no cell list: batches)
};

// Scalar parameters of one fluid step, passed by value to the kernels.
template <class C>
struct FluidConsts {
  int nx, ny, nz;
  int64_t N;
  C G[2][2];
  C omega[2];   // 1/tau
  C tau[2];
  C kT;
  int forcing;  // LBMD_FORCE_*
  int noise;    // kT > 0
  uint64_t seed;
  int64_t step;         // filled in the kernel from *stepp (load_step)
  const int64_t* stepp; // device step counter, advanced by the last kernel of a step
  int nt;  // non-temporal hint on the population stores
  C rho0;  // reference density of deviation storage (0 otherwise)
  uint32_t srkey;  // per-step key of the stochastic rounding of deviations (load_step)
  C lam[4];        // MRT eigenvalues {momentum, bulk, shear, kinetic} (MRT kernels only)
  C namp[4];       // fluctuation factor per mode group, sqrt(3 kT (1 - (1 + lambda_g)^2))
                   // (same group order; BGK: lambda_g = -1/tau_A for every group)
};

// Step index of the launch from the device counter (so that a captured step
// sequence can be replayed), and the stochastic-rounding key derived from it.
template <class C>
__device__ __forceinline__ void load_step(FluidConsts<C>& K) {
  K.step = *K.stepp;
  K.srkey = mix32(uint32_t(K.step) ^
                  mix32(uint32_t(uint64_t(K.step) >> 32) ^ mix32(uint32_t(K.seed) ^ uint32_t(K.seed >> 32))));
}

// ------------------------------------------------------------ moment field
// Moments of one step for the push organisation: rho_A, rho_B and the raw
// momentum j of every site, R[q][N] (q = 0..4), plus the contributions that
// crossed an x boundary of the 64-wide tiles the previous pass used, kept
// apart so that they could be written without atomics:
// H[tile][side][q][z][y], side 0 = the column left of the tile, side 1 = the
// column right of it.  A site in the first column of tile b receives its
// left neighbour tile's side-1 entry, one in the last column its right
// neighbour tile's side-0 entry (periodic in the tile index).  Accessed
// through buffer resources: a 32-bit byte offset per lane and the
// quantity's offset as a scalar (the field stays below 4 GiB).
template <class C>
__device__ __forceinline__ C rsrc_load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  if constexpr (sizeof(C) == 8)
    return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64(r, int(vo), int(so), 0));
  else
    return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b32(r, int(vo), int(so), 0));
}
template <class C>
__device__ __forceinline__ void rsrc_store(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, C v) {
  if constexpr (sizeof(C) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) uint32_t, v), r,
                                          int(vo), int(so), 0);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, int(vo), int(so), 0);
}
template <class C>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const C* base, uint64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<C*>(base), (short)0, int(uint32_t(bytes)), 0x00020000);
}

template <class C>
struct MomentView {
  __amdgpu_buffer_rsrc_t R, H;
  uint32_t qR;     // bytes between quantities of R (N values)
  uint32_t qH;     // bytes between quantities of a side block (nz * ny values)
  uint32_t sideH;  // bytes of one side block (5 quantities)
  int nx, ny, nz, tiles_x;
  __device__ __forceinline__ C at(int q, int x, int y, int z) const {
    const uint32_t s = (uint32_t(z) * uint32_t(ny) + uint32_t(y)) * uint32_t(nx) + uint32_t(x);
    C v = rsrc_load<C>(R, s * uint32_t(sizeof(C)), uint32_t(q) * qR);
    const int bx = x >> 6, xl = x & 63;
    const int tw = nx - (bx << 6) < 64 ? nx - (bx << 6) : 64;
    const uint32_t off = (uint32_t(z) * uint32_t(ny) + uint32_t(y)) * uint32_t(sizeof(C));
    // the side-buffer terms at the first and last column of a tile, without
    // branches: elsewhere the offset lies beyond the side buffer's record
    // count, where a raw buffer load returns zero and touches no memory
    // (adding that zero leaves v unchanged)
    const uint32_t ol = xl == 0 ? off + uint32_t(2 * (bx == 0 ? tiles_x - 1 : bx - 1) + 1) * sideH : kBeyond;
    const uint32_t orr = xl == tw - 1 ? off + uint32_t(2 * (bx == tiles_x - 1 ? 0 : bx + 1)) * sideH : kBeyond;
    v += rsrc_load<C>(H, ol, uint32_t(q) * qH);
    return v + rsrc_load<C>(H, orr, uint32_t(q) * qH);
  }
  static constexpr uint32_t kBeyond = 0xFFFFFF00u;  // above any side buffer (< 4 GiB)
};
// the view of step `step` into R[3][5][N] and H[2][tiles_x][2][5][nz][ny]
template <class C>
__device__ __forceinline__ MomentView<C> moment_view(const C* Rall, const C* Hall, int64_t step, int nx, int ny,
                                                     int nz, int64_t N) {
  MomentView<C> v;
  v.tiles_x = (nx + 63) >> 6;
  v.qR = uint32_t(N) * uint32_t(sizeof(C));
  v.qH = uint32_t(nz) * uint32_t(ny) * uint32_t(sizeof(C));
  v.sideH = 5 * v.qH;
  v.R = rsrc_of(Rall + int64_t(uint64_t(step) % 3u) * 5 * N, uint64_t(5) * v.qR);
  v.H = rsrc_of(Hall + int64_t(step & 1) * v.tiles_x * 2 * 5 * int64_t(nz) * ny,
                uint64_t(v.tiles_x) * 2 * v.sideH);
  v.nx = nx;
  v.ny = ny;
  v.nz = nz;
  return v;
}

}  // namespace lbmd

namespace lbmd {
// One job of a multi-lattice batch (FP32 populations, the paper's forcing,
// fused organisation).  The batch kernels walk the flattened work of all
// jobs: lattice tiles, blocks of 256 particles and blocks of 256 entries of
// the touched-node list, each job owning a contiguous range.  A job advances
// while its step counter is below its target and its status word is clear;
// the current populations are f[step & 1].
struct BatchJob {
  FluidConsts<float> K;  // K.stepp = step
  int64_t* step;
  int64_t target;
  const float* f[2];
  uint32_t* mask;  // nullptr without particles
  float* rec;
  float* gP;
  float* gS;  // fluid solvation sums (nullptr without lambda)
  double* red_fluid;
  double* red_part;
  double* red_out;
  uint32_t* status;
  long long* bad;
  int32_t* flag_list;
  int32_t* nflag;
  int tiles_x, tz, nblk;  // fused tiling, 4 rows per tile
  PartArgs A;             // A.stepp = step
  double* x;
  double* v;
  double* F;
  double* Fc;
  int32_t* type;
  int64_t npblk, nfixblk;                     // particle and node-list blocks
  int64_t words, ncmpblk;                     // mask words, their compaction blocks
  int64_t tile_begin, pblk_begin, fix_begin;  // offsets in the flattened work
  int64_t cmp_begin;
};
struct BatchHeader {
  int32_t njobs;
  int32_t pad;
  int64_t ntiles, npblk, nfixblk, ncmpblk;
};
constexpr int BATCH_TY = 4;
constexpr int BATCH_FLUID_GRID = 2048;  // blocks of the fused batch kernel
// launchers (lbmd_fluid.hip / lbmd_particles.hip); grids are fixed so that a
// captured step serves any composition of the job table
hipError_t batch_fluid_pass(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr, bool noise);
hipError_t batch_fluid_fix(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr, bool noise);
hipError_t batch_finalize(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr, int max_jobs);
hipError_t batch_particles_begin(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr);
hipError_t batch_particles_couple(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr);
hipError_t batch_particles_end(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr);
hipError_t batch_gather(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr, int max_jobs, int64_t* out);
void batch_fill_fluid(const lbmd_ctx* h, BatchJob& J, int tz);  // K, buffers, tiling
void batch_fill_particles(const lbmd_ctx* h, BatchJob& J);  // A, particle buffers
}  // namespace lbmd

struct lbmd_batch_s;

struct lbmd_ctx {
  lbmd_params p;
  int64_t N = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t side = nullptr;  // second stream: pair forces next to the density pass
  hipEvent_t ev_sorted = nullptr, ev_pairs = nullptr;
  size_t s_bytes = 8;  // bytes per stored population
  size_t c_bytes = 8;  // bytes per arithmetic value (density field, records, node forces)

  // fluid state: populations in the pull layout (buffer value at s for
  // velocity i streams to s + c_i at the next step)
  void* f[2] = {nullptr, nullptr};
  int cur = 0;
  void* rho = nullptr;  // [2][N] density field (two-pass kernel)
  int tile_y = 8, tile_z = 16;
  int hold = 1;  // fused kernel keeps the next plane's populations in registers
  int xcd = 0;   // XCD-aware block order of the z-march kernels
  int nt = 1;    // non-temporal population stores
  bool tiling_set = false;  // false: per-organisation defaults (see tiles())

  // particle coupling
  uint32_t* mask = nullptr;  // one bit per site: touched by a particle
  int32_t* flag_list = nullptr;
  int32_t* nflag = nullptr;  // device counter
  int64_t flag_cap = 0;
  void* rec = nullptr;  // [N][16]: N_A(3), N_B(3), u_c(3), rho_A, rho_B at touched nodes
  void* R = nullptr;    // push organisation: moment field [3][5][N], step n in R[n % 3]
  void* H = nullptr;    // and its x-boundary terms [2][tiles_x][2][5][nz][ny], step n in H[n % 2]
  int64_t push_step = -1;  // step whose moments R[step % 3] holds (-1: none)
  void* gP = nullptr;   // [N][4]: particle force density accumulated at nodes
  void* gS = nullptr;   // [N][8]: fluid solvation sums U_A(3), U_B(3) (with lambda only)

  // particles (always float64)
  int64_t np = 0, np_cap = 0;
  double *x = nullptr, *v = nullptr, *F = nullptr, *Fc = nullptr;
  double* Fcons = nullptr;  // conservative forces of the step being taken
  int32_t* type = nullptr;
  int32_t* cell_of = nullptr;  // pair-force cell of each particle
  double* xs = nullptr;        // [n][4] positions and charges in cell order (pair forces)
  int32_t* rank_of = nullptr;  // arrival rank inside its cell
  lbmd::ParticleTypes types;
  lbmd::PairParams pair;
  double rcut = 0.0;  // largest non-bonded cut-off
  int ncell[3] = {1, 1, 1};
  int64_t ncells = 0;
  int32_t *cell_count = nullptr, *cell_start = nullptr, *cell_perm = nullptr;
  int32_t* scan_block = nullptr;
  int64_t nbonds = 0;
  int32_t *bond_start = nullptr, *bond_nbr = nullptr;  // CSR, both directions

  // reductions and status
  double* red_fluid = nullptr;  // [blocks][5]
  int64_t red_fluid_cap = 0;
  int64_t red_fluid_used = 0;
  double* red_part = nullptr;  // [blocks][3]
  int64_t red_part_cap = 0;
  int64_t red_part_used = 0;
  double* red_out = nullptr;     // [8]
  uint32_t* status = nullptr;    // bit 0: fluid, bit 1: particles
  long long* bad_step = nullptr; // first failing step
  double* export_tmp = nullptr;  // staging for host transfers
  size_t export_cap = 0;

  int64_t step = 0;              // steps enqueued (host count)
  int64_t* step_dev = nullptr;   // steps completed on the device (kernels read it)
  bool latched = false;
  std::string err;

  lbmd_batch_s* batch = nullptr;  // attached to a multi-lattice batch
  bool mrt = false;                // MRT collision (two-pass and push organisations)
  double mrt_lam[4] = {0, 0, 0, 0};  // momentum, bulk, shear, kinetic

  // replay of captured two-step sequences, one per ping-pong parity
  bool use_graph = false;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};

  // optional event timing of the collide-stream kernel
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;  // start/stop pairs
  size_t prof_n = 0;                // pairs recorded
};

namespace lbmd {
// event pair around a timed launch (no-op unless timing is enabled)
hipError_t prof_begin(lbmd_ctx* h);
hipError_t prof_end(lbmd_ctx* h);
// launchers (lbmd_fluid.hip)
hipError_t fluid_init(lbmd_ctx* h, const double* rho_dev);
hipError_t fluid_import(lbmd_ctx* h, const double* pop_dev);
// field: [2][N] density-field scratch in the arithmetic type (the export
// writes it, then reads it for the neighbour sums of u)
hipError_t fluid_export(lbmd_ctx* h, uint32_t mask, double* out_dev, void* field);
hipError_t fluid_pull_copy(lbmd_ctx* h);
hipError_t fluid_pass_a(lbmd_ctx* h);  // moments, SC force, records (+ fused collide)
hipError_t fluid_pass_b(lbmd_ctx* h);  // collision with the particle force
hipError_t finalize_step(lbmd_ctx* h);  // reductions, counters
int organisation_of(const lbmd_ctx* h);  // LBMD_KERNEL_FUSED, _TWOPASS or _PUSH this step
// push organisation (lbmd_push.hip)
struct PushLaunch {
  int ty, tz, tiles_x, xcd;
  int64_t nblk;
};
hipError_t push_init(lbmd_ctx* h);  // R[step % 3] from the populations, the other two cleared
// most rows per tile of the push kernel: 16 only for the deterministic BGK
// step with 4-byte arithmetic (FP64's LDS ring and row exchange do not fit
// 160 KiB at 16 rows; the fluctuating and MRT kernels need about 190
// registers, which 1,024 threads per block cannot have)
inline int push_rows_max(const lbmd_ctx* h) {
  return h->p.precision == LBMD_FP64 || h->p.kT > 0.0 || h->mrt ? 8 : 16;
}
hipError_t push_pass(lbmd_ctx* h, const PushLaunch& L);  // collide + stream + next moments
// launchers (lbmd_particles.hip)
hipError_t particles_begin(lbmd_ctx* h);  // reduction terms, half kick, drift, flags, cells
hipError_t particles_mark_sorted(lbmd_ctx* h);  // cell sort done (event for the side stream)
hipError_t particles_pairs(lbmd_ctx* h);  // conservative forces (side stream)
hipError_t particles_join_pairs(lbmd_ctx* h);  // main stream waits for them
hipError_t particles_forces(lbmd_ctx* h); // coupling forces, total force, spread
hipError_t particles_end(lbmd_ctx* h);    // second half kick
}  // namespace lbmd
