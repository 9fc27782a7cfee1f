// Particle kernels of the lbmd library: velocity-Verlet integration of the
// Langevin equation of Sec. 2 (Eq. NEWTON) coupled to the lattice fluid.
//
// Per step (time step 1):
//   k_begin   conservation terms of the state at the start of the step,
//             half kick, drift, periodic wrap; marks the 8 nodes around each
//             particle in a bit mask and appends newly marked nodes to a
//             compact list (one atomic per wave); counts particles per cell
//             of the pair-force cell list
//   k_scan_*  exclusive scan of the cell counts, then a scatter into
//             cell-sorted order
//   k_pairs   conservative pair forces from the cell list and FENE bonds
//             (second stream, beside the fluid passes; 8 lanes per particle)
//   k_couple8 trilinear interpolation of u_c and grad rho_zeta from the node
//             records (forming the neighbour sums from the density field in
//             the two-pass organisation), friction + solvation (Eq.
//             solvation_kappa) + random force; the opposite coupling force
//             is spread onto the 8 nodes with hardware float atomics (8 lanes
//             per particle, one per node)
//   k_end     second half kick with the coupling and conservative forces
// All particle quantities are float64.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbmd_internal.h"

namespace lbmd {


// Minimum image of a difference d of two positions in [0, L) (so |d| < L):
// a compare and a subtraction instead of an FP64 division.  It differs from
// d - L floor(d / L + 1/2) only at |d| = L/2 exactly, beyond every cut-off
// (the pair and bond ranges are checked to stay below half the box).
__device__ __forceinline__ double min_image(double d, double L) {
  const double h = 0.5 * L;
  return d > h ? d - L : (d < -h ? d + L : d);
}

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ void interp(const double* x, int nx, int ny, int nz, int64_t (&node)[8], double (&W)[8]) {
  const double fx = floor(x[0]), fy = floor(x[1]), fz = floor(x[2]);
  const double dx = x[0] - fx, dy = x[1] - fy, dz = x[2] - fz;
  const int ix = cell_coord(fx, nx), iy = cell_coord(fy, ny), iz = cell_coord(fz, nz);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ox = k & 1, oy = (k >> 1) & 1, oz = (k >> 2) & 1;
    W[k] = (ox ? dx : 1.0 - dx) * (oy ? dy : 1.0 - dy) * (oz ? dz : 1.0 - dz);
    const int X = wrapi(ix + ox, nx), Y = wrapi(iy + oy, ny), Z = wrapi(iz + oz, nz);
    node[k] = (int64_t(Z) * ny + Y) * nx + X;
  }
}

__device__ __forceinline__ int cell_index(const double* x, const PartArgs& A) {
  const double L[3] = {double(A.nx), double(A.ny), double(A.nz)};
  int c[3];
  for (int a = 0; a < 3; ++a) {
    // clamped before the conversion (non-finite positions go to cell 0)
    const double q = x[a] / L[a] * A.ncell[a];
    c[a] = q >= 0.0 && q < double(A.ncell[a]) ? int(q) : (q >= double(A.ncell[a]) ? A.ncell[a] - 1 : 0);
  }
  return (c[2] * A.ncell[1] + c[1]) * A.ncell[0] + c[0];
}

__device__ __forceinline__ void flag_unstable(uint32_t* status, long long* bad, uint32_t bit, long long step) {
  atomicOr(status, bit);
  atomicMin(bad, step);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// one block of 256 particles (block index blk within the lattice's particles)
__device__ __forceinline__ void begin_block(const PartArgs& A, double* __restrict__ x, double* __restrict__ v,
                                            const double* __restrict__ F, const double* __restrict__ Fc,
                                            const int32_t* __restrict__ type, uint32_t* __restrict__ mask,
                                            int32_t* __restrict__ cell_count, int32_t* __restrict__ cell_of,
                                            int32_t* __restrict__ rank_of, double* __restrict__ red, int64_t blk) {
  __shared__ double part[4][3];
  const int64_t p = blk * 256 + threadIdx.x;
  const bool valid = p < A.np;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double mom[3] = {0, 0, 0};
  int64_t node[8];
  double W[8];
  if (valid) {
    const int t = type[p];
    const double m = A.T.mass[t];
    const double L[3] = {double(A.nx), double(A.ny), double(A.nz)};
    double xp[3];
    for (int a = 0; a < 3; ++a) {
      const double va = v[3 * p + a];
      mom[a] = m * va + 0.5 * Fc[3 * p + a];
      const double vn = va + 0.5 * F[3 * p + a] / m;
      v[3 * p + a] = vn;
      xp[a] = wrapd(x[3 * p + a] + vn, L[a]);
      x[3 * p + a] = xp[a];
    }
    if (A.mark_in_begin) interp(xp, A.nx, A.ny, A.nz, node, W);
    if (A.use_cells) {
      const int c = cell_index(xp, A);
      cell_of[p] = c;
      rank_of[p] = atomicAdd(&cell_count[c], 1);
    }
  }
  // mark the 8 nodes here only without a cell list (batches): otherwise they
  // are marked in cell order, where neighbouring particles' nodes share
  // cache lines (push organisation: by the coupling kernel; else by
  // k_mark_sorted after the sort); the fused organisation's list of touched
  // nodes is then compacted from the mask in site order (k_compact)
  if (valid && A.mark_in_begin)
    for (int k = 0; k < 8; ++k) atomicOr(&mask[node[k] >> 5], 1u << (node[k] & 31));
  for (int a = 0; a < 3; ++a) mom[a] = wave_sum(mom[a]);
  if (lane == 0)
    for (int a = 0; a < 3; ++a) part[wv][a] = mom[a];
  __syncthreads();
  if (threadIdx.x < 3) red[3 * blk + threadIdx.x] = part[0][threadIdx.x] + part[1][threadIdx.x] +
                                                   part[2][threadIdx.x] + part[3][threadIdx.x];
}

__global__ __launch_bounds__(256) void k_begin(PartArgs A, double* __restrict__ x, double* __restrict__ v,
                                               const double* __restrict__ F, const double* __restrict__ Fc,
                                               const int32_t* __restrict__ type, uint32_t* __restrict__ mask,
                                               int32_t* __restrict__ cell_count, int32_t* __restrict__ cell_of,
                                               int32_t* __restrict__ rank_of, double* __restrict__ red) {
  begin_block(A, x, v, F, Fc, type, mask, cell_count, cell_of, rank_of, red, blockIdx.x);
}

// The touched-node list of the fused organisation from the mask: block blk
// takes 256 mask words (8,192 sites), scans their bit counts and reserves
// its place in the list with one counter update, then each thread writes
// its word's marked sites in increasing order.  The list is in site order
// within each block's range (the order of the ranges follows the counter
// updates; the re-collision of a node does not depend on it), so that the
// re-collision's consecutive threads pull from neighbouring sites.
constexpr int COMPACT_WORDS = 256;
__device__ __forceinline__ void compact_block(const uint32_t* __restrict__ mask, int64_t words,
                                              int32_t* __restrict__ list, int32_t* __restrict__ nlist, int64_t blk) {
  __shared__ int wsum[COMPACT_WORDS / 64];
  __shared__ int base;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t w = blk * COMPACT_WORDS + threadIdx.x;
  const uint32_t m = w < words ? mask[w] : 0u;
  const int mine = __popc(m);
  int incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int i = 0; i < COMPACT_WORDS / 64; ++i) tot += wsum[i];
    base = tot > 0 ? atomicAdd(nlist, tot) : 0;
  }
  __syncthreads();
  int slot = base + incl - mine;
  for (int i = 0; i < wv; ++i) slot += wsum[i];
  for (uint32_t b = m; b != 0u; b &= b - 1u) list[slot++] = int32_t(w * 32 + (__ffs(b) - 1));
}

__global__ __launch_bounds__(COMPACT_WORDS) void k_compact(const uint32_t* __restrict__ mask, int64_t words,
                                                           int32_t* __restrict__ list, int32_t* __restrict__ nlist) {
  compact_block(mask, words, list, nlist, blockIdx.x);
}

// exclusive scan of cell counts: per-1024 block, then block totals, then add.
// Within a block: inclusive scans of the 16 waves by shuffles, then a scan
// of the 16 wave totals by the first wave (two barriers in all).
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = int(threadIdx.x & 63);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}
// exclusive prefix of v over the 1024 threads of the block; *total = sum
__device__ __forceinline__ int block_excl_scan(int v, int* total) {
  __shared__ int wsum[16];
  const int lane = int(threadIdx.x & 63), wv = int(threadIdx.x >> 6);
  const int incl = wave_incl_scan(v);
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (wv == 0) {
    const int w = wave_incl_scan(lane < 16 ? wsum[lane] : 0);
    if (lane < 16) wsum[lane] = w;
  }
  __syncthreads();
  const int r = (wv > 0 ? wsum[wv - 1] : 0) + incl - v;
  *total = wsum[15];
  __syncthreads();  // wsum is reused by the next call
  return r;
}

__global__ __launch_bounds__(1024) void k_scan_blocks(const int32_t* __restrict__ cnt, int32_t* __restrict__ start,
                                                      int32_t* __restrict__ btot, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  const int32_t v = i < n ? cnt[i] : 0;
  int tot;
  const int ex = block_excl_scan(v, &tot);
  if (i < n) start[i] = ex;
  if (threadIdx.x == 0) btot[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(int32_t* __restrict__ btot, int64_t nb) {
  int32_t carry = 0;
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int32_t v = i < nb ? btot[i] : 0;
    int tot;
    const int ex = block_excl_scan(v, &tot);
    if (i < nb) btot[i] = carry + ex;
    carry += tot;
  }
}

// cell-sorted order: perm[k] = particle at sorted position k, and xs[k] =
// its position and charge, so that a neighbour cell's particles are read as
// one contiguous run
// (the start of cell c is start[c] + btot[c / 1024]: the per-block scan
// plus its block's offset; the cell counts are cleared here for the next
// step, every non-zero count belonging to a cell that holds a particle)
__device__ __forceinline__ int32_t cell_begin(const int32_t* __restrict__ start, const int32_t* __restrict__ btot,
                                              int c) {
  return start[c] + btot[c >> 10];
}
__global__ void k_scatter(const int32_t* __restrict__ cell_of, const int32_t* __restrict__ rank_of,
                          const int32_t* __restrict__ start, const int32_t* __restrict__ btot,
                          int32_t* __restrict__ cnt, int32_t* __restrict__ perm, const double* __restrict__ x,
                          const int32_t* __restrict__ type, ParticleTypes T, double* __restrict__ xs, int64_t np) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int c = cell_of[p];
  const int64_t k = cell_begin(start, btot, c) + rank_of[p];
  cnt[c] = 0;
  perm[k] = int32_t(p);
  xs[4 * k] = x[3 * p];
  xs[4 * k + 1] = x[3 * p + 1];
  xs[4 * k + 2] = x[3 * p + 2];
  xs[4 * k + 3] = T.charge[type[p]];
}

// marks the 8 nodes of each particle in cell order (two-pass and fused
// organisations, which need the mask before the coupling kernel runs)
__global__ void k_mark_sorted(const double* __restrict__ xs, int64_t np, int nx, int ny, int nz,
                              uint32_t* __restrict__ mask) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= np) return;
  const double xp[3] = {xs[4 * k], xs[4 * k + 1], xs[4 * k + 2]};
  int64_t node[8];
  double W[8];
  interp(xp, nx, ny, nz, node, W);
  for (int j = 0; j < 8; ++j) atomicOr(&mask[node[j] >> 5], 1u << (node[j] & 31));
}

__device__ __forceinline__ void add_radial(double fr_over_r, const double (&d)[3], double (&Fp)[3]) {
  // fr = -dU/dr (positive = repulsive), passed divided by r; d points from p
  // to the partner
  for (int a = 0; a < 3; ++a) Fp[a] -= fr_over_r * d[a];
}

// Conservative forces (pair potentials from the cell list, FENE bonds) at
// the new positions; independent of the fluid, so it runs on a second stream
// while the density pass streams the populations.
// sum over the 8 lanes of an aligned lane group, identical on every lane
// (each butterfly level adds the same two values).  The partners come from
// DPP lane moves, no LDS round trip: quad permutations for lane ^ 1 and
// lane ^ 2, then the half-row mirror (lane i of the group with lane 7 - i),
// which after the first two levels holds the other quad's sum, the same
// value lane ^ 4 holds.  All 8 lanes of a group take part together.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b)), CTRL, 0xf, 0xf, false));
  const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), CTRL, 0xf, 0xf, false));
  return __builtin_bit_cast(double, uint64_t(lo) | (uint64_t(hi) << 32));
}
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  v += dpp_move<0x141>(v);  // row_half_mirror: lane 7 - i within 8
  return v;
}

// Pair and bond forces, LANES (1 or 8) lanes per particle in cell order.  The cells
// of one x row are consecutive in the sorted order, so each (y, z) row of
// neighbour cells is one contiguous run of xs (two where the row wraps in
// x); rows and columns of cells whose nearest face lies beyond the cut-off
// from the particle are skipped (the face distance is measured in FP64 with
// a margin, so no pair inside the cut-off is lost).  The lanes look up all
// run bounds together (one round trip to memory) into an LDS table, then
// take consecutive candidates of each run together (with eight lanes, one
// 256-byte piece of xs per round) in one rolled loop over the runs, which
// keeps the kernel at 94 registers.  Each pair term is evaluated as in a
// one-lane loop; eight lanes' partial sums are added by the 8-lane
// butterfly.
constexpr int PAIRS_BLOCK = 256;

// -dU/dr / r of the pair potentials at squared distance r2 (0 beyond both
// cut-offs); qq = q_p q_j
__device__ __forceinline__ double pair_fr_over_r(const PartArgs& A, double r2, double qq, double dh_pre2) {
  const bool wca = A.pp.wca_on && r2 < A.pp.wca_rc2;
  // the square root only for candidates that can lie inside the screened
  // Coulomb cut-off (dh_pre2 is rc^2 rounded up); the cut-off test itself is
  // on r, as in the definition
  if (!(wca || (A.pp.dh_on && r2 < dh_pre2))) return 0.0;
  const double r = sqrt(r2);
  const bool dh = A.pp.dh_on && r < A.pp.dh_rc;
  if (!(wca || dh)) return 0.0;
  const double inv_r = 1.0 / r, inv_r2 = inv_r * inv_r;
  double fr_over_r = 0.0;
  if (wca) {
    const double s2 = A.pp.wca_sigma * A.pp.wca_sigma * inv_r2;
    const double s6 = s2 * s2 * s2;
    fr_over_r += 24.0 * A.pp.wca_eps * (2.0 * s6 * s6 - s6) * inv_r2;
  }
  if (dh) fr_over_r += qq * A.pp.dh_lB * exp(-A.pp.dh_kappa * r) * (1.0 + A.pp.dh_kappa * r) * inv_r2 * inv_r;
  return fr_over_r;
}

template <int LANES>
__global__ __launch_bounds__(PAIRS_BLOCK) void k_pairs(PartArgs A, const double* __restrict__ x,
                                                       const int32_t* __restrict__ type,
                                                       const int32_t* __restrict__ cell_start,
                                                       const int32_t* __restrict__ btot,
                                                       const int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ cell_of,
                                                       const double* __restrict__ xs,
                                                       const int32_t* __restrict__ bstart,
                                                       const int32_t* __restrict__ bnbr, double* __restrict__ Fcons) {
  // per group: the [begin, end) of the up to 18 runs of xs it scans
  static_assert(LANES == 1 || LANES == 8, "one or eight lanes per particle");
  constexpr int PER_BLOCK = PAIRS_BLOCK / LANES;
  __shared__ int2 runs[PER_BLOCK][18];
  const int grp = int(threadIdx.x / LANES), lane = int(threadIdx.x % LANES);
  // sorted position of the group's particle
  const int64_t k = int64_t(blockIdx.x) * PER_BLOCK + grp;
  const bool live = k < A.np;
  const int64_t p = !live ? 0 : (A.use_cells ? int64_t(perm[k]) : k);
  const double xp[3] = {live ? x[3 * p] : 0.0, live ? x[3 * p + 1] : 0.0, live ? x[3 * p + 2] : 0.0};
  double Fp[3] = {0, 0, 0};
  const double L[3] = {double(A.nx), double(A.ny), double(A.nz)};
  if (A.use_cells && (A.pp.wca_on || A.pp.dh_on)) {  // the same for the whole block
    const int c = live ? cell_of[p] : 0;
    const int nc0 = A.ncell[0], nc1 = A.ncell[1], nc2 = A.ncell[2];
    const int cc[3] = {c % nc0, (c / nc0) % nc1, c / (nc0 * nc1)};
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (A.ncell[a] < 3) {  // the whole (periodic) axis is one cell row
        lo[a] = 0;
        hi[a] = 0;
        continue;
      }
      const double edge = L[a] / A.ncell[a];
      const double off = xp[a] - cc[a] * edge;  // distance to the cell's lower face
      const double margin = 1e-9 * L[a];
      lo[a] = off < A.rcut + margin ? -1 : 0;
      hi[a] = edge - off < A.rcut + margin ? 1 : 0;
    }
    // the x run of cells cc[0] + lo .. cc[0] + hi as up to two runs of cell
    // indices within a row, split where it wraps
    int ra0, ra1, rb0 = 0, rb1 = 0;
    const int x0 = cc[0] + lo[0], x1 = cc[0] + hi[0];
    if (nc0 < 3) {
      ra0 = 0;
      ra1 = nc0;
    } else if (x0 < 0) {
      ra0 = nc0 - 1;
      ra1 = nc0;
      rb0 = 0;
      rb1 = x1 + 1;
    } else if (x1 >= nc0) {
      ra0 = x0;
      ra1 = nc0;
      rb0 = 0;
      rb1 = 1;
    } else {
      ra0 = x0;
      ra1 = x1 + 1;
    }
    // the lanes look up the rows' run bounds together (lane l: rows l and
    // l + 8), one round trip to memory
    for (int i = lane; i < 9; i += LANES) {
      const int dz = i / 3 - 1, dy = i % 3 - 1;
      const bool on = live && dz >= lo[2] && dz <= hi[2] && dy >= lo[1] && dy <= hi[1];
      const int row = (wrapi(cc[2] + dz, nc2) * nc1 + wrapi(cc[1] + dy, nc1)) * nc0;
      runs[grp][2 * i] =
          on ? make_int2(cell_begin(cell_start, btot, row + ra0), cell_begin(cell_start, btot, row + ra1))
             : make_int2(0, 0);
      runs[grp][2 * i + 1] = on && rb1 > rb0 ? make_int2(cell_begin(cell_start, btot, row + rb0),
                                                         cell_begin(cell_start, btot, row + rb1))
                                             : make_int2(0, 0);
    }
    __syncthreads();
    const double qp = live ? A.T.charge[type[p]] : 0.0;
    const double dh_pre2 = A.pp.dh_rc * A.pp.dh_rc * (1.0 + 1e-12);
    // where no neighbour cell wraps around the box and the box holds at
    // least 5 cells per axis, every separation is below two cell edges, less
    // than half the box, so the minimum image is the plain difference
    bool inner = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) inner = inner && A.ncell[a] >= 5 && cc[a] + lo[a] >= 0 && cc[a] + hi[a] < A.ncell[a];
    auto scan = [&](auto wrap) {
#pragma unroll 1
      for (int r = 0; r < 18; ++r) {
        const int2 rr = runs[grp][r];
        for (int jj = rr.x + lane; jj < rr.y; jj += LANES) {
          if (jj == k) continue;
          const double4 q = *reinterpret_cast<const double4*>(xs + 4 * int64_t(jj));
          double d[3] = {q.x - xp[0], q.y - xp[1], q.z - xp[2]};
          if (decltype(wrap)::value)
            for (int a = 0; a < 3; ++a) d[a] = min_image(d[a], L[a]);
          const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          const double fr_over_r = pair_fr_over_r(A, r2, qp * q.w, dh_pre2);
          if (fr_over_r != 0.0) add_radial(fr_over_r, d, Fp);
        }
      }
    };
    if (inner)
      scan(std::false_type{});
    else
      scan(std::true_type{});
  }
  if (!live) return;  // whole groups, after the block's barrier
  if (A.pp.fene_on && bstart) {
    for (int jj = bstart[p] + lane; jj < bstart[p + 1]; jj += LANES) {
      const int q = bnbr[jj];
      double d[3];
      for (int a = 0; a < 3; ++a) d[a] = min_image(x[3 * q + a] - xp[a], L[a]);
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double qr = r / A.pp.fene_R0;
      // -dU/dr / r of FENE: -k / (1 - (r/R0)^2)
      const double fr_over_r = qr < 1.0 ? -A.pp.fene_k / (1.0 - qr * qr) : __builtin_nan("");
      add_radial(fr_over_r, d, Fp);
    }
  }
  if (LANES == 1) {
    for (int a = 0; a < 3; ++a) Fcons[3 * p + a] = Fp[a];
  } else {
    const double F0 = group8_sum(Fp[0]), F1 = group8_sum(Fp[1]), F2 = group8_sum(Fp[2]);
    if (lane < 3) Fcons[3 * p + lane] = lane == 0 ? F0 : (lane == 1 ? F1 : F2);
  }
}

// Coupling force: trilinear interpolation of u_c and the lattice density
// gradients (N / c_s^2) from the node records, friction + solvation (Eq.
// solvation_kappa) + random force; total force F = coupling + conservative;
// the opposite coupling force spread onto the 8 nodes.
// Fluid solvation force of particle p (Sec. 2, Eq. solvation_lambda) on the
// 8 vertices of its cell: at vertex r, with d = x_p - r, the links j with
// d . c_j > 0 (Theta read as 0 < cos <= 1) contribute c_j / |c_j|^2 to S_r;
// U_zeta(r) += lambda_zeta S_r (the collision applies -rho_zeta U_zeta) and
// the particle gets back sum_r sum_zeta lambda_zeta rho_zeta(r) S_r, the
// momentum its force gave the fluid.  The link test is exact in FP64 (the
// c_j are 0 or +-1).
template <class C>
__device__ __forceinline__ void solvation_lambda(const PartArgs& A, const double (&xp)[3], int t,
                                                 const int64_t (&node)[8], const C* __restrict__ rec,
                                                 C* __restrict__ gS, double (&back)[3]) {
  const double la = A.T.lambda[t][0], lb = A.T.lambda[t][1];
  const double fl[3] = {floor(xp[0]), floor(xp[1]), floor(xp[2])};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double d[3] = {xp[0] - (fl[0] + (k & 1)), xp[1] - (fl[1] + ((k >> 1) & 1)),
                         xp[2] - (fl[2] + ((k >> 2) & 1))};
    double S[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      const int cx = D3Q19::cx[i], cy = D3Q19::cy[i], cz = D3Q19::cz[i];
      const double dot = d[0] * cx + d[1] * cy + d[2] * cz;
      const double wgt = (cx * cx + cy * cy + cz * cz) == 1 ? 1.0 : 0.5;
      if (dot > 0.0) {
        S[0] += wgt * cx;
        S[1] += wgt * cy;
        S[2] += wgt * cz;
      }
    }
    const double ra = double(rec[node[k] * 16 + 9]), rb = double(rec[node[k] * 16 + 10]);
    for (int a = 0; a < 3; ++a) {
      atomicAdd(&gS[node[k] * 8 + a], C(la * S[a]));
      atomicAdd(&gS[node[k] * 8 + 3 + a], C(lb * S[a]));
      back[a] += (la * ra + lb * rb) * S[a];
    }
  }
}

template <class C>
__device__ __forceinline__ void couple_one(PartArgs A, const double* __restrict__ x, const double* __restrict__ v,
                                           double* __restrict__ F, double* __restrict__ Fc,
                                           const double* __restrict__ Fcons, const int32_t* __restrict__ type,
                                           const C* __restrict__ rec, C* __restrict__ gP, C* __restrict__ gS,
                                           const int32_t* __restrict__ perm, uint32_t* status, long long* bad,
                                           int64_t tid) {
  if (tid >= A.np) return;
  const int64_t step = *A.stepp;  // a local: writing into A would copy it to scratch
  const int64_t p = A.use_cells ? int64_t(perm[tid]) : tid;
  const int t = type[p];
  const double xp[3] = {x[3 * p], x[3 * p + 1], x[3 * p + 2]};
  int64_t node[8];
  double W[8];
  interp(xp, A.nx, A.ny, A.nz, node, W);
  double up[3] = {0, 0, 0}, gA[3] = {0, 0, 0}, gB[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const C* r = rec + node[k] * 16;
    for (int a = 0; a < 3; ++a) {
      gA[a] += W[k] * 3.0 * double(r[a]);
      gB[a] += W[k] * 3.0 * double(r[3 + a]);
      up[a] += W[k] * double(r[6 + a]);
    }
  }
  double R[4] = {0, 0, 0, 0};
  if (A.kT > 0.0) {
    normals4<double>(A.seed, step, uint32_t(p), 0u, 1u, R);
    const double amp = sqrt(2.0 * A.kT * A.gamma);
    for (int a = 0; a < 3; ++a) R[a] *= amp;
  }
  double fc[3], back[3] = {0, 0, 0};
  if (gS && (A.T.lambda[t][0] != 0.0 || A.T.lambda[t][1] != 0.0)) solvation_lambda<C>(A, xp, t, node, rec, gS, back);
  bool ok = true;
  for (int a = 0; a < 3; ++a) {
    fc[a] = -A.gamma * (v[3 * p + a] - up[a]) - (A.T.kappa[t][0] * gA[a] + A.T.kappa[t][1] * gB[a]) + R[a];
    // Fc: everything the fluid exerts on the particle
    Fc[3 * p + a] = fc[a] + back[a];
    const double Ft = fc[a] + back[a] + (Fcons ? Fcons[3 * p + a] : 0.0);
    F[3 * p + a] = Ft;
    ok = ok && isfinite(Ft);
  }
  if (!ok) flag_unstable(status, bad, 2u, step);
  // the interpolated part goes back to the fluid by the same interpolation
#pragma unroll
  for (int k = 0; k < 8; ++k)
    for (int a = 0; a < 3; ++a) atomicAdd(&gP[node[k] * 4 + a], C(-W[k] * fc[a]));
}

// Coupling with 8 lanes per particle (single-job path): lane k owns node k
// of the particle's cell, gathers that node's record, and the 8 partial
// sums are combined with a butterfly of shuffles inside the lane group
// (identical on every lane: each level adds the same two values); every
// lane then has the interpolated u and grad rho, lane 0 writes the forces,
// and each lane spreads onto its own node.  Eight times the parallelism of
// one thread per particle for the scattered record loads and the atomics.
// Same arithmetic as couple_one, with the 8-term sums in tree order.
//
// rho (may be null): the density field [2][N].  With it the node records
// hold only the raw momentum (slots 6-8) and the densities (9, 10), as the
// streaming density pass writes them, and each lane forms its node's
// neighbour sums N_zeta from the field and u_c = (j + g_SC/2)/rho itself;
// Rall (push organisation; may be null): the moment field [3][5][N] whose
// buffer step % 3 holds rho_A, rho_B and the raw momentum of every site of
// this step, used in place of the density field and the records; without
// either the records are complete (fused organisation).
constexpr int COUPLE8_BLOCK = 256;
template <class C>
__global__ __launch_bounds__(COUPLE8_BLOCK) void k_couple8(PartArgs A, const double* __restrict__ x,
                                                           const double* __restrict__ v, double* __restrict__ F,
                                                           double* __restrict__ Fc, const int32_t* __restrict__ type,
                                                           const C* __restrict__ rec, const C* __restrict__ rho,
                                                           const C* __restrict__ Rall, const C* __restrict__ Hall,
                                                           C* __restrict__ gP, C* __restrict__ gS,
                                                           const int32_t* __restrict__ perm, uint32_t* __restrict__ mask,
                                                           uint32_t* status, long long* bad) {
  const int64_t tid = int64_t(blockIdx.x) * (COUPLE8_BLOCK / 8) + (threadIdx.x >> 3);
  const int k = threadIdx.x & 7;
  // every lane of a group takes part in the shuffles; a group past the last
  // particle works on the last one and writes nothing
  const bool on = tid < A.np;
  const int64_t tc = on ? tid : A.np - 1;
  const int64_t step = *A.stepp;  // a local: writing into A would copy it to scratch
  const int64_t p = A.use_cells ? int64_t(perm[tc]) : tc;
  const int t = type[p];
  const double xp[3] = {x[3 * p], x[3 * p + 1], x[3 * p + 2]};
  const double fl[3] = {floor(xp[0]), floor(xp[1]), floor(xp[2])};
  const double d[3] = {xp[0] - fl[0], xp[1] - fl[1], xp[2] - fl[2]};
  const int ox = k & 1, oy = (k >> 1) & 1, oz = (k >> 2) & 1;
  const double Wk = (ox ? d[0] : 1.0 - d[0]) * (oy ? d[1] : 1.0 - d[1]) * (oz ? d[2] : 1.0 - d[2]);
  const int X = wrapi(cell_coord(fl[0], A.nx) + ox, A.nx), Y = wrapi(cell_coord(fl[1], A.ny) + oy, A.ny),
            Z = wrapi(cell_coord(fl[2], A.nz) + oz, A.nz);
  const int64_t nk = (int64_t(Z) * A.ny + Y) * A.nx + X;
  if (on && A.mark_in_couple) atomicOr(&mask[nk >> 5], 1u << uint32_t(nk & 31));
  const C* r = rec + nk * 16;
  // the node's neighbour sums and coupling velocity; ra, rb: its densities
  C NA[3], NB[3], uc[3], ra, rb;
  if (rho || Rall) {
    MomentView<C> mv;
    if (Rall) mv = moment_view<C>(Rall, Hall, step, A.nx, A.ny, A.nz, A.N);
    // density of component c at (xx, yy, zz): the moment field (push
    // organisation) or the density field (two-pass)
    auto dens = [&](int c, int xx, int yy, int zz) -> C {
      return Rall ? mv.at(c, xx, yy, zz) : rho[c * A.N + (int64_t(zz) * A.ny + yy) * A.nx + xx];
    };
    // The neighbours of the cell's 8 nodes fill the 4 x 4 x 4 cube of sites
    // from one below to two above the cell corner.  The group's 8 lanes stage
    // the cube's two density planes in LDS (16 loads each instead of 38),
    // then each lane takes its node's 18 neighbours from it: the same sites
    // and summation order as reading them one by one.
    // one padding word per group, so that the 8 groups' cubes do not start
    // on the same LDS bank
    __shared__ C cube[COUPLE8_BLOCK / 8][2 * 64 + 1];
    const int grp = int(threadIdx.x >> 3);
    {
      const int X0 = cell_coord(fl[0], A.nx), Y0 = cell_coord(fl[1], A.ny), Z0 = cell_coord(fl[2], A.nz);
      // wrap of X0 - 1 .. X0 + 2 into the box (twice: a box may be 1 site wide)
      auto wrap2 = [](int v, int n) { return wrapi(wrapi(v, n), n); };
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int e = k + 8 * m;  // component e / 64, cube site e % 64 (x fastest)
        const int c = e >> 6, cs = e & 63;
        cube[grp][c * 64 + cs] = dens(c, wrap2(X0 - 1 + (cs & 3), A.nx), wrap2(Y0 - 1 + ((cs >> 2) & 3), A.ny),
                                wrap2(Z0 - 1 + (cs >> 4), A.nz));
      }
    }
    __syncthreads();
    auto cub = [&](int c, int i, int j, int l) -> C { return cube[grp][c * 64 + ((l << 4) | (j << 2) | i)]; };
#pragma unroll
    for (int a = 0; a < 3; ++a) NA[a] = NB[a] = C(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      const int cx = D3Q19::cx[i], cy = D3Q19::cy[i], cz = D3Q19::cz[i];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const C wr = weight<C>(i) * cub(c, 1 + ox + cx, 1 + oy + cy, 1 + oz + cz);
        C(&Nc)[3] = c == 0 ? NA : NB;
        if (cx) Nc[0] += cx > 0 ? wr : -wr;
        if (cy) Nc[1] += cy > 0 ? wr : -wr;
        if (cz) Nc[2] += cz > 0 ? wr : -wr;
      }
    }
    ra = Rall ? cub(0, 1 + ox, 1 + oy, 1 + oz) : r[9];
    rb = Rall ? cub(1, 1 + ox, 1 + oy, 1 + oz) : r[10];
    const C inv = C(1) / (ra + rb);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const C gsc = -ra * (C(A.G[0][0]) * NA[a] + C(A.G[0][1]) * NB[a]) -
                    rb * (C(A.G[1][0]) * NA[a] + C(A.G[1][1]) * NB[a]);
      uc[a] = ((Rall ? mv.at(2 + a, X, Y, Z) : r[6 + a]) + C(0.5) * gsc) * inv;
    }
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      NA[a] = r[a];
      NB[a] = r[3 + a];
      uc[a] = r[6 + a];
    }
    ra = r[9];
    rb = r[10];
  }
  double gA[3], gB[3], up[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gA[a] = group8_sum(Wk * 3.0 * double(NA[a]));
    gB[a] = group8_sum(Wk * 3.0 * double(NB[a]));
    up[a] = group8_sum(Wk * double(uc[a]));
  }
  double R[4] = {0, 0, 0, 0};
  if (A.kT > 0.0) {
    normals4<double>(A.seed, step, uint32_t(p), 0u, 1u, R);
    const double amp = sqrt(2.0 * A.kT * A.gamma);
    for (int a = 0; a < 3; ++a) R[a] *= amp;
  }
  double back[3] = {0, 0, 0};
  if (gS && (A.T.lambda[t][0] != 0.0 || A.T.lambda[t][1] != 0.0)) {
    // fluid solvation force at this lane's vertex (as solvation_lambda)
    const double la = A.T.lambda[t][0], lb = A.T.lambda[t][1];
    const double dv[3] = {xp[0] - (fl[0] + ox), xp[1] - (fl[1] + oy), xp[2] - (fl[2] + oz)};
    double S[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      const int cx = D3Q19::cx[i], cy = D3Q19::cy[i], cz = D3Q19::cz[i];
      const double dot = dv[0] * cx + dv[1] * cy + dv[2] * cz;
      const double wgt = (cx * cx + cy * cy + cz * cz) == 1 ? 1.0 : 0.5;
      if (dot > 0.0) {
        S[0] += wgt * cx;
        S[1] += wgt * cy;
        S[2] += wgt * cz;
      }
    }
    for (int a = 0; a < 3; ++a) {
      if (on) {
        atomicAdd(&gS[nk * 8 + a], C(la * S[a]));
        atomicAdd(&gS[nk * 8 + 3 + a], C(lb * S[a]));
      }
      back[a] = group8_sum((la * double(ra) + lb * double(rb)) * S[a]);
    }
  }
  double fc[3];
  bool ok = true;
  for (int a = 0; a < 3; ++a) {
    fc[a] = -A.gamma * (v[3 * p + a] - up[a]) - (A.T.kappa[t][0] * gA[a] + A.T.kappa[t][1] * gB[a]) + R[a];
    const double Ft = fc[a] + back[a] + 0.0;  // the pair forces are added by the second half kick
    if (on && k == 0) {
      Fc[3 * p + a] = fc[a] + back[a];
      F[3 * p + a] = Ft;
    }
    ok = ok && isfinite(Ft);
  }
  if (on && k == 0 && !ok) flag_unstable(status, bad, 2u, step);
  // the interpolated part goes back to the fluid by the same interpolation:
  // -W_k fc_a onto node k.  The 24 values are laid out over the group's
  // lanes so that each atomic instruction covers two (y, z) rows of the
  // cell, the three components of both x nodes of a row being adjacent in
  // memory (gP[4 n + a]): about two cache lines per particle and
  // instruction instead of four.
  if (on) {
    const int X0 = cell_coord(fl[0], A.nx), Y0 = cell_coord(fl[1], A.ny), Z0 = cell_coord(fl[2], A.nz);
#pragma unroll
    for (int it = 0; it < 3; ++it) {
      const int vv = 8 * it + k;  // value index: row (vv / 6), then x node, then component
      const int row = vv / 6, w = vv - 6 * row;
      const int sx = w / 3, a = w - 3 * sx, sy = row & 1, sz = row >> 1;
      const double Ws = (sx ? d[0] : 1.0 - d[0]) * (sy ? d[1] : 1.0 - d[1]) * (sz ? d[2] : 1.0 - d[2]);
      const int64_t ns = (int64_t(wrapi(Z0 + sz, A.nz)) * A.ny + wrapi(Y0 + sy, A.ny)) * A.nx + wrapi(X0 + sx, A.nx);
      const double fa = a == 0 ? fc[0] : (a == 1 ? fc[1] : fc[2]);
      atomicAdd(&gP[ns * 4 + a], C(-Ws * fa));
    }
  }
}

// Second half kick.  Fcons (may be null): the conservative forces, added
// here to the coupling force so that the pair forces can run beside the
// fluid passes; F then holds the total force for the next step's kick.
__device__ __forceinline__ void end_one(PartArgs A, const double* __restrict__ x, double* __restrict__ v,
                                        double* __restrict__ F, const double* __restrict__ Fcons,
                                        const int32_t* __restrict__ type, uint32_t* status, long long* bad,
                                        int64_t p) {
  if (p >= A.np) return;
  const int64_t step = *A.stepp;  // a local: writing into A would copy it to scratch
  const double m = A.T.mass[type[p]];
  bool ok = true;
  for (int a = 0; a < 3; ++a) {
    double Ft = F[3 * p + a];
    if (Fcons) {
      Ft += Fcons[3 * p + a];
      F[3 * p + a] = Ft;
    }
    const double vn = v[3 * p + a] + 0.5 * Ft / m;
    v[3 * p + a] = vn;
    ok = ok && isfinite(Ft) && isfinite(vn) && isfinite(x[3 * p + a]);
  }
  if (!ok) flag_unstable(status, bad, 2u, step);
}

__global__ void k_end(PartArgs A, const double* __restrict__ x, double* __restrict__ v, double* __restrict__ F,
                      const double* __restrict__ Fcons, const int32_t* __restrict__ type, uint32_t* status,
                      long long* bad) {
  end_one(A, x, v, F, Fcons, type, status, bad, int64_t(blockIdx.x) * blockDim.x + threadIdx.x);
}

// ------------------------------------------------------------ launchers
static PartArgs args(const lbmd_ctx* h) {
  PartArgs A;
  A.np = h->np;
  A.nx = h->p.nx;
  A.ny = h->p.ny;
  A.nz = h->p.nz;
  A.N = h->N;
  A.gamma = h->p.gamma;
  A.kT = h->p.kT;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) A.G[a][b] = h->p.G[a][b];
  A.seed = h->p.seed;
  A.stepp = h->step_dev;
  A.T = h->types;
  A.pp = h->pair;
  for (int a = 0; a < 3; ++a) A.ncell[a] = h->ncell[a];
  A.rcut = h->rcut;
  A.use_cells = h->np > 0 && h->cell_start ? 1 : 0;  // particles sorted by cell (always, when there are any)
  A.build_list = organisation_of(h) == LBMD_KERNEL_FUSED ? 1 : 0;
  A.mark_in_couple = organisation_of(h) == LBMD_KERNEL_PUSH ? 1 : 0;
  A.mark_in_begin = !A.mark_in_couple && !A.use_cells ? 1 : 0;
  return A;
}

hipError_t particles_begin(lbmd_ctx* h) {
  PartArgs A = args(h);
  const int64_t nb = (h->np + 255) / 256;
  h->red_part_used = nb;
  hipLaunchKernelGGL(k_begin, dim3(nb), dim3(256), 0, h->stream, A, h->x, h->v, h->F, h->Fc, h->type, h->mask,
                     h->cell_count, h->cell_of, h->rank_of, h->red_part);
  if (A.use_cells) {
    const int64_t n = h->ncells;
    const int64_t nblk = (n + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_blocks, dim3(nblk), dim3(1024), 0, h->stream, h->cell_count, h->cell_start,
                       h->scan_block, n + 1);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, h->stream, h->scan_block, (n + 1 + 1023) / 1024);
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(256), 0, h->stream, h->cell_of, h->rank_of, h->cell_start,
                       h->scan_block, h->cell_count, h->cell_perm, h->x, h->type, h->types, h->xs, h->np);
    if (!A.mark_in_couple)
      hipLaunchKernelGGL(k_mark_sorted, dim3(nb), dim3(256), 0, h->stream, h->xs, h->np, h->p.nx, h->p.ny, h->p.nz,
                         h->mask);
  }
  if (A.build_list) {
    const int64_t words = (h->N + 31) / 32;
    hipLaunchKernelGGL(k_compact, dim3((words + COMPACT_WORDS - 1) / COMPACT_WORDS), dim3(COMPACT_WORDS), 0,
                       h->stream, h->mask, words, h->flag_list, h->nflag);
  }
  return hipGetLastError();
}

bool has_conservative(const lbmd_ctx* h) {
  return h->pair.wca_on || h->pair.dh_on || (h->pair.fene_on && h->bond_start);
}

// Conservative forces on the side stream, ordered after the kick/drift/cell
// sort on the main stream (particles_mark_sorted records that point); they
// run beside the coupling kernel (and the density pass of the two-pass
// organisation), and the main stream waits for them before the
// collide-stream pass.
hipError_t particles_mark_sorted(lbmd_ctx* h) {
  if (!has_conservative(h)) return hipSuccess;
  return hipEventRecord(h->ev_sorted, h->stream);
}

hipError_t particles_pairs(lbmd_ctx* h) {
  if (!has_conservative(h)) return hipSuccess;
  PartArgs A = args(h);
  if (hipError_t e = hipStreamWaitEvent(h->side, h->ev_sorted, 0)) return e;
  // eight lanes per particle where a particle has many candidates (about 6
  // or more on average over the scanned cells), one where it has few: there
  // the eight-lane grid would take slots from the coupling kernel beside it
  const double cand = h->ncells > 0 ? 27.0 * double(h->np) / double(h->ncells) : 0.0;
  if (cand >= 6.0)
    hipLaunchKernelGGL(k_pairs<8>, dim3((h->np + PAIRS_BLOCK / 8 - 1) / (PAIRS_BLOCK / 8)), dim3(PAIRS_BLOCK), 0,
                       h->side, A, h->x, h->type, h->cell_start, h->scan_block, h->cell_perm, h->cell_of, h->xs,
                       h->bond_start, h->bond_nbr, h->Fcons);
  else
    hipLaunchKernelGGL(k_pairs<1>, dim3((h->np + PAIRS_BLOCK - 1) / PAIRS_BLOCK), dim3(PAIRS_BLOCK), 0, h->side, A,
                       h->x, h->type, h->cell_start, h->scan_block, h->cell_perm, h->cell_of, h->xs, h->bond_start,
                       h->bond_nbr, h->Fcons);
  if (hipError_t e = hipGetLastError()) return e;
  return hipEventRecord(h->ev_pairs, h->side);
}

hipError_t particles_join_pairs(lbmd_ctx* h) {
  if (!has_conservative(h)) return hipSuccess;
  return hipStreamWaitEvent(h->stream, h->ev_pairs, 0);
}

hipError_t particles_forces(lbmd_ctx* h) {
  PartArgs A = args(h);
  // pair forces: added by the second half kick
  const int64_t nb = (h->np + COUPLE8_BLOCK / 8 - 1) / (COUPLE8_BLOCK / 8);
  // two-pass organisation: records hold j and rho only, the density field is
  // current; push organisation: the moment field holds both
  const int org = organisation_of(h);
  const void* field = org == LBMD_KERNEL_TWOPASS ? h->rho : nullptr;
  const void* R = org == LBMD_KERNEL_PUSH ? h->R : nullptr;
  const void* H = org == LBMD_KERNEL_PUSH ? h->H : nullptr;
  if (org == LBMD_KERNEL_PUSH && (!R || !H)) return hipErrorInvalidValue;  // the field must be allocated
  if (h->p.precision == LBMD_FP64)
    hipLaunchKernelGGL(k_couple8<double>, dim3(nb), dim3(COUPLE8_BLOCK), 0, h->stream, A, h->x, h->v, h->F, h->Fc,
                       h->type, (const double*)h->rec, (const double*)field, (const double*)R, (const double*)H,
                       (double*)h->gP, (double*)h->gS, h->cell_perm, h->mask, h->status, h->bad_step);
  else
    hipLaunchKernelGGL(k_couple8<float>, dim3(nb), dim3(COUPLE8_BLOCK), 0, h->stream, A, h->x, h->v, h->F, h->Fc,
                       h->type, (const float*)h->rec, (const float*)field, (const float*)R, (const float*)H,
                       (float*)h->gP, (float*)h->gS, h->cell_perm, h->mask, h->status, h->bad_step);
  return hipGetLastError();
}

hipError_t particles_end(lbmd_ctx* h) {
  PartArgs A = args(h);
  const bool cons = has_conservative(h);  // joined before the collide-stream pass
  hipLaunchKernelGGL(k_end, dim3((h->np + 255) / 256), dim3(256), 0, h->stream, A, h->x, h->v, h->F,
                     cons ? (const double*)h->Fcons : nullptr, h->type, h->status, h->bad_step);
  return hipGetLastError();
}

// ------------------------------------------------------------ batches
template <int64_t BatchJob::*BEGIN>
__device__ __forceinline__ int batch_job_of(const BatchJob* __restrict__ jobs, int nj, int64_t u) {
  int lo = 0, hi = nj - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].*BEGIN <= u)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}
__device__ __forceinline__ bool batch_active(const BatchJob& J) { return *J.step < J.target && *J.status == 0u; }

// Each block walks blocks of 256 particles of the flattened particle range.
__global__ __launch_bounds__(256) void k_begin_batch(const BatchJob* __restrict__ jobs,
                                                     const BatchHeader* __restrict__ hdr) {
  __shared__ int act;
  const int nj = hdr->njobs;
  const int64_t total = hdr->npblk;
  for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
    const BatchJob& J = jobs[batch_job_of<&BatchJob::pblk_begin>(jobs, nj, u)];
    if (threadIdx.x == 0) act = batch_active(J) ? 1 : 0;
    __syncthreads();
    const bool a = act != 0;
    __syncthreads();
    if (a)
      begin_block(J.A, J.x, J.v, J.F, J.Fc, J.type, J.mask, nullptr, nullptr, nullptr, J.red_part,
                  u - J.pblk_begin);
    __syncthreads();
  }
}

// Each block walks blocks of 256 mask words of the flattened mask range.
__global__ __launch_bounds__(COMPACT_WORDS) void k_compact_batch(const BatchJob* __restrict__ jobs,
                                                                 const BatchHeader* __restrict__ hdr) {
  __shared__ int act;
  const int nj = hdr->njobs;
  const int64_t total = hdr->ncmpblk;
  for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
    const BatchJob& J = jobs[batch_job_of<&BatchJob::cmp_begin>(jobs, nj, u)];
    if (threadIdx.x == 0) act = batch_active(J) ? 1 : 0;
    __syncthreads();
    const bool a = act != 0;
    __syncthreads();
    if (a) compact_block(J.mask, J.words, J.flag_list, J.nflag, u - J.cmp_begin);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_couple_batch(const BatchJob* __restrict__ jobs,
                                                      const BatchHeader* __restrict__ hdr) {
  const int nj = hdr->njobs;
  const int64_t total = hdr->npblk;
  for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
    const BatchJob& J = jobs[batch_job_of<&BatchJob::pblk_begin>(jobs, nj, u)];
    if (!batch_active(J)) continue;
    couple_one<float>(J.A, J.x, J.v, J.F, J.Fc, nullptr, J.type, J.rec, J.gP, J.gS, nullptr, J.status, J.bad,
                      (u - J.pblk_begin) * 256 + threadIdx.x);
  }
}

__global__ __launch_bounds__(256) void k_end_batch(const BatchJob* __restrict__ jobs,
                                                   const BatchHeader* __restrict__ hdr) {
  const int nj = hdr->njobs;
  const int64_t total = hdr->npblk;
  for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
    const BatchJob& J = jobs[batch_job_of<&BatchJob::pblk_begin>(jobs, nj, u)];
    if (!batch_active(J)) continue;
    end_one(J.A, J.x, J.v, J.F, nullptr, J.type, J.status, J.bad, (u - J.pblk_begin) * 256 + threadIdx.x);
  }
}

constexpr int BATCH_PART_GRID = 1024;

hipError_t batch_particles_begin(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr) {
  hipLaunchKernelGGL(k_begin_batch, dim3(BATCH_PART_GRID), dim3(256), 0, st, jobs, hdr);
  hipLaunchKernelGGL(k_compact_batch, dim3(BATCH_PART_GRID), dim3(COMPACT_WORDS), 0, st, jobs, hdr);
  return hipGetLastError();
}
hipError_t batch_particles_couple(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr) {
  hipLaunchKernelGGL(k_couple_batch, dim3(BATCH_PART_GRID), dim3(256), 0, st, jobs, hdr);
  return hipGetLastError();
}
hipError_t batch_particles_end(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr) {
  hipLaunchKernelGGL(k_end_batch, dim3(BATCH_PART_GRID), dim3(256), 0, st, jobs, hdr);
  return hipGetLastError();
}

// Particle arguments of a batch job: no pair potentials (no cell list), the
// touched nodes compacted into the list for the re-collision.
void batch_fill_particles(const lbmd_ctx* h, BatchJob& J) {
  J.A = args(h);
  J.A.use_cells = 0;
  J.A.build_list = 1;
  J.A.mark_in_couple = 0;
  J.A.mark_in_begin = 1;
  J.x = h->x;
  J.v = h->v;
  J.F = h->F;
  J.Fc = h->Fc;
  J.type = h->type;
  J.red_part = h->red_part;
  J.npblk = (h->np + 255) / 256;
  J.words = (h->N + 31) / 32;
  J.ncmpblk = (J.words + COMPACT_WORDS - 1) / COMPACT_WORDS;
}

}  // namespace lbmd
