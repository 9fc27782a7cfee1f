// Device helpers of the fluid kernels shared by their translation units:
// population access through buffer resources (pulled loads, stores with
// the deviation encoding), the z-march tile with its LDS density ring and
// neighbour sums, block reductions, and the per-step constants.
#pragma once
#include <algorithm>
#include <cmath>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbmd_internal.h"
#include "lbmd_site.h"

namespace lbmd {

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }


// Population arrays are read and written through one buffer resource per
// component: base address in scalar registers, the population's offset
// i*N*sizeof(S) as the scalar offset and the site as a 32-bit vector offset.
// A component's 19 arrays must stay below 4 GiB (checked at create).  An
// access outside the resource's range reads zero instead of faulting.
template <class S>
struct Pops {
  __amdgpu_buffer_rsrc_t r[2];
  uint32_t pstride;  // N * sizeof(S)
  arith_t<S> rho0;   // deviation storage: w_i rho0 is added on load, removed on store
  uint32_t srkey;    // deviation storage: key of the stochastic rounding
};
template <class S>
__device__ __forceinline__ Pops<S> make_pops(const S* base, int64_t N, arith_t<S> rho0 = 0, uint32_t srkey = 0) {
  Pops<S> p;
  p.rho0 = rho0;
  p.srkey = srkey;
  const uint32_t bytes = uint32_t(19 * N * int64_t(sizeof(S)));
#pragma unroll
  for (int c = 0; c < 2; ++c)
    p.r[c] = __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(base + int64_t(c) * 19 * N), (short)0, int(bytes),
                                               0x00020000);
  p.pstride = uint32_t(N * int64_t(sizeof(S)));
  return p;
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float*) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(vo), int(so), 0));
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, double*) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(vo), int(so), 0));
}
template <bool IEEE>
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, dev16<IEEE>*) {
  return dev_decode(__builtin_amdgcn_raw_buffer_load_b16(r, int(vo), int(so), 0), (dev16<IEEE>*)nullptr);
}
// population i of component c at byte offset vo, as the arithmetic type
template <class S>
__device__ __forceinline__ arith_t<S> load_pop(const Pops<S>& p, int c, uint32_t vo, int i) {
  const arith_t<S> v = bload(p.r[c], vo, uint32_t(i) * p.pstride, (S*)nullptr);
  if constexpr (Storage<S>::deviation)
    return v + weight<arith_t<S>>(i) * p.rho0;
  else
    return v;
}
// AUX = 2: non-temporal store hint (the new populations are not read again
// by this step); AUX = 0: plain store
template <int AUX>
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, int(vo), int(so), AUX);
}
template <int AUX>
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) uint32_t, v), r,
                                        int(vo), int(so), AUX);
}

// store population i of component c at byte offset vo (AUX as above);
// r: random bits for the stochastic rounding of a deviation
// Returns the value the next load of it will give (the decoded deviation
// plus w_i rho0 for 16-bit storage, v itself otherwise).
template <int AUX, class S>
__device__ __forceinline__ arith_t<S> put_pop(const Pops<S>& p, int c, uint32_t vo, int i, arith_t<S> v, uint32_t r) {
  if constexpr (Storage<S>::deviation) {
    const uint16_t b = dev_encode_sr(v - weight<float>(i) * p.rho0, r, (S*)nullptr);
    __builtin_amdgcn_raw_buffer_store_b16(b, p.r[c], int(vo), int(uint32_t(i) * p.pstride), AUX);
    return dev_decode(b, (S*)nullptr) + weight<arith_t<S>>(i) * p.rho0;
  } else {
    bstore<AUX>(S(v), p.r[c], vo, uint32_t(i) * p.pstride);
    return v;
  }
}

// fn(i, vo) for the 19 velocities of site (x,y,z), vo = byte offset of the
// upstream site s - c_i (periodic)
template <class S, class Fn>
__device__ __forceinline__ void for_pulled(int x, int y, int z, int nx, int ny, int nz, Fn&& fn) {
  const uint32_t xm = wrapi(x - 1, nx), xp = wrapi(x + 1, nx), x0 = x;
  const uint32_t plane = uint32_t(nx) * uint32_t(ny);
  const uint32_t ym = wrapi(y - 1, ny) * nx, yp = wrapi(y + 1, ny) * nx, y0 = uint32_t(y) * nx;
  const uint32_t zm = wrapi(z - 1, nz) * plane, zp = wrapi(z + 1, nz) * plane, z0 = uint32_t(z) * plane;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const uint32_t sx = D3Q19::cx[i] > 0 ? xm : (D3Q19::cx[i] < 0 ? xp : x0);
    const uint32_t sy = D3Q19::cy[i] > 0 ? ym : (D3Q19::cy[i] < 0 ? yp : y0);
    const uint32_t sz = D3Q19::cz[i] > 0 ? zm : (D3Q19::cz[i] < 0 ? zp : z0);
    fn(i, (sz + sy + sx) * uint32_t(sizeof(S)));
  }
}

// pulled populations of site (x,y,z): f_i(s) = src[i][s - c_i]
template <class S, class C>
__device__ __forceinline__ void pull(const Pops<S>& src, int x, int y, int z, int nx, int ny, int nz,
                                     C (&f)[2][19]) {
  for_pulled<S>(x, y, z, nx, ny, nz, [&](int i, uint32_t vo) {
#pragma unroll
    for (int c = 0; c < 2; ++c) f[c][i] = C(load_pop(src, c, vo, i));
  });
}

// Stores the 38 post-collision populations of site s.  Deviation storage
// draws 32 random bits per velocity (16 per component): the site's word
// mix32(s ^ step key) seeds a xorshift32 sequence whose i-th output serves
// velocity i (cheap shift/xor steps instead of a multiplying hash per
// value), the same on every tiling, organisation and run.
// SPLIT: one branch on the store hint for the whole site; otherwise one per
// velocity, which keeps each pair's stores next to its arithmetic (measured
// faster for the deterministic FP32/FP64 collision, slower with the noise
// or the 16-bit encoding, whose extra arithmetic then sits between stores).
// WB: f receives the stored values as the next step will load them (they
// differ from f only for 16-bit deviation storage, by its rounding).
template <class S, class C, bool SPLIT = false, bool WB = false>
__device__ __forceinline__ void store(const Pops<S>& dst, uint32_t s, C (&f)[2][19], bool nt = true) {
  const uint32_t vo = s * uint32_t(sizeof(S));
  uint32_t hs = 0;
  if constexpr (Storage<S>::deviation) {
    hs = mix32(s ^ dst.srkey);
    if (hs == 0u) hs = 0x9E3779B9u;  // xorshift32 needs a nonzero seed
  }
  auto put2 = [&](auto aux, int i, uint32_t r) {
    const C a = C(put_pop<decltype(aux)::value>(dst, 0, vo, i, arith_t<S>(f[0][i]), r));
    const C b = C(put_pop<decltype(aux)::value>(dst, 1, vo, i, arith_t<S>(f[1][i]), r >> 16));
    if constexpr (WB) {
      f[0][i] = a;
      f[1][i] = b;
    }
  };
  auto put_all = [&](auto aux) {
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      uint32_t r = 0;
      if constexpr (Storage<S>::deviation) r = hs = xorshift32(hs);
      put2(aux, i, r);
    }
  };
  if constexpr (SPLIT) {
    if (nt)
      put_all(std::integral_constant<int, 2>());
    else
      put_all(std::integral_constant<int, 0>());
  } else {
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      uint32_t r = 0;
      if constexpr (Storage<S>::deviation) r = hs = xorshift32(hs);
      if (nt)
        put2(std::integral_constant<int, 2>(), i, r);
      else
        put2(std::integral_constant<int, 0>(), i, r);
    }
  }
}

__device__ __forceinline__ void flag_unstable(uint32_t* status, long long* bad, uint32_t bit, long long step) {
  atomicOr(status, bit);
  atomicMin(bad, step);
}

template <class C>
__device__ __forceinline__ bool moments_ok(const SiteOut<C>& o) {
  return o.rho[0] > C(0) && o.rho[1] > C(0) && isfinite(o.rho[0]) && isfinite(o.rho[1]) && isfinite(o.j[0]) &&
         isfinite(o.j[1]) && isfinite(o.j[2]);
}

// wave64 sum of a double
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block sum of 5 doubles into out[5] (thread 0 writes); nthreads multiple of 64
template <int NW>
__device__ __forceinline__ void block_sum5(double (&v)[5], double* out) {
  __shared__ double part[NW][5];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 5; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 5; ++q) part[wv][q] = v[q];
  __syncthreads();
  if (threadIdx.x < 5) {
    double s = 0;
    for (int w = 0; w < NW; ++w) s += part[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// ------------------------------------------------------------ layouts
// Per-node records (one 64-byte line per node in FP32, two in FP64), written
// at the nodes the particles touch: N_A (3), N_B (3), u_c (3), rho_A,
// rho_B.  The particle force density accumulated at a node: gP[4 * s + a];
// the fluid solvation sums U_zeta (if any lambda is set): gS[8 * s + 3 zeta
// + a].
constexpr int REC = 16;
constexpr int GPS = 4;
constexpr int GSS = 8;

// ------------------------------------------------------------ z-march tiles
// Block = TY waves; wave w owns row y0+w, lane l owns column x0+l of a
// 64-wide tile; the block marches z over [z0, z1).  An LDS ring holds four
// density planes of the tile plus a one-site border; the border sites are
// shared out over the lanes of every wave.
template <int TY>
struct Tile {
  int x0, y0, z0, z1, twv, thv, ringA, nring, x, y, lane, wv;
  bool inside;
  int bid;
  // block: this block's index among the nblk blocks of the lattice
  __device__ Tile(int nx, int ny, int nz, int tz, int tiles_x, int xcd, int block, int nblk) {
    lane = threadIdx.x & 63;
    wv = threadIdx.x >> 6;
    const int nchunk = (nz + tz - 1) / tz;
    int bx, by, bz;
    if (xcd) {
      // blocks are dealt to the 8 XCDs in turn; renumber so that each XCD
      // runs a contiguous range of tiles ordered x, then y, then z: tiles
      // that share border rows then run together on one L2
      const int k = block & 7, m = block >> 3;
      const int q = nblk >> 3, r = nblk & 7;
      bid = k * q + min(k, r) + m;
      const int tiles_y = (ny + TY - 1) / TY;
      bx = bid % tiles_x;
      by = (bid / tiles_x) % tiles_y;
      bz = bid / (tiles_x * tiles_y);
    } else {
      // consecutive block ids walk the z chunks of one column of tiles
      bid = block;
      bz = bid % nchunk;
      const int bxy = bid / nchunk;
      bx = bxy % tiles_x;
      by = bxy / tiles_x;
    }
    x0 = bx * 64;
    y0 = by * TY;
    z0 = bz * tz;
    z1 = min(z0 + tz, nz);
    twv = min(64, nx - x0);
    thv = min(TY, ny - y0);
    inside = lane < twv && wv < thv;
    x = x0 + lane;
    y = y0 + wv;
    ringA = twv + 2;
    nring = 2 * ringA + 2 * thv;
  }
  // ring coordinates of border item h: the row below the tile, the row
  // above, then the left and right columns (rows run along x)
  __device__ void border(int h, int& hr, int& hc) const {
    if (h < ringA) {
      hr = 0;
      hc = h;
    } else if (h < 2 * ringA) {
      hr = thv + 1;
      hc = h - ringA;
    } else if (h < 2 * ringA + thv) {
      hr = 1 + (h - 2 * ringA);
      hc = 0;
    } else {
      hr = 1 + (h - 2 * ringA - thv);
      hc = twv + 1;
    }
  }
  // Calls fn(hr, hc) for the ring sites this thread loads.  Each group of 16
  // lanes takes a run of 16 consecutive border items (16 neighbouring sites
  // of a row: one load instruction touches a few cache lines), and the runs
  // are dealt to the waves in turn, so every wave issues the same number of
  // border loads.
  template <class F>
  __device__ void for_border(F&& fn) const {
    for (int h = (((lane >> 4) * TY + wv) << 4) + (lane & 15); h < nring; h += 64 * TY) {
      int hr, hc;
      border(h, hr, hc);
      fn(hr, hc);
    }
  }
};

// neighbour sums N_zeta = sum_i w_i rho_zeta(r + c_i) c_i from the ring
template <class C, int TY>
__device__ __forceinline__ void nsum_ring(const C (&ring)[4][2][TY + 2][66], int sm, int s0, int sp, int wv, int lane,
                                          C (&NA)[3], C (&NB)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) NA[a] = NB[a] = C(0);
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    const int cx = D3Q19::cx[i], cy = D3Q19::cy[i], cz = D3Q19::cz[i];
    const int sl = cz > 0 ? sp : (cz < 0 ? sm : s0);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const C wr = weight<C>(i) * ring[sl][c][wv + 1 + cy][lane + 1 + cx];
      C(&Nc)[3] = c == 0 ? NA : NB;
      if (cx) Nc[0] += cx > 0 ? wr : -wr;
      if (cy) Nc[1] += cy > 0 ? wr : -wr;
      if (cz) Nc[2] += cz > 0 ? wr : -wr;
    }
  }
}

template <class S>
FluidConsts<arith_t<S>> consts(const lbmd_ctx* h) {
  using C = arith_t<S>;
  FluidConsts<C> K;
  K.nx = h->p.nx;
  K.ny = h->p.ny;
  K.nz = h->p.nz;
  K.N = h->N;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) K.G[a][b] = C(h->p.G[a][b]);
  for (int c = 0; c < 2; ++c) {
    K.tau[c] = C(h->p.tau[c]);
    K.omega[c] = C(1.0 / h->p.tau[c]);
  }
  K.kT = C(h->p.kT);
  K.rho0 = Storage<S>::deviation ? C(h->p.rho0) : C(0);
  for (int q = 0; q < 4; ++q) K.lam[q] = C(h->mrt_lam[q]);
  for (int q = 0; q < 4; ++q) {
    // the mode-group part of the fluctuation amplitude (Appendix, Eq. MODES):
    // each site multiplies it by sqrt(rho_zeta) and a per-mode constant
    const double l1 = 1.0 + (h->mrt ? h->mrt_lam[q] : -1.0 / h->p.tau[0]);
    K.namp[q] = C(std::sqrt(std::max(0.0, 3.0 * h->p.kT * (1.0 - l1 * l1))));
  }
  K.srkey = 0;  // set from the device step counter in the kernel
  K.forcing = h->p.forcing;
  K.noise = h->p.kT > 0.0;
  K.seed = h->p.seed;
  K.step = 0;  // likewise
  K.stepp = h->step_dev;
  K.nt = h->nt;
  return K;
}

}  // namespace lbmd
