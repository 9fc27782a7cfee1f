// Fluid kernels of the lbmd library (gfx950, wave64).
//
// Storage: populations are structure-of-arrays [zeta][i][z][y][x] (x fastest)
// in "pull" form: the value stored for velocity i at site s is the
// post-collision population that streams to s + c_i.  A step therefore reads
// src[zeta][i][s - c_i] (the post-streaming population at s) and writes the
// new post-collision value to dst[zeta][i][s]: 38 coalesced reads and 38
// coalesced writes per site, the algorithmic minimum of one LB step.
//
// The Shan-Chen force at s needs the densities of the 18 neighbours
// (Sec. 2, Eq. SCforce), each a sum of 19 pulled populations.  Two kernel
// organisations are provided:
//   two-pass  k_dens streams the pulled populations, one site per thread,
//             and writes rho[2][N]; k_collide marches a tile along z with
//             the densities staged in an LDS ring from that field, so the
//             pass pair moves 38 + 38 + 38 values per site plus the field;
//   fused     k_fused marches a 64 x TY tile along z, builds the density of
//             each new plane (tile + one-site ring) into a 4-slot LDS ring,
//             keeps the tile's own populations of the next plane in
//             registers, and collides the middle plane: HBM traffic stays at
//             38 + 38 values per site; the ring's extra loads hit L2.
// Particle coupling: the collision at a node touched by a particle needs the
// particle force, which needs the node's u_c and grad rho of the same step.
// The fused kernel therefore collides every site without it, stores u_c and
// the neighbour sums at the touched nodes (records), and k_fix re-collides
// only those nodes once the particle forces are spread.  In the two-pass
// organisation the density pass stores the raw momentum and the densities
// at the touched nodes, the coupling kernel forms the neighbour sums from
// the density field, and the collide pass applies the spread force in-line.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lbmd_internal.h"
#include "lbmd_site.h"
#include "lbmd_stencil.h"

namespace lbmd {

// ------------------------------------------------------------ init / io
// host-side value v of population i in storage form (deviations are taken
// in double and rounded once)
template <class S>
__device__ __forceinline__ S encode_pop(double v, int i, double rho0) {
  if constexpr (Storage<S>::deviation)
    return S{dev_encode(float(v - weight<double>(i) * rho0), (S*)nullptr)};
  else
    return S(v);
}

template <class S>
__global__ void k_init(S* __restrict__ f, const double* __restrict__ rho, int nx, int ny, int nz, double rho0) {
  const int64_t N = int64_t(nx) * ny * nz;
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const int x = int(s % nx), y = int((s / nx) % ny), z = int(s / (int64_t(nx) * ny));
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int64_t t = (int64_t(wrapi(z + D3Q19::cz[i], nz)) * ny + wrapi(y + D3Q19::cy[i], ny)) * nx +
                      wrapi(x + D3Q19::cx[i], nx);
    for (int c = 0; c < 2; ++c)
      f[(int64_t(c) * 19 + i) * N + s] = encode_pop<S>(weight<double>(i) * (rho ? rho[c * N + t] : 1.0), i, rho0);
  }
}

template <class S>
__global__ void k_import(S* __restrict__ f, const double* __restrict__ pop, int nx, int ny, int nz, double rho0) {
  const int64_t N = int64_t(nx) * ny * nz;
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const int x = int(s % nx), y = int((s / nx) % ny), z = int(s / (int64_t(nx) * ny));
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int64_t t = (int64_t(wrapi(z + D3Q19::cz[i], nz)) * ny + wrapi(y + D3Q19::cy[i], ny)) * nx +
                      wrapi(x + D3Q19::cx[i], nx);
    for (int c = 0; c < 2; ++c)
      f[(int64_t(c) * 19 + i) * N + s] = encode_pop<S>(pop[(int64_t(c) * 19 + i) * N + t], i, rho0);
  }
}

// density field rho[2][N] (two-pass kernel and exports)
template <class S>
__global__ void k_density(const S* __restrict__ src, arith_t<S>* __restrict__ rho, int nx, int ny, int nz,
                          arith_t<S> rho0) {
  using C = arith_t<S>;
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int z = blockIdx.z;
  if (x >= nx || y >= ny) return;
  const int64_t N = int64_t(nx) * ny * nz;
  C f[2][19];
  pull<S, C>(make_pops(src, N, rho0), x, y, z, nx, ny, nz, f);
  const int64_t s = (int64_t(z) * ny + y) * nx + x;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    C r = f[c][0];
#pragma unroll
    for (int i = 1; i < 19; ++i) r += f[c][i];
    rho[c * N + s] = r;
  }
}

// neighbour sums from a density field
template <class S, class C>
__device__ __forceinline__ void nsum_field(const S* __restrict__ rho, int x, int y, int z, int nx, int ny, int nz,
                                          int64_t N, C (&NA)[3], C (&NB)[3]) {
  C a[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    const int64_t t = (int64_t(wrapi(z + D3Q19::cz[i], nz)) * ny + wrapi(y + D3Q19::cy[i], ny)) * nx +
                      wrapi(x + D3Q19::cx[i], nx);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const C wr = weight<C>(i) * C(rho[c * N + t]);
      if (D3Q19::cx[i]) a[c][0] += D3Q19::cx[i] > 0 ? wr : -wr;
      if (D3Q19::cy[i]) a[c][1] += D3Q19::cy[i] > 0 ? wr : -wr;
      if (D3Q19::cz[i]) a[c][2] += D3Q19::cz[i] > 0 ? wr : -wr;
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    NA[q] = a[0][q];
    NB[q] = a[1][q];
  }
}

template <class C>
__device__ __forceinline__ void velocity_uc(const SiteOut<C>& o, const C (&NA)[3], const C (&NB)[3],
                                            const FluidConsts<C>& K, C (&uc)[3]) {
  const C rt = o.rho[0] + o.rho[1];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const C g0 = -o.rho[0] * (K.G[0][0] * NA[a] + K.G[0][1] * NB[a]);
    const C g1 = -o.rho[1] * (K.G[1][0] * NA[a] + K.G[1][1] * NB[a]);
    uc[a] = (o.j[a] + C(0.5) * (g0 + g1)) / rt;
  }
}

template <class C>
__device__ __forceinline__ SiteOut<C> moments_only(const C (&f)[2][19]) {
  SiteOut<C> o;
  o.j[0] = o.j[1] = o.j[2] = 0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    C r = f[c][0], jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      r += f[c][i];
      if (D3Q19::cx[i]) jx += D3Q19::cx[i] > 0 ? f[c][i] : -f[c][i];
      if (D3Q19::cy[i]) jy += D3Q19::cy[i] > 0 ? f[c][i] : -f[c][i];
      if (D3Q19::cz[i]) jz += D3Q19::cz[i] > 0 ? f[c][i] : -f[c][i];
    }
    o.rho[c] = r;
    o.j[0] += jx;
    o.j[1] += jy;
    o.j[2] += jz;
  }
  return o;
}

// export: rho [2][N], u_c [3][N], populations [2][19][N] as float64
template <class S>
__global__ void k_export(const S* __restrict__ src, const arith_t<S>* __restrict__ rho, double* __restrict__ out,
                         FluidConsts<arith_t<S>> K, uint32_t mask) {
  using C = arith_t<S>;
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int z = blockIdx.z;
  const int nx = K.nx, ny = K.ny, nz = K.nz;
  if (x >= nx || y >= ny) return;
  const int64_t N = K.N;
  const int64_t s = (int64_t(z) * ny + y) * nx + x;
  C f[2][19];
  pull<S, C>(make_pops(src, N, K.rho0), x, y, z, nx, ny, nz, f);
  double* o = out;
  if (mask & LBMD_RHO) {
    o[s] = double(rho[s]);
    o[N + s] = double(rho[N + s]);
    o += 2 * N;
  }
  if (mask & LBMD_U) {
    C NA[3], NB[3], uc[3];
    nsum_field<C, C>(rho, x, y, z, nx, ny, nz, N, NA, NB);
    SiteOut<C> m = moments_only<C>(f);
    velocity_uc<C>(m, NA, NB, K, uc);
    for (int a = 0; a < 3; ++a) o[a * N + s] = double(uc[a]);
    o += 3 * N;
  }
  if (mask & LBMD_POP)
    for (int c = 0; c < 2; ++c)
      for (int i = 0; i < 19; ++i) o[(int64_t(c) * 19 + i) * N + s] = double(f[c][i]);
}

__global__ void k_zero_words(uint32_t* __restrict__ w, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) w[i] = 0u;
}

// ------------------------------------------------------------ fused path
// One pass per step: density ring from the pulled populations, collision of
// every site without particle force, records at touched nodes; k_fix then
// re-collides the touched nodes.  Best when few nodes are touched.
template <class S, int TY, int FORCING, bool NOISE, bool HOLD>
__device__ __forceinline__ void fused_tile(const S* __restrict__ src_, S* __restrict__ dst_, FluidConsts<arith_t<S>> K,
                                           int tz, int tiles_x, int xcd, const uint32_t* __restrict__ mask,
                                           arith_t<S>* __restrict__ rec, double* __restrict__ red, uint32_t* status,
                                           long long* bad, int block, int nblk) {
  using C = arith_t<S>;
  load_step(K);
  __shared__ C ring[4][2][TY + 2][66];
  const int nx = K.nx, ny = K.ny, nz = K.nz;
  const int64_t N = K.N;
  const int64_t plane = int64_t(nx) * ny;
  const Pops<S> src = make_pops(src_, N, K.rho0), dst = make_pops<S>(dst_, N, K.rho0, K.srkey);
  const Tile<TY> T(nx, ny, nz, tz, tiles_x, xcd, block, nblk);
  const int lane = T.lane, wv = T.wv, x = T.x, y = T.y;

  C cur[2][19], nxt[2][19];
  double acc[5] = {0, 0, 0, 0, 0};

  // density of the tile's own sites of plane zp -> ring; with HOLD the
  // populations stay in registers for the collision one plane later,
  // otherwise they are read again then (from cache)
  auto load_interior = [&](int zp_raw, int slot) {
    const int zz = wrapi(zp_raw, nz);
    if (T.inside) {
      pull<S, C>(src, x, y, zz, nx, ny, nz, nxt);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        C r = nxt[c][0];
#pragma unroll
        for (int i = 1; i < 19; ++i) r += nxt[c][i];
        ring[slot][c][wv + 1][lane + 1] = r;
      }
    }
  };
  auto load_border = [&](int zp_raw, int slot) {
    const int zz = wrapi(zp_raw, nz);
    T.for_border([&](int hr, int hc) {
      C hf[2][19];
      pull<S, C>(src, wrapi(T.x0 - 1 + hc, nx), wrapi(T.y0 - 1 + hr, ny), zz, nx, ny, nz, hf);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        C r = hf[c][0];
#pragma unroll
        for (int i = 1; i < 19; ++i) r += hf[c][i];
        ring[slot][c][hr][hc] = r;
      }
    });
  };

  // prologue: planes z0-1 and z0 complete, border of z0+1; plane q lives in
  // ring slot (q - z0 + 1) & 3
  const int z0 = T.z0, z1 = T.z1;
  load_interior(z0 - 1, 0);
  load_border(z0 - 1, 0);
  load_interior(z0, 1);
  load_border(z0, 1);
  load_border(z0 + 1, 2);
  if (HOLD) {
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i = 0; i < 19; ++i) cur[c][i] = nxt[c][i];
  }
  // iteration z: interior of z+1, barrier, collide z, border of z+2 (into
  // the slot last read in iteration z-1, which this barrier separates)
  for (int z = z0; z < z1; ++z) {
    const int k = z - z0;
    load_interior(z + 1, (k + 2) & 3);
    __syncthreads();
    if (T.inside) {
      C NA[3], NB[3];
      nsum_ring<C, TY>(ring, k & 3, (k + 1) & 3, (k + 2) & 3, wv, lane, NA, NB);
      const int64_t s = z * plane + int64_t(y) * nx + x;
      const C gp[3] = {0, 0, 0}, gu[6] = {0, 0, 0, 0, 0, 0};
      if (!HOLD) pull<S, C>(src, x, y, z, nx, ny, nz, cur);
      const Macro<C> m = macro<C, FORCING>(cur, NA, NB, gp, K, gu, false);
      if (mask && ((mask[s >> 5] >> (s & 31)) & 1u)) {
        C uc[3];
        coupling_velocity<C, FORCING>(m, uc);
        C* r = rec + s * REC;
        for (int a = 0; a < 3; ++a) {
          r[a] = NA[a];
          r[3 + a] = NB[a];
          r[6 + a] = uc[a];
        }
        r[9] = m.rho[0];
        r[10] = m.rho[1];
      }
      SiteOut<C> o;
      o.rho[0] = m.rho[0];
      o.rho[1] = m.rho[1];
      o.j[0] = m.j[0];
      o.j[1] = m.j[1];
      o.j[2] = m.j[2];
      if (!moments_ok(o)) flag_unstable(status, bad, 1u, K.step);
      relax_site<C, FORCING, NOISE>(cur, m, K, uint32_t(s));
      store<S, C>(dst, uint32_t(s), cur, K.nt);
      acc[0] += o.rho[0];
      acc[1] += o.rho[1];
      acc[2] += o.j[0];
      acc[3] += o.j[1];
      acc[4] += o.j[2];
    }
    if (z + 2 <= z1) load_border(z + 2, (k + 3) & 3);
    if (HOLD) {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i = 0; i < 19; ++i) cur[c][i] = nxt[c][i];
    }
  }
  block_sum5<TY>(acc, red + 5 * int64_t(T.bid));
}

template <class S, int TY, int FORCING, bool NOISE, bool HOLD>
__global__ __launch_bounds__(64 * TY) void k_fused(const S* __restrict__ src_, S* __restrict__ dst_,
                                                    FluidConsts<arith_t<S>> K, int tz, int tiles_x, int xcd,
                                                    const uint32_t* __restrict__ mask, arith_t<S>* __restrict__ rec,
                                                    double* __restrict__ red, uint32_t* status, long long* bad) {
  fused_tile<S, TY, FORCING, NOISE, HOLD>(src_, dst_, K, tz, tiles_x, xcd, mask, rec, red, status, bad, blockIdx.x,
                                          gridDim.x);
}

// re-collide the touched nodes with the spread particle force; clears the
// node force and the mask as it goes
template <class S, int FORCING, bool NOISE>
__device__ __forceinline__ void fix_node(const S* __restrict__ src, S* __restrict__ dst, FluidConsts<arith_t<S>> K,
                                         const int32_t* __restrict__ list, const int32_t* __restrict__ nlist,
                                         const arith_t<S>* __restrict__ rec, arith_t<S>* __restrict__ gP,
                                         arith_t<S>* __restrict__ gS, uint32_t* __restrict__ mask, int64_t t) {
  using C = arith_t<S>;
  load_step(K);
  if (t >= *nlist) return;
  const int64_t N = K.N;
  const int64_t s = list[t];
  const int nx = K.nx, ny = K.ny, nz = K.nz;
  const int x = int(s % nx), y = int((s / nx) % ny), z = int(s / (int64_t(nx) * ny));
  C f[2][19], NA[3], NB[3], gp[3];
  pull<S, C>(make_pops(src, N, K.rho0), x, y, z, nx, ny, nz, f);
  for (int a = 0; a < 3; ++a) {
    NA[a] = rec[s * REC + a];
    NB[a] = rec[s * REC + 3 + a];
    gp[a] = gP[s * GPS + a];
    gP[s * GPS + a] = C(0);
  }
  mask[s >> 5] = 0u;
  C gu[6] = {0, 0, 0, 0, 0, 0};
  if (gS)
    for (int q = 0; q < 6; ++q) {
      gu[q] = gS[s * GSS + q];
      gS[s * GSS + q] = C(0);
    }
  collide<C, FORCING, NOISE>(f, NA, NB, gp, K, uint32_t(s), gu, gS != nullptr);
  store<S, C>(make_pops<S>(dst, N, K.rho0, K.srkey), uint32_t(s), f);
}

template <class S, int FORCING, bool NOISE>
__global__ __launch_bounds__(256) void k_fix(const S* __restrict__ src, S* __restrict__ dst, FluidConsts<arith_t<S>> K,
                                             const int32_t* __restrict__ list, const int32_t* __restrict__ nlist,
                                             const arith_t<S>* __restrict__ rec, arith_t<S>* __restrict__ gP,
                                             arith_t<S>* __restrict__ gS, uint32_t* __restrict__ mask) {
  fix_node<S, FORCING, NOISE>(src, dst, K, list, nlist, rec, gP, gS, mask,
                              int64_t(blockIdx.x) * blockDim.x + threadIdx.x);
}

// ------------------------------------------------------------ split path
// Pass P, flat: one site per thread per pass over the lattice (a grid of at
// most DENS_GRID blocks strides through it, so the per-block FP64 partials
// stay few for the final reduction), no tiling.  The density field, the
// conservation sums and the status; at the nodes particles touch, the raw
// momentum and the two densities go to the node record (the coupling kernel
// forms the neighbour sums there from the density field).  A plain
// streaming read of the 38 pulled populations per site.  512 blocks of 512
// threads (half the chip's wave slots) still stream at the full rate and
// leave the other half to the pair forces beside the pass.
constexpr int DENS_BLOCK = 512, DENS_GRID = 512;
template <class S>
__global__ __launch_bounds__(DENS_BLOCK) void k_dens(const S* __restrict__ src_, arith_t<S>* __restrict__ rho,
                                                     FluidConsts<arith_t<S>> K, const uint32_t* __restrict__ mask,
                                                     arith_t<S>* __restrict__ rec, double* __restrict__ red,
                                                     uint32_t* status, long long* bad) {
  using C = arith_t<S>;
  load_step(K);
  const int nx = K.nx, ny = K.ny, nz = K.nz;
  const int64_t N = K.N;
  const Pops<S> src = make_pops(src_, N, K.rho0);
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t s = int64_t(blockIdx.x) * DENS_BLOCK + threadIdx.x; s < N; s += int64_t(gridDim.x) * DENS_BLOCK) {
    const int x = int(s % nx), y = int((s / nx) % ny), z = int(s / (int64_t(nx) * ny));
    C f[2][19];
    pull<S, C>(src, x, y, z, nx, ny, nz, f);
    SiteOut<C> o;
    C jt[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      C jj[3];
      moments_pairs<C>(f[c], o.rho[c], jj);
#pragma unroll
      for (int a = 0; a < 3; ++a) jt[a] += jj[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) o.j[a] = jt[a];
    rho[s] = o.rho[0];
    rho[N + s] = o.rho[1];
    if (mask && ((mask[s >> 5] >> (s & 31)) & 1u)) {
      C* r = rec + s * REC;
      r[6] = o.j[0];
      r[7] = o.j[1];
      r[8] = o.j[2];
      r[9] = o.rho[0];
      r[10] = o.rho[1];
    }
    if (!moments_ok(o)) flag_unstable(status, bad, 1u, K.step);
    acc[0] += o.rho[0];
    acc[1] += o.rho[1];
    acc[2] += o.j[0];
    acc[3] += o.j[1];
    acc[4] += o.j[2];
  }
  block_sum5<DENS_BLOCK / 64>(acc, red + 5 * int64_t(blockIdx.x));
}

// Pass C: collision and streaming of every site, the particle force applied
// where a particle touches; the density ring is filled from the density
// field written by the density pass (two values per site instead of 38).
template <class S, int TY, int FORCING, bool NOISE, bool MRT>
__global__ __launch_bounds__(64 * TY) void k_collide(const S* __restrict__ src_, S* __restrict__ dst_,
                                                      const arith_t<S>* __restrict__ rho, FluidConsts<arith_t<S>> K,
                                                      int tz, int tiles_x, int xcd, const uint32_t* __restrict__ mask,
                                                      arith_t<S>* __restrict__ gP, arith_t<S>* __restrict__ gS) {
  using C = arith_t<S>;
  load_step(K);
  __shared__ C ring[4][2][TY + 2][66];
  const int nx = K.nx, ny = K.ny, nz = K.nz;
  const int64_t N = K.N;
  const int64_t plane = int64_t(nx) * ny;
  const Pops<S> src = make_pops(src_, N, K.rho0), dst = make_pops<S>(dst_, N, K.rho0, K.srkey);
  const Tile<TY> T(nx, ny, nz, tz, tiles_x, xcd, blockIdx.x, gridDim.x);
  const int lane = T.lane, wv = T.wv, x = T.x, y = T.y;

  auto load_interior = [&](int zp_raw, int slot) {
    const int64_t zz = wrapi(zp_raw, nz);
    if (T.inside) {
      const int64_t s = zz * plane + int64_t(y) * nx + x;
      ring[slot][0][wv + 1][lane + 1] = rho[s];
      ring[slot][1][wv + 1][lane + 1] = rho[N + s];
    }
  };
  auto load_border = [&](int zp_raw, int slot) {
    const int64_t zz = wrapi(zp_raw, nz);
    T.for_border([&](int hr, int hc) {
      const int64_t s = zz * plane + int64_t(wrapi(T.y0 - 1 + hr, ny)) * nx + wrapi(T.x0 - 1 + hc, nx);
      ring[slot][0][hr][hc] = rho[s];
      ring[slot][1][hr][hc] = rho[N + s];
    });
  };

  const int z0 = T.z0, z1 = T.z1;
  load_interior(z0 - 1, 0);
  load_border(z0 - 1, 0);
  load_interior(z0, 1);
  load_border(z0, 1);
  load_border(z0 + 1, 2);
  for (int z = z0; z < z1; ++z) {
    const int k = z - z0;
    load_interior(z + 1, (k + 2) & 3);
    __syncthreads();
    if (T.inside) {
      C NA[3], NB[3], f[2][19];
      const int64_t s = z * plane + int64_t(y) * nx + x;
      pull<S, C>(src, x, y, z, nx, ny, nz, f);
      nsum_ring<C, TY>(ring, k & 3, (k + 1) & 3, (k + 2) & 3, wv, lane, NA, NB);
      C gp[3] = {0, 0, 0}, gu[6];
      bool fs = false;
      if (mask && ((mask[s >> 5] >> (s & 31)) & 1u)) {
        for (int a = 0; a < 3; ++a) {
          gp[a] = gP[s * GPS + a];
          gP[s * GPS + a] = C(0);
        }
        if (gS) {
          fs = true;
          for (int q = 0; q < 6; ++q) {
            gu[q] = gS[s * GSS + q];
            gS[s * GSS + q] = C(0);
          }
        }
      }
      const Macro<C> m = macro<C, FORCING>(f, NA, NB, gp, K, gu, fs);
      relax_site<C, FORCING, NOISE, MRT>(f, m, K, uint32_t(s));
      store<S, C, NOISE || Storage<S>::deviation>(dst, uint32_t(s), f, K.nt);
    }
    if (z + 2 <= z1) load_border(z + 2, (k + 3) & 3);
  }
}

// The collide-stream pass's memory traffic without its arithmetic: every
// site's 38 pulled population words are read (src[i][s - c_i]) and written
// unchanged to dst[i][s] (non-temporal), one site per thread.  Timing it
// gives the bandwidth this access pattern reaches on the device, the
// practical ceiling of the collide-stream kernels.
template <class S>
__global__ __launch_bounds__(256) void k_pull_copy(const S* __restrict__ src_, S* __restrict__ dst_, int nx, int ny,
                                                   int nz, int64_t N) {
  const int64_t s = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (s >= N) return;
  const int x = int(s % nx), y = int((s / nx) % ny), z = int(s / (int64_t(nx) * ny));
  const Pops<S> src = make_pops(src_, N), dst = make_pops(dst_, N);
  const uint32_t vs = uint32_t(s) * uint32_t(sizeof(S));
  for_pulled<S>(x, y, z, nx, ny, nz, [&](int i, uint32_t vo) {
    const int so = int(uint32_t(i) * src.pstride);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if constexpr (sizeof(S) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_amdgcn_raw_buffer_load_b64(src.r[c], int(vo), so, 0), dst.r[c],
                                              int(vs), so, 2);
      else if constexpr (sizeof(S) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_amdgcn_raw_buffer_load_b32(src.r[c], int(vo), so, 0), dst.r[c],
                                              int(vs), so, 2);
      else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_amdgcn_raw_buffer_load_b16(src.r[c], int(vo), so, 0), dst.r[c],
                                              int(vs), so, 2);
    }
  });
}

// final reductions: fluid partials [nf][5], particle partials [np][3] -> out[8]
__device__ __forceinline__ void finalize_sums(const double* __restrict__ rf, int64_t nf, const double* __restrict__ rp,
                                              int64_t npb, double* __restrict__ out, int32_t* nflag, int64_t* step) {
  // one pass over the partials (5 fluid and 3 particle sums per thread),
  // wave sums by shuffles, then the 4 waves' sums through LDS
  __shared__ double sh[8][4];
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < nf; b += 256)
#pragma unroll
    for (int q = 0; q < 5; ++q) s[q] += rf[5 * b + q];
  for (int64_t b = threadIdx.x; b < npb; b += 256)
#pragma unroll
    for (int q = 0; q < 3; ++q) s[5 + q] += rp[3 * b + q];
#pragma unroll
  for (int q = 0; q < 8; ++q) s[q] = wave_sum(s[q]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 8; ++q) sh[q][threadIdx.x >> 6] = s[q];
  __syncthreads();
  if (threadIdx.x < 8) out[threadIdx.x] = (sh[threadIdx.x][0] + sh[threadIdx.x][1]) + (sh[threadIdx.x][2] + sh[threadIdx.x][3]);
  if (threadIdx.x == 0) {
    *nflag = 0;
    *step += 1;
  }
}
__global__ void k_finalize(const double* __restrict__ rf, int64_t nf, const double* __restrict__ rp, int64_t npb,
                           double* __restrict__ out, int32_t* nflag, int64_t* step) {
  finalize_sums(rf, nf, rp, npb, out, nflag, step);
}

// ------------------------------------------------------------ launchers
static dim3 plane_grid(const lbmd_ctx* h) {
  return dim3((h->p.nx + 63) / 64, (h->p.ny + 3) / 4, h->p.nz);
}

template <class S>
static hipError_t init_t(lbmd_ctx* h, const double* rho_dev) {
  const int64_t N = h->N;
  hipLaunchKernelGGL(k_init<S>, dim3((N + 255) / 256), dim3(256), 0, h->stream, (S*)h->f[h->cur], rho_dev, h->p.nx,
                     h->p.ny, h->p.nz, h->p.rho0);
  return hipGetLastError();
}
// calls FN<storage type>(args...) for the handle's precision
#define LBMD_BY_STORAGE(FN, ...)                                        \
  switch (h->p.precision) {                                              \
    case LBMD_FP64: return FN<double>(__VA_ARGS__);                      \
    case LBMD_FP16DEV: return FN<half_dev>(__VA_ARGS__);                 \
    case LBMD_BF16DEV: return FN<bf16_dev>(__VA_ARGS__);                 \
    default: return FN<float>(__VA_ARGS__);                              \
  }
hipError_t fluid_init(lbmd_ctx* h, const double* rho_dev) { LBMD_BY_STORAGE(init_t, h, rho_dev) }

template <class S>
static hipError_t import_t(lbmd_ctx* h, const double* pop) {
  const int64_t N = h->N;
  hipLaunchKernelGGL(k_import<S>, dim3((N + 255) / 256), dim3(256), 0, h->stream, (S*)h->f[h->cur], pop, h->p.nx,
                     h->p.ny, h->p.nz, h->p.rho0);
  return hipGetLastError();
}
hipError_t fluid_import(lbmd_ctx* h, const double* pop) { LBMD_BY_STORAGE(import_t, h, pop) }

template <class S>
static hipError_t export_t(lbmd_ctx* h, uint32_t mask, double* out, void* field) {
  using C = arith_t<S>;
  const S* src = (const S*)h->f[h->cur];
  const FluidConsts<C> K = consts<S>(h);
  hipLaunchKernelGGL(k_density<S>, plane_grid(h), dim3(256), 0, h->stream, src, (C*)field, h->p.nx, h->p.ny,
                     h->p.nz, K.rho0);
  hipLaunchKernelGGL(k_export<S>, plane_grid(h), dim3(256), 0, h->stream, src, (const C*)field, out, K, mask);
  return hipGetLastError();
}
hipError_t fluid_export(lbmd_ctx* h, uint32_t mask, double* out, void* field) {
  LBMD_BY_STORAGE(export_t, h, mask, out, field)
}

template <class S>
static hipError_t pull_copy_t(lbmd_ctx* h) {
  const int64_t N = h->N;
  hipLaunchKernelGGL(k_pull_copy<S>, dim3((N + 255) / 256), dim3(256), 0, h->stream, (const S*)h->f[h->cur],
                     (S*)h->f[1 - h->cur], h->p.nx, h->p.ny, h->p.nz, N);
  return hipGetLastError();
}
hipError_t fluid_pull_copy(lbmd_ctx* h) { LBMD_BY_STORAGE(pull_copy_t, h) }

// organisation actually used this step
static int organisation(const lbmd_ctx* h) {
  // with thermal noise the push kernel's in-block gather comes on top of
  // the per-site normals; its collide pass then runs longer than the
  // density pass it saves (bead-spring chains at 256^3: 2.39 against
  // 2.26 ms per step), so fluctuating steps use the two-pass organisation.
  // On 16-bit storage the five 4-byte moments per site the push pass writes
  // and reads weigh more against the 76 two-byte populations than the
  // density pass it saves (256^3 with 160k particles: 13,600 against 11,500
  // MLUPS binary16, 14,000 against 11,500 bfloat16), so those use it too.
  const bool half = h->p.precision == LBMD_FP16DEV || h->p.precision == LBMD_BF16DEV;
  const int many = h->p.kT > 0.0 || half ? LBMD_KERNEL_TWOPASS : LBMD_KERNEL_PUSH;
  // the MRT collision is built into the two-pass and push kernels only
  if (h->mrt)
    return h->p.kernel == LBMD_KERNEL_TWOPASS || h->p.kernel == LBMD_KERNEL_PUSH ? h->p.kernel : many;
  if (h->p.kernel != LBMD_KERNEL_AUTO) return h->p.kernel;
  // the fused pass re-collides every touched node with scattered accesses
  // (about 76 per node); the push pass writes and reads a five-value moment
  // field per site.  At 256^3 FP32 the fused step is faster without
  // particles (1.285 against 1.329 ms) and slower from 2,000 particles on
  // (1.398 against 1.373 ms; 10,000: 1.491 against 1.393): break-even near
  // one touched node per 2,048 sites.
  return (h->np == 0 || 8 * h->np * 2048 < h->N) ? LBMD_KERNEL_FUSED : many;
}

struct Launch {
  int tiles_x, tz, ty;
  int64_t nblk;
};
// Tiling actually launched: the caller's (lbmd_set_tiling or
// lbmd_autotune), else defaults from measurements on MI355X: the fused
// kernel with 4 rows and its populations held in registers, the two-pass
// kernels with 8 rows (16 on 16-bit storage or with noise) in XCD order; the z chunk is
// chosen so that a launch has about 256 blocks (16, 128 and 64 planes at
// 256^3, the measured optima), within [2, 16] planes for the fused kernel
// and [4, 128] for the two-pass kernels.  Rows never exceed the lattice
// height.
static int pow2_floor(int64_t v) {
  int p = 1;
  while (int64_t(p) * 2 <= v) p *= 2;
  return p;
}
static Launch tiles(lbmd_ctx* h) {
  const int org = organisation_of(h);
  if (!h->tiling_set) {
    const bool fused = org == LBMD_KERNEL_FUSED;
    // rows: 16 for the two-pass kernels on 16-bit storage or with thermal
    // noise, 8 otherwise
    const bool wide = h->p.precision == LBMD_FP16DEV || h->p.precision == LBMD_BF16DEV || h->p.kT > 0.0;
    const int want = fused ? 4 : (wide ? 16 : 8);
    int ty = 2;
    while (ty < want && ty * 2 <= h->p.ny) ty *= 2;
    const int64_t cols = int64_t((h->p.nx + 63) / 64) * ((h->p.ny + ty - 1) / ty);
    const int tz = pow2_floor(std::max<int64_t>(1, cols * h->p.nz / 256));
    h->tile_y = ty;
    h->tile_z = fused ? std::min(16, std::max(2, tz)) : std::min(128, std::max(4, tz));
    h->hold = 1;
    h->xcd = fused ? 0 : 1;
  }
  Launch L;
  L.tiles_x = (h->p.nx + 63) / 64;
  L.ty = h->tile_y;
  if (org == LBMD_KERNEL_PUSH && L.ty > push_rows_max(h)) L.ty = push_rows_max(h);
  const int tiles_y = (h->p.ny + L.ty - 1) / L.ty;
  L.tz = std::max(1, std::min(h->tile_z, h->p.nz));
  L.nblk = int64_t(L.tiles_x) * tiles_y * ((h->p.nz + L.tz - 1) / L.tz);
  return L;
}

#define LBMD_BY_TY(TY, CALL) \
  switch (TY) {              \
    case 2: {                \
      constexpr int TYV = 2; \
      CALL;                  \
    } break;                 \
    case 4: {                \
      constexpr int TYV = 4; \
      CALL;                  \
    } break;                 \
    case 16: {               \
      constexpr int TYV = 16; \
      CALL;                  \
    } break;                 \
    default: {               \
      constexpr int TYV = 8; \
      CALL;                  \
    } break;                 \
  }

template <class S, int FORCING, bool NOISE>
static hipError_t pass_a_t(lbmd_ctx* h) {
  using C = arith_t<S>;
  const S* src = (const S*)h->f[h->cur];
  S* dst = (S*)h->f[1 - h->cur];
  const FluidConsts<C> K = consts<S>(h);
  const Launch L = tiles(h);
  h->red_fluid_used = L.nblk;
  const uint32_t* mask = h->np > 0 ? h->mask : nullptr;
  if (organisation(h) == LBMD_KERNEL_FUSED) {
    if (hipError_t e = prof_begin(h)) return e;
    if (h->hold) {
      LBMD_BY_TY(L.ty, hipLaunchKernelGGL((k_fused<S, TYV, FORCING, NOISE, true>), dim3(L.nblk), dim3(64 * TYV), 0,
                                          h->stream, src, dst, K, L.tz, L.tiles_x, h->xcd, mask, (C*)h->rec, h->red_fluid,
                                          h->status, h->bad_step));
    } else {
      LBMD_BY_TY(L.ty, hipLaunchKernelGGL((k_fused<S, TYV, FORCING, NOISE, false>), dim3(L.nblk), dim3(64 * TYV), 0,
                                          h->stream, src, dst, K, L.tz, L.tiles_x, h->xcd, mask, (C*)h->rec, h->red_fluid,
                                          h->status, h->bad_step));
    }
    if (hipError_t e = prof_end(h)) return e;
  } else if (organisation(h) == LBMD_KERNEL_TWOPASS) {
    const int64_t nb = std::min<int64_t>((h->N + DENS_BLOCK - 1) / DENS_BLOCK, DENS_GRID);
    h->red_fluid_used = nb;
    hipLaunchKernelGGL(k_dens<S>, dim3(nb), dim3(DENS_BLOCK), 0, h->stream, src, (C*)h->rho, K, mask, (C*)h->rec,
                       h->red_fluid, h->status, h->bad_step);
  }
  return hipGetLastError();
}

template <class S, int FORCING, bool NOISE>
static hipError_t pass_b_t(lbmd_ctx* h) {
  using C = arith_t<S>;
  const S* src = (const S*)h->f[h->cur];
  S* dst = (S*)h->f[1 - h->cur];
  const FluidConsts<C> K = consts<S>(h);
  if (organisation(h) == LBMD_KERNEL_PUSH) {
    const Launch L = tiles(h);
    h->red_fluid_used = L.nblk;
    if (hipError_t e = prof_begin(h)) return e;
    if (hipError_t e = push_pass(h, PushLaunch{L.ty, L.tz, L.tiles_x, h->xcd, L.nblk})) return e;
    if (hipError_t e = prof_end(h)) return e;
    if (h->np > 0) {
      const int64_t words = (h->N + 31) / 32;
      hipLaunchKernelGGL(k_zero_words, dim3((words + 255) / 256), dim3(256), 0, h->stream, h->mask, words);
    }
  } else if (organisation(h) == LBMD_KERNEL_FUSED) {
    if (h->np > 0)
      hipLaunchKernelGGL((k_fix<S, FORCING, NOISE>), dim3((h->flag_cap + 255) / 256), dim3(256), 0, h->stream, src,
                         dst, K, h->flag_list, h->nflag, (const C*)h->rec, (C*)h->gP, (C*)h->gS, h->mask);
  } else {
    const Launch L = tiles(h);
    const uint32_t* mask = h->np > 0 ? h->mask : nullptr;
    if (hipError_t e = prof_begin(h)) return e;
    if (FORCING == LBMD_FORCE_PAPER && h->mrt) {
      LBMD_BY_TY(L.ty, hipLaunchKernelGGL((k_collide<S, TYV, LBMD_FORCE_PAPER, NOISE, true>), dim3(L.nblk),
                                          dim3(64 * TYV), 0, h->stream, src, dst, (const C*)h->rho, K, L.tz, L.tiles_x,
                                          h->xcd, mask, (C*)h->gP, (C*)h->gS));
    } else {
      LBMD_BY_TY(L.ty, hipLaunchKernelGGL((k_collide<S, TYV, FORCING, NOISE, false>), dim3(L.nblk), dim3(64 * TYV), 0,
                                          h->stream, src, dst, (const C*)h->rho, K, L.tz, L.tiles_x, h->xcd, mask,
                                          (C*)h->gP, (C*)h->gS));
    }
    if (hipError_t e = prof_end(h)) return e;
    if (h->np > 0) {
      const int64_t words = (h->N + 31) / 32;
      hipLaunchKernelGGL(k_zero_words, dim3((words + 255) / 256), dim3(256), 0, h->stream, h->mask, words);
    }
  }
  return hipGetLastError();
}

#define LBMD_DISPATCH_S(NAME, S)                                                         \
  if (h->p.forcing == LBMD_FORCE_SHIFT) return NAME##_t<S, LBMD_FORCE_SHIFT, false>(h); \
  return noise ? NAME##_t<S, LBMD_FORCE_PAPER, true>(h) : NAME##_t<S, LBMD_FORCE_PAPER, false>(h);
#define LBMD_DISPATCH(NAME)                                     \
  hipError_t fluid_##NAME(lbmd_ctx* h) {                        \
    const bool noise = h->p.kT > 0.0;                           \
    switch (h->p.precision) {                                   \
      case LBMD_FP64: { LBMD_DISPATCH_S(NAME, double) }         \
      case LBMD_FP16DEV: { LBMD_DISPATCH_S(NAME, half_dev) }    \
      case LBMD_BF16DEV: { LBMD_DISPATCH_S(NAME, bf16_dev) }    \
      default: { LBMD_DISPATCH_S(NAME, float) }                 \
    }                                                           \
  }
LBMD_DISPATCH(pass_a)
LBMD_DISPATCH(pass_b)
#undef LBMD_DISPATCH
#undef LBMD_DISPATCH_S
#undef LBMD_BY_STORAGE

hipError_t finalize_step(lbmd_ctx* h) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, h->stream, h->red_fluid, h->red_fluid_used, h->red_part,
                     h->red_part_used, h->red_out, h->nflag, h->step_dev);
  return hipGetLastError();
}

int organisation_of(const lbmd_ctx* h) { return organisation(h); }

// ------------------------------------------------------------ batches
// Index of the job whose range [begin, next begin) holds unit u (jobs in
// order of increasing begin; a job with no units shares its begin with the
// next one, and the last such job is the one that owns u).
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

// Fluid pass of every job: each block walks lattice tiles of the flattened
// tile range (the global tile queue), one z-march per tile.
template <bool NOISE>
__global__ __launch_bounds__(64 * BATCH_TY) void k_fused_batch(const BatchJob* __restrict__ jobs,
                                                                const BatchHeader* __restrict__ hdr) {
  __shared__ int act;
  const int nj = hdr->njobs;
  const int64_t total = hdr->ntiles;
  for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
    const BatchJob& J = jobs[batch_job_of<&BatchJob::tile_begin>(jobs, nj, u)];
    if (threadIdx.x == 0) act = batch_active(J) ? 1 : 0;  // the status word may change meanwhile
    __syncthreads();
    const bool a = act != 0;
    __syncthreads();
    if (a) {
      const int par = int(*J.step & 1);
      fused_tile<float, BATCH_TY, LBMD_FORCE_PAPER, NOISE, true>(J.f[par], const_cast<float*>(J.f[1 - par]), J.K,
                                                                 J.tz, J.tiles_x, 0, J.mask, J.rec, J.red_fluid,
                                                                 J.status, J.bad, int(u - J.tile_begin), J.nblk);
    }
    __syncthreads();  // the LDS ring is reused by the next tile
  }
}

// Re-collision of the touched nodes of every job.
template <bool NOISE>
__global__ __launch_bounds__(256) void k_fix_batch(const BatchJob* __restrict__ jobs,
                                                   const BatchHeader* __restrict__ hdr) {
  const int nj = hdr->njobs;
  const int64_t total = hdr->nfixblk;
  for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
    const BatchJob& J = jobs[batch_job_of<&BatchJob::fix_begin>(jobs, nj, u)];
    if (!batch_active(J)) continue;
    const int par = int(*J.step & 1);
    fix_node<float, LBMD_FORCE_PAPER, NOISE>(J.f[par], const_cast<float*>(J.f[1 - par]), J.K, J.flag_list, J.nflag,
                                             J.rec, J.gP, J.gS, J.mask, (u - J.fix_begin) * 256 + threadIdx.x);
  }
}

// Conservation sums and step counter of every job (one block per job slot).
__global__ void k_finalize_batch(const BatchJob* __restrict__ jobs, const BatchHeader* __restrict__ hdr) {
  __shared__ int act;
  const int j = blockIdx.x;
  if (j >= hdr->njobs) return;
  const BatchJob& J = jobs[j];
  if (threadIdx.x == 0) act = batch_active(J) ? 1 : 0;
  __syncthreads();
  if (!act) return;
  finalize_sums(J.red_fluid, J.nblk, J.red_part, J.npblk, J.red_out, J.nflag, J.step);
}

constexpr int BATCH_FIX_GRID = 1024;

hipError_t batch_fluid_pass(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr, bool noise) {
  if (noise)
    hipLaunchKernelGGL(k_fused_batch<true>, dim3(BATCH_FLUID_GRID), dim3(64 * BATCH_TY), 0, st, jobs, hdr);
  else
    hipLaunchKernelGGL(k_fused_batch<false>, dim3(BATCH_FLUID_GRID), dim3(64 * BATCH_TY), 0, st, jobs, hdr);
  return hipGetLastError();
}
hipError_t batch_fluid_fix(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr, bool noise) {
  if (noise)
    hipLaunchKernelGGL(k_fix_batch<true>, dim3(BATCH_FIX_GRID), dim3(256), 0, st, jobs, hdr);
  else
    hipLaunchKernelGGL(k_fix_batch<false>, dim3(BATCH_FIX_GRID), dim3(256), 0, st, jobs, hdr);
  return hipGetLastError();
}
hipError_t batch_finalize(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr, int max_jobs) {
  hipLaunchKernelGGL(k_finalize_batch, dim3(max_jobs), dim3(256), 0, st, jobs, hdr);
  return hipGetLastError();
}

// (step, status) of every job of the table, for the host's poll
__global__ void k_gather_batch(const BatchJob* __restrict__ jobs, const BatchHeader* __restrict__ hdr,
                               int64_t* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= hdr->njobs) return;
  out[2 * j] = *jobs[j].step;
  out[2 * j + 1] = int64_t(*jobs[j].status);
}
hipError_t batch_gather(hipStream_t st, const BatchJob* jobs, const BatchHeader* hdr, int max_jobs, int64_t* out) {
  hipLaunchKernelGGL(k_gather_batch, dim3((max_jobs + 63) / 64), dim3(64), 0, st, jobs, hdr, out);
  return hipGetLastError();
}

// The job's constants, buffers and fused tiling: 4 rows per tile and z
// chunks of at most tz planes (the batch picks tz for the whole table).
void batch_fill_fluid(const lbmd_ctx* h, BatchJob& J, int tz) {
  J.K = consts<float>(h);
  J.step = h->step_dev;
  J.f[0] = (const float*)h->f[0];
  J.f[1] = (const float*)h->f[1];
  J.mask = h->np > 0 ? h->mask : nullptr;
  J.rec = (float*)h->rec;
  J.gP = (float*)h->gP;
  J.gS = (float*)h->gS;
  J.red_fluid = h->red_fluid;
  J.red_out = h->red_out;
  J.status = h->status;
  J.bad = h->bad_step;
  J.nflag = h->nflag;
  J.flag_list = h->flag_list;
  J.tiles_x = (h->p.nx + 63) / 64;
  const int64_t tiles_y = (h->p.ny + BATCH_TY - 1) / BATCH_TY;
  J.tz = std::max(1, std::min(tz, h->p.nz));
  J.nblk = int(J.tiles_x * tiles_y * ((h->p.nz + J.tz - 1) / J.tz));
  J.nfixblk = h->np > 0 ? (h->flag_cap + 255) / 256 : 0;
}

}  // namespace lbmd
