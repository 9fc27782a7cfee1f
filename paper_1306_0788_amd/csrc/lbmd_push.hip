// Push organisation of the particle-laden fluid step (gfx950, wave64).
//
// The Shan-Chen force of step n needs every site's neighbour densities of
// step n, and the particle coupling needs the raw momentum and densities at
// the particles' nodes, before any site is collided.  Instead of a separate
// pass that re-reads the 38 populations of every site to form them, the
// collide-stream pass of step n-1 builds them: the post-collision value
// f*_zeta,i(r) it writes is exactly the population that site r + c_i pulls
// at step n (Eq. LBMIX), so the pass adds it to the next step's moments of
// r + c_i,
//   rho_zeta(s, n) = sum_i f*_zeta,i(s - c_i, n-1),
//   j(s, n)        = sum_zeta sum_i f*_zeta,i(s - c_i, n-1) c_i.
// These five values per site form the moment field R[3][5][N] (rho_A, rho_B,
// j_x, j_y, j_z; three rotating buffers, the one holding step n is
// R[n % 3], chosen in the kernels from the device step counter so that a
// captured step replays).  A step then reads 38 + 38 population words and
// the two densities of R(n) (the LDS density ring), and writes the 38 new
// words and the five values of R(n+1): 304 + 28 B per site in FP32.
//
// Inside a block (a 64 x TY tile marched along z) the sums are gathered
// without atomics: the velocities with c_x = +-1 move one lane with a wave
// shuffle, the three (c_y = 0) groups stay in the thread's own column, the
// groups with c_y = +-1 go to the row above or below through LDS, and the
// destination planes are held in registers until the plane z-1 has all its
// in-block contributions.  Contributions that leave the box:
//   through x  -> the side buffer H of the moment field (plain stores; the
//                 readers add it at the first and last column of a tile,
//                 see MomentView), so no scattered atomics are needed;
//   through y  -> float atomics on whole rows of R (coalesced), onto the
//                 face rows the previous step set to zero;
//   through z  -> float atomics on the face planes, likewise.
// A face site has two contributors (itself and one neighbour box), whose sum
// does not depend on their order; the few sites on box edges in y and z
// (and the x-y box corners) can differ in the last bit between runs, as the
// nodes that receive the particles' spread force do.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbmd_internal.h"
#include "lbmd_site.h"
#include "lbmd_stencil.h"

namespace lbmd {

constexpr int RQ = 5;  // rho_A, rho_B, j_x, j_y, j_z
constexpr int RINIT_BLOCK = 512, RINIT_GRID = 2048;

// moment field of the current state: R[step % 3] from the pulled
// populations, its x-boundary terms H[step % 2] zero; the two other R
// buffers cleared (the next step adds into one and clears the face sites of
// the other)
template <class S>
__global__ __launch_bounds__(RINIT_BLOCK) void k_rinit(const S* __restrict__ src_, arith_t<S>* __restrict__ Rall,
                                                       arith_t<S>* __restrict__ Hall, FluidConsts<arith_t<S>> K) {
  using C = arith_t<S>;
  load_step(K);
  const int nx = K.nx, ny = K.ny, nz = K.nz;
  const int64_t N = K.N;
  const int rin = int(uint64_t(K.step) % 3u);
  C* R = Rall + int64_t(rin) * RQ * N;
  C* R1 = Rall + int64_t(rin == 2 ? 0 : rin + 1) * RQ * N;
  C* R2 = Rall + int64_t(rin == 0 ? 2 : rin - 1) * RQ * N;
  const int tiles_x = (nx + 63) >> 6;
  const int64_t nh = int64_t(tiles_x) * 2 * RQ * nz * ny;
  C* H = Hall + int64_t(K.step & 1) * nh;
  const Pops<S> src = make_pops(src_, N, K.rho0);
  const int64_t stride = int64_t(gridDim.x) * RINIT_BLOCK;
  for (int64_t s = int64_t(blockIdx.x) * RINIT_BLOCK + threadIdx.x; s < N; s += stride) {
    const int x = int(s % nx), y = int((s / nx) % ny), z = int(s / (int64_t(nx) * ny));
    C f[2][19];
    pull<S, C>(src, x, y, z, nx, ny, nz, f);
    C rho[2], jt[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      C jj[3];
      moments_pairs<C>(f[c], rho[c], jj);
#pragma unroll
      for (int a = 0; a < 3; ++a) jt[a] += jj[a];
    }
    R[s] = rho[0];
    R[N + s] = rho[1];
#pragma unroll
    for (int a = 0; a < 3; ++a) R[(2 + a) * N + s] = jt[a];
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      R1[q * N + s] = C(0);
      R2[q * N + s] = C(0);
    }
  }
  for (int64_t i = int64_t(blockIdx.x) * RINIT_BLOCK + threadIdx.x; i < nh; i += stride) H[i] = C(0);
}

// value of the lane upstream in x (dx = +1: lane - 1, dx = -1: lane + 1);
// zero where that lane lies outside the 64-wide tile.  A whole-wave DPP
// shift (wave_shr:1 / wave_shl:1): a plain vector move, no LDS round trip.
// The edge lane (0 for wave_shr, 63 for wave_shl) has no source lane: with
// bound_ctrl it is written with zero (and the old value is zero as well), so
// no select is needed.
__device__ __forceinline__ uint32_t lane_shift(uint32_t v, int dx) {
  return dx > 0 ? uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x138, 0xf, 0xf, true))
                : uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_lane(float v, int dx, int) {
  return __builtin_bit_cast(float, lane_shift(__builtin_bit_cast(uint32_t, v), dx));
}
__device__ __forceinline__ double from_lane(double v, int dx, int) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = lane_shift(uint32_t(b), dx), hi = lane_shift(uint32_t(b >> 32), dx);
  return __builtin_bit_cast(double, lo | (hi << 32));
}

// In-tile sums of the velocities with (c_y, c_z) = (CY, CZ) that arrive in
// this lane's column: TA, TB per component and X = the x momentum they carry.
template <class C, int CY, int CZ>
__device__ __forceinline__ void group_sums(const C (&f)[2][19], int lane, C& TA, C& TB, C& X) {
  TA = TB = X = C(0);
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    if (D3Q19::cy[i] != CY || D3Q19::cz[i] != CZ) continue;
    const int cx = D3Q19::cx[i];
    C a = f[0][i], b = f[1][i];
    if (cx != 0) {
      a = from_lane(a, cx, lane);
      b = from_lane(b, cx, lane);
    }
    TA += a;
    TB += b;
    if (cx > 0) X += a + b;
    if (cx < 0) X -= a + b;
  }
}

// adds a group's sums to the five moments of a destination site
template <class C, int CY, int CZ>
__device__ __forceinline__ void add_group(C (&A)[RQ], C TA, C TB, C X) {
  A[0] += TA;
  A[1] += TB;
  A[2] += X;
  if (CY > 0) A[3] += TA + TB;
  if (CY < 0) A[3] -= TA + TB;
  if (CZ > 0) A[4] += TA + TB;
  if (CZ < 0) A[4] -= TA + TB;
}

// Occupancy: the deterministic BGK step with 4-byte arithmetic is held to
// 128 registers (4 waves per SIMD); the fluctuating and MRT steps (about 190
// registers) and FP64 run at 2 waves per SIMD and at most 8 rows, so that
// they are not squeezed into spills.
template <class S, bool NOISE, bool MRT>
constexpr int push_min_waves() {
  return sizeof(arith_t<S>) == 4 && !NOISE && !MRT ? 4 : 2;
}

template <class S, int TY, int FORCING, bool NOISE, bool MRT>
__global__ __launch_bounds__(64 * TY) __attribute__((amdgpu_waves_per_eu(push_min_waves<S, NOISE, MRT>(), 8)))
void k_push(const S* __restrict__ src_, S* __restrict__ dst_, arith_t<S>* __restrict__ Rall,
            FluidConsts<arith_t<S>> K, int tz, int tiles_x, int xcd, const uint32_t* __restrict__ mask,
            arith_t<S>* __restrict__ gP, arith_t<S>* __restrict__ gS, arith_t<S>* __restrict__ Hall,
            double* __restrict__ red, uint32_t* status, long long* bad) {
  using C = arith_t<S>;
  load_step(K);
  const int nx = K.nx, ny = K.ny, nz = K.nz;
  const int64_t N = K.N;
  const int64_t plane = int64_t(nx) * ny;
  const MomentView<C> in = moment_view<C>(Rall, Hall, K.step, nx, ny, nz, N);
  const int rin = int(uint64_t(K.step) % 3u);
  C* __restrict__ Rout = Rall + int64_t(rin == 2 ? 0 : rin + 1) * RQ * N;
  C* __restrict__ Rclr = Rall + int64_t(rin == 0 ? 2 : rin - 1) * RQ * N;
  const __amdgpu_buffer_rsrc_t rout = rsrc_of(Rout, uint64_t(RQ) * in.qR), rclr = rsrc_of(Rclr, uint64_t(RQ) * in.qR);
  const __amdgpu_buffer_rsrc_t hout =
      rsrc_of(Hall + int64_t((K.step + 1) & 1) * tiles_x * 2 * RQ * int64_t(nz) * ny, uint64_t(tiles_x) * 2 * in.sideH);

  __shared__ C ring[4][2][TY + 2][66];  // densities of step n (SC force)
  __shared__ C xb[2][TY][64][7];         // packs moving to row y+1 [0] and y-1 [1]
  __shared__ C srow[2][3][64][RQ];       // rows y0-1 [0] and y0+thv [1], per destination plane
  __shared__ C scol[2][3][TY + 2][RQ];   // columns x0-1 [0] and x0+twv [1], rows y0-1..y0+thv
  __shared__ double sums[5][64 * TY];    // per-thread FP64 conservation sums

  const Pops<S> src = make_pops(src_, N, K.rho0), dst = make_pops<S>(dst_, N, K.rho0, K.srkey);
  const Tile<TY> T(nx, ny, nz, tz, tiles_x, xcd, blockIdx.x, gridDim.x);
  const int lane = T.lane, wv = T.wv, x = T.x, y = T.y;
  const int twv = T.twv, thv = T.thv, z0 = T.z0, z1 = T.z1;
  const uint32_t hmine = uint32_t(T.x0 >> 6) * 2 * in.sideH;  // this tile's side blocks in hout

  auto load_interior = [&](int zp_raw, int slot) {
    const int zz = wrapi(zp_raw, nz);
    if (T.inside) {
      ring[slot][0][wv + 1][lane + 1] = in.at(0, x, y, zz);
      ring[slot][1][wv + 1][lane + 1] = in.at(1, x, y, zz);
    }
  };
  auto load_border = [&](int zp_raw, int slot) {
    const int zz = wrapi(zp_raw, nz);
    T.for_border([&](int hr, int hc) {
      const int bxx = wrapi(T.x0 - 1 + hc, nx), byy = wrapi(T.y0 - 1 + hr, ny);
      ring[slot][0][hr][hc] = in.at(0, bxx, byy, zz);
      ring[slot][1][hr][hc] = in.at(1, bxx, byy, zz);
    });
  };
  // site index of (xx, yy, zz) with periodic wrap of each coordinate
  auto site = [&](int xx, int yy, int zz) {
    return (uint32_t(wrapi(zz, nz)) * uint32_t(ny) + uint32_t(wrapi(yy, ny))) * uint32_t(nx) + uint32_t(wrapi(xx, nx));
  };
  // add v to quantity q of site s of the next step's field (buffer atomic in
  // FP32; FP64 has no buffer form: global atomic)
  auto radd = [&](uint32_t s, int q, C v) {
    if constexpr (sizeof(C) == 4)
      __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(v, rout, int(s * 4u), int(uint32_t(q) * in.qR), 0);
    else
      atomicAdd(&Rout[int64_t(q) * N + s], v);
  };

  for (int q = threadIdx.x; q < 2 * 3 * 64 * RQ; q += 64 * TY) (&srow[0][0][0][0])[q] = C(0);
  for (int q = threadIdx.x; q < 2 * 3 * (TY + 2) * RQ; q += 64 * TY) (&scol[0][0][0][0])[q] = C(0);
#pragma unroll
  for (int q = 0; q < 5; ++q) sums[q][threadIdx.x] = 0.0;

  // contributions gathered for destination plane Z (LDS slot sl) that leave
  // the box: rows y0-1 and y0+thv (atomics, waves 0 and thv-1), columns x0-1
  // and x0+twv (wave 0: the box's own rows of its own planes into the side
  // buffer, the corner rows and planes outside the box as atomics); the LDS
  // entries are cleared for reuse
  auto flush_shell = [&](int Z, int sl) {
    if (wv == 0 && lane < twv) {
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        radd(site(x, T.y0 - 1, Z), q, srow[0][sl][lane][q]);
        srow[0][sl][lane][q] = C(0);
      }
    }
    if (wv == thv - 1 && lane < twv) {
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        radd(site(x, T.y0 + thv, Z), q, srow[1][sl][lane][q]);
        srow[1][sl][lane][q] = C(0);
      }
    }
    if (wv == 0) {
      const bool own_plane = Z >= z0 && Z < z1;
      const int per = (thv + 2) * RQ;
      for (int it = lane; it < 2 * per; it += 64) {
        const int side = it / per, r = (it % per) / RQ, q = it % RQ;
        const C v = scol[side][sl][r][q];
        if (own_plane && r >= 1 && r <= thv)
          rsrc_store<C>(hout, hmine + uint32_t(side) * in.sideH + (uint32_t(Z) * uint32_t(ny) + uint32_t(T.y0 - 1 + r)) *
                                     uint32_t(sizeof(C)), uint32_t(q) * in.qH, v);
        else
          radd(site(side ? T.x0 + twv : T.x0 - 1, T.y0 - 1 + r, Z), q, v);
        scol[side][sl][r][q] = C(0);
      }
    }
  };
  const bool yface = wv == 0 || wv == thv - 1;
  // writes this column's moments of plane Z: atomics on the face rows and
  // face planes of the box and on the planes just outside it, plain stores
  // elsewhere (x faces included: what crosses x goes to the side buffer)
  auto flush_own = [&](const C (&A)[RQ], int Z) {
    if (!T.inside) return;
    const uint32_t s = site(x, y, Z);
    if (yface || Z <= z0 || Z >= z1 - 1) {
#pragma unroll
      for (int q = 0; q < RQ; ++q) radd(s, q, A[q]);
    } else {
#pragma unroll
      for (int q = 0; q < RQ; ++q) rsrc_store<C>(rout, s * uint32_t(sizeof(C)), uint32_t(q) * in.qR, A[q]);
    }
  };

  load_interior(z0 - 1, 0);
  load_border(z0 - 1, 0);
  load_interior(z0, 1);
  load_border(z0, 1);
  load_border(z0 + 1, 2);
  // moments of plane z-1 (contributions of planes z-2, z-1) and of plane z
  // (of plane z-1) carried into iteration z
  C Pm[RQ], P0[RQ];
#pragma unroll
  for (int q = 0; q < RQ; ++q) Pm[q] = P0[q] = C(0);

  for (int z = z0; z < z1; ++z) {
    const int k = z - z0;
    const int slm = k % 3, sl0 = (k + 1) % 3, slp = (k + 2) % 3;  // slots of planes z-1, z, z+1
    load_interior(z + 1, (k + 2) & 3);
    __syncthreads();
    C f[2][19];
    const int64_t s = z * plane + int64_t(y) * nx + x;
    if (T.inside) {
      C NA[3], NB[3];
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
      {
        SiteOut<C> o;
        o.rho[0] = m.rho[0];
        o.rho[1] = m.rho[1];
        o.j[0] = m.j[0];
        o.j[1] = m.j[1];
        o.j[2] = m.j[2];
        if (!moments_ok(o)) flag_unstable(status, bad, 1u, K.step);
        // one LDS add per quantity, no read back (each thread owns its column)
        atomicAdd(&sums[0][threadIdx.x], double(o.rho[0]));
        atomicAdd(&sums[1][threadIdx.x], double(o.rho[1]));
        atomicAdd(&sums[2][threadIdx.x], double(o.j[0]));
        atomicAdd(&sums[3][threadIdx.x], double(o.j[1]));
        atomicAdd(&sums[4][threadIdx.x], double(o.j[2]));
      }
      relax_site<C, FORCING, NOISE, MRT>(f, m, K, uint32_t(s));
      store<S, C, NOISE || Storage<S>::deviation, true>(dst, uint32_t(s), f, K.nt);
      // clear the sites of the buffer step n+1 adds into with atomics
      if (yface || z == z0 || z == z1 - 1) {
#pragma unroll
        for (int q = 0; q < RQ; ++q) rsrc_store<C>(rclr, uint32_t(s) * uint32_t(sizeof(C)), uint32_t(q) * in.qR, C(0));
      }
    } else {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i = 0; i < 19; ++i) f[c][i] = C(0);
    }
    if (z + 2 <= z1) load_border(z + 2, (k + 3) & 3);

    // --- gather of the next step's moments
    C Pp[RQ] = {0, 0, 0, 0, 0};
    {
      C TA, TB, X;
      group_sums<C, 0, 0>(f, lane, TA, TB, X);
      add_group<C, 0, 0>(P0, TA, TB, X);
      group_sums<C, 0, 1>(f, lane, TA, TB, X);
      add_group<C, 0, 1>(Pp, TA, TB, X);
      group_sums<C, 0, -1>(f, lane, TA, TB, X);
      add_group<C, 0, -1>(Pm, TA, TB, X);
    }
    {
      // groups moving to the row above: (c_y, c_z) = (1, 0), (1, 1), (1, -1)
      C u[7], X;
      group_sums<C, 1, 0>(f, lane, u[0], u[1], u[2]);
      group_sums<C, 1, 1>(f, lane, u[3], u[4], X);
      group_sums<C, 1, -1>(f, lane, u[5], u[6], X);
#pragma unroll
      for (int q = 0; q < 7; ++q) xb[0][wv][lane][q] = u[q];
      if (T.inside && wv == thv - 1) {  // the row above the box (single writer per entry)
        C t[RQ] = {0, 0, 0, 0, 0};
        add_group<C, 1, 0>(t, u[0], u[1], u[2]);
#pragma unroll
        for (int q = 0; q < RQ; ++q) srow[1][sl0][lane][q] += t[q], t[q] = C(0);
        add_group<C, 1, 1>(t, u[3], u[4], C(0));
#pragma unroll
        for (int q = 0; q < RQ; ++q) srow[1][slp][lane][q] += t[q], t[q] = C(0);
        add_group<C, 1, -1>(t, u[5], u[6], C(0));
#pragma unroll
        for (int q = 0; q < RQ; ++q) srow[1][slm][lane][q] += t[q];
      }
    }
    {
      // groups moving to the row below: (-1, 0), (-1, -1), (-1, 1)
      C d[7], X;
      group_sums<C, -1, 0>(f, lane, d[0], d[1], d[2]);
      group_sums<C, -1, -1>(f, lane, d[3], d[4], X);
      group_sums<C, -1, 1>(f, lane, d[5], d[6], X);
#pragma unroll
      for (int q = 0; q < 7; ++q) xb[1][wv][lane][q] = d[q];
      if (T.inside && wv == 0) {  // the row below the box
        C t[RQ] = {0, 0, 0, 0, 0};
        add_group<C, -1, 0>(t, d[0], d[1], d[2]);
#pragma unroll
        for (int q = 0; q < RQ; ++q) srow[0][sl0][lane][q] += t[q], t[q] = C(0);
        add_group<C, -1, -1>(t, d[3], d[4], C(0));
#pragma unroll
        for (int q = 0; q < RQ; ++q) srow[0][slm][lane][q] += t[q], t[q] = C(0);
        add_group<C, -1, 1>(t, d[5], d[6], C(0));
#pragma unroll
        for (int q = 0; q < RQ; ++q) srow[0][slp][lane][q] += t[q];
      }
    }
    // the columns left and right of the box: the velocities leaving through
    // x (several waves add to one entry).  The left-moving and right-moving
    // velocity of each (c_y, c_z) pair go out of lanes 0 and twv-1 in the
    // same instructions; a one-column tile sends both from lane 0.
    if (T.inside && (lane == 0 || lane == twv - 1)) {
      auto out = [&](int side, int il, int ir, int cy, int cz) {
        const C a = side == 0 ? f[0][il] : f[0][ir], b = side == 0 ? f[1][il] : f[1][ir], t = a + b;
        const int r = wv + 1 + cy;
        const int sl = cz > 0 ? slp : (cz < 0 ? slm : sl0);
        atomicAdd(&scol[side][sl][r][0], a);
        atomicAdd(&scol[side][sl][r][1], b);
        atomicAdd(&scol[side][sl][r][2], side == 0 ? -t : t);
        if (cy != 0) atomicAdd(&scol[side][sl][r][3], cy > 0 ? t : -t);
        if (cz != 0) atomicAdd(&scol[side][sl][r][4], cz > 0 ? t : -t);
      };
      const int npass = twv == 1 ? 2 : 1;
      for (int pass = 0; pass < npass; ++pass) {
        const int side = twv == 1 ? pass : (lane == 0 ? 0 : 1);
        // (left, right) velocity pairs: (-1,0,0)/(1,0,0), (-1,-1,0)/(1,-1,0),
        // (-1,1,0)/(1,1,0), (-1,0,-1)/(1,0,-1), (-1,0,1)/(1,0,1)
        out(side, 2, 1, 0, 0);
        out(side, 8, 9, -1, 0);
        out(side, 10, 7, 1, 0);
        out(side, 12, 13, 0, -1);
        out(side, 14, 11, 0, 1);
      }
    }
    __syncthreads();
    if (T.inside) {
      if (wv > 0) {  // from the row below: its c_y = +1 groups
        const C* u = xb[0][wv - 1][lane];
        add_group<C, 1, 0>(P0, u[0], u[1], u[2]);
        add_group<C, 1, 1>(Pp, u[3], u[4], C(0));
        add_group<C, 1, -1>(Pm, u[5], u[6], C(0));
      }
      if (wv + 1 < thv) {  // from the row above: its c_y = -1 groups
        const C* d = xb[1][wv + 1][lane];
        add_group<C, -1, 0>(P0, d[0], d[1], d[2]);
        add_group<C, -1, -1>(Pm, d[3], d[4], C(0));
        add_group<C, -1, 1>(Pp, d[5], d[6], C(0));
      }
    }
    // plane z-1 has all its in-block contributions now
    flush_own(Pm, z - 1);
    flush_shell(z - 1, slm);
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      Pm[q] = P0[q];
      P0[q] = Pp[q];
    }
  }
  // the last plane of the box and the plane after it
  const int kend = z1 - z0;
  flush_own(Pm, z1 - 1);
  flush_shell(z1 - 1, kend % 3);
  flush_own(P0, z1);
  flush_shell(z1, (kend + 1) % 3);
  double acc[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) acc[q] = sums[q][threadIdx.x];
  block_sum5<TY>(acc, red + 5 * int64_t(T.bid));
}

#ifndef LBMD_PUSH_ONLY_DECL
// ------------------------------------------------------------ launchers
template <class S>
static hipError_t rinit_t(lbmd_ctx* h) {
  using C = arith_t<S>;
  const FluidConsts<C> K = consts<S>(h);
  const int64_t nb = std::min<int64_t>((h->N + RINIT_BLOCK - 1) / RINIT_BLOCK, RINIT_GRID);
  hipLaunchKernelGGL(k_rinit<S>, dim3(nb), dim3(RINIT_BLOCK), 0, h->stream, (const S*)h->f[h->cur], (C*)h->R,
                     (C*)h->H, K);
  return hipGetLastError();
}

hipError_t push_init(lbmd_ctx* h) {
  if (!h->R || !h->H) return hipErrorInvalidValue;  // the field must be allocated
  switch (h->p.precision) {
    case LBMD_FP64: return rinit_t<double>(h);
    case LBMD_FP16DEV: return rinit_t<half_dev>(h);
    case LBMD_BF16DEV: return rinit_t<bf16_dev>(h);
    default: return rinit_t<float>(h);
  }
}

template <class S, int TY, int FORCING, bool NOISE, bool MRT>
static hipError_t push_launch(lbmd_ctx* h, const PushLaunch& L) {
  using C = arith_t<S>;
  const FluidConsts<C> K = consts<S>(h);
  const uint32_t* mask = h->np > 0 ? h->mask : nullptr;
  hipLaunchKernelGGL((k_push<S, TY, FORCING, NOISE, MRT>), dim3(L.nblk), dim3(64 * TY), 0, h->stream,
                     (const S*)h->f[h->cur], (S*)h->f[1 - h->cur], (C*)h->R, K, L.tz, L.tiles_x, L.xcd, mask,
                     (C*)h->gP, (C*)h->gS, (C*)h->H, h->red_fluid, h->status, h->bad_step);
  return hipGetLastError();
}

// 16 rows exist only for the deterministic BGK step with 4-byte arithmetic
// (push_rows_max); the tiling clamps the others to 8
template <class S, int TY>
static hipError_t push_by_physics(lbmd_ctx* h, const PushLaunch& L) {
  if (h->p.forcing == LBMD_FORCE_SHIFT) return push_launch<S, TY, LBMD_FORCE_SHIFT, false, false>(h, L);
  const bool noise = h->p.kT > 0.0;
  if constexpr (TY <= 8) {
    if (h->mrt)
      return noise ? push_launch<S, TY, LBMD_FORCE_PAPER, true, true>(h, L)
                   : push_launch<S, TY, LBMD_FORCE_PAPER, false, true>(h, L);
    if (noise) return push_launch<S, TY, LBMD_FORCE_PAPER, true, false>(h, L);
  } else {
    if (h->mrt || noise) return hipErrorInvalidConfiguration;
  }
  return push_launch<S, TY, LBMD_FORCE_PAPER, false, false>(h, L);
}

template <class S>
static hipError_t push_by_rows(lbmd_ctx* h, const PushLaunch& L) {
  if (L.ty > push_rows_max(h)) return hipErrorInvalidConfiguration;
  switch (L.ty) {
    case 2: return push_by_physics<S, 2>(h, L);
    case 4: return push_by_physics<S, 4>(h, L);
    case 16:
      if constexpr (sizeof(arith_t<S>) == 4) return push_by_physics<S, 16>(h, L);
      return hipErrorInvalidConfiguration;
    default: return push_by_physics<S, 8>(h, L);
  }
}

hipError_t push_pass(lbmd_ctx* h, const PushLaunch& L) {
  if (!h->R || !h->H) return hipErrorInvalidValue;  // the field must be allocated
  switch (h->p.precision) {
    case LBMD_FP64: return push_by_rows<double>(h, L);
    case LBMD_FP16DEV: return push_by_rows<half_dev>(h, L);
    case LBMD_BF16DEV: return push_by_rows<bf16_dev>(h, L);
    default: return push_by_rows<float>(h, L);
  }
}
#endif

}  // namespace lbmd
