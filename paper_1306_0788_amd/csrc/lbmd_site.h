// Per-site arithmetic of the fluid step, shared by every fluid kernel:
// moments, Shan-Chen force, particle-force split, BGK collision with the
// paper's forcing source term (or the velocity shift) and the fluctuating
// part.  Templated on the arithmetic type C (float or double).
#pragma once
#include "lbmd_internal.h"

namespace lbmd {

// Mode polynomials of the D3Q19 velocities, orthogonal under the weighted
// sum_i w_i e_ki e_li (Appendix: the mode basis comes from orthogonalised
// polynomials of c_i).  k = 0 mass, 1-3 momentum, 4 bulk, 5-9 shear, 10-18
// kinetic modes.  Evaluated at compile time after unrolling.
__host__ __device__ constexpr int mode_e(int k, int i) {
  const int x = D3Q19::cx[i], y = D3Q19::cy[i], z = D3Q19::cz[i];
  const int c2 = x * x + y * y + z * z;
  switch (k) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1;
    case 5: return 3 * x * x - c2;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return x * z;
    case 10: return (3 * c2 - 5) * x;
    case 11: return (3 * c2 - 5) * y;
    case 12: return (3 * c2 - 5) * z;
    case 13: return (y * y - z * z) * x;
    case 14: return (z * z - x * x) * y;
    case 15: return (x * x - y * y) * z;
    case 16: return 3 * c2 * c2 - 6 * c2 + 1;
    case 17: return (2 * c2 - 3) * (3 * x * x - c2);
    case 18: return (2 * c2 - 3) * (y * y - z * z);
  }
  return 0;
}
// 36 * b_k = 36 * sum_i w_i e_ki^2 (an integer)
__host__ __device__ constexpr int mode_b36(int k) {
  int s = 0;
  for (int i = 0; i < 19; ++i) s += (i == 0 ? 12 : (i <= 6 ? 2 : 1)) * mode_e(k, i) * mode_e(k, i);
  return s;
}

template <class C>
struct SiteOut {
  C rho[2];
  C j[3];  // raw momentum sum_zeta sum_i f c_i
};

template <class C>
__device__ __forceinline__ C csqrt(C v) { return sqrt(v); }

// f[2][19]: post-streaming populations at the site (overwritten with the
// post-collision values).  NA, NB: neighbour sums N_zeta = sum_i w_i
// rho_zeta(r+c_i) c_i.  gp: total particle force density at the node.
template <class C, int FORCING, bool NOISE>
__device__ __forceinline__ SiteOut<C> collide(C (&f)[2][19], const C (&NA)[3], const C (&NB)[3],
                                              const C (&gp)[3], const FluidConsts<C>& K, uint32_t site) {
  SiteOut<C> o;
  C jc[2][3];
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
    jc[c][0] = jx;
    jc[c][1] = jy;
    jc[c][2] = jz;
  }
  o.j[0] = jc[0][0] + jc[1][0];
  o.j[1] = jc[0][1] + jc[1][1];
  o.j[2] = jc[0][2] + jc[1][2];
  const C rt = o.rho[0] + o.rho[1];
  const C inv_rt = C(1) / rt;
  // Shan-Chen force g_zeta = -rho_zeta sum_zeta' G N_zeta' (Sec. 2, Eq.
  // SCforce) plus the particle force split by mass fraction
  C g[2][3];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const C frac = o.rho[c] * inv_rt;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      g[c][a] = -o.rho[c] * (K.G[c][0] * NA[a] + K.G[c][1] * NB[a]) + frac * gp[a];
  }
  C ueq[2][3];
  if (FORCING == LBMD_FORCE_PAPER) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const C u = (o.j[a] + C(0.5) * (g[0][a] + g[1][a])) * inv_rt;
      ueq[0][a] = u;
      ueq[1][a] = u;
    }
  } else {
    const C den = C(1) / (o.rho[0] * K.omega[0] + o.rho[1] * K.omega[1]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const C up = (jc[0][a] * K.omega[0] + jc[1][a] * K.omega[1]) * den;
#pragma unroll
      for (int c = 0; c < 2; ++c) ueq[c][a] = up + K.tau[c] * g[c][a] / o.rho[c];
    }
  }
  // fluctuations: 3 shared momentum normals (opposite sign for A and B), 15
  // per component for the bulk, shear and kinetic modes
  C z[36];
  C sc[2] = {0, 0}, sm = 0;
  if (NOISE) {
#pragma unroll
    for (int b = 0; b < 9; ++b) normals4<C>(K.seed, K.step, site, b, 0, &z[4 * b]);
    const C om = K.omega[0];
    const C relax = C(1) - (C(1) - om) * (C(1) - om);
    const C t = C(3) * K.kT * relax;  // (kT / c_s^2) (1 - (1+lambda)^2)
    sc[0] = csqrt(fmax(o.rho[0], C(0)) * t);
    sc[1] = csqrt(fmax(o.rho[1], C(0)) * t);
    sm = csqrt(fmax(o.rho[0] * o.rho[1] * inv_rt, C(0)) * t);
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const C om = K.omega[c];
    const C ux = ueq[c][0], uy = ueq[c][1], uz = ueq[c][2];
    const C usq = C(1.5) * (ux * ux + uy * uy + uz * uz);
    const C gx = g[c][0], gy = g[c][1], gz = g[c][2];
    const C ug = ux * gx + uy * gy + uz * gz;
    const C fpre = C(1) - C(0.5) * om;  // (2 + lambda)/2 with lambda = -1/tau
    // noise amplitudes per mode: sqrt(rho (kT/c_s^2) relax / b_k) r_k
    C a[19];
    if (NOISE) {
#pragma unroll
      for (int k = 1; k < 4; ++k)
        a[k] = (c == 0 ? sm : -sm) * z[k - 1] * C(6) / csqrt(C(mode_b36(k)));
#pragma unroll
      for (int k = 4; k < 19; ++k) a[k] = sc[c] * z[3 + 15 * c + (k - 4)] * C(6) / csqrt(C(mode_b36(k)));
    }
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const int cx = D3Q19::cx[i], cy = D3Q19::cy[i], cz = D3Q19::cz[i];
      const C cu = C(cx) * ux + C(cy) * uy + C(cz) * uz;
      const C w = weight<C>(i);
      const C feq = w * o.rho[c] * (C(1) + C(3) * cu + C(4.5) * cu * cu - usq);
      C fn = f[c][i] + om * (feq - f[c][i]);
      if (FORCING == LBMD_FORCE_PAPER) {
        const C cg = C(cx) * gx + C(cy) * gy + C(cz) * gz;
        fn += fpre * w * (C(3) * (cg - ug) + C(9) * cu * cg);
      }
      if (NOISE) {
        C s = 0;
#pragma unroll
        for (int k = 1; k < 19; ++k)
          if (mode_e(k, i) != 0) s += C(mode_e(k, i)) * a[k];
        fn += w * s;
      }
      f[c][i] = fn;
    }
  }
  return o;
}

}  // namespace lbmd
