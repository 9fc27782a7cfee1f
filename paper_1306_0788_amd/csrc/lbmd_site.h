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

// Mode group of mode k: 0 momentum (1-3), 1 bulk (4), 2 shear (5-9),
// 3 kinetic (10-18).
__host__ __device__ constexpr int mode_group(int k) { return k <= 3 ? 0 : (k == 4 ? 1 : (k <= 9 ? 2 : 3)); }
// Parity of mode k under c -> -c: odd modes change sign between the two
// velocities of an opposite pair (i, i + 1 for odd i), even modes do not.
__host__ __device__ constexpr bool mode_odd(int k) {
  for (int i = 1; i < 19; i += 2)
    if (mode_e(k, i) != 0) return mode_e(k, i + 1) == -mode_e(k, i);
  return false;
}
__host__ __device__ constexpr bool mode_parity_ok(int k) {
  for (int i = 1; i < 19; i += 2)
    if (mode_e(k, i + 1) != (mode_odd(k) ? -mode_e(k, i) : mode_e(k, i))) return false;
  return !mode_odd(k) || mode_e(k, 0) == 0;
}
// square root by Newton's iteration (compile-time tables)
__host__ __device__ constexpr double ct_sqrt(double x) {
  double r = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 80; ++i) r = 0.5 * (r + x / r);
  return r;
}
// per-mode constant of the fluctuation amplitude: 6 / sqrt(36 b_k), i.e.
// 1 / sqrt(b_k)
struct NoiseScale {
  double v[19];
  constexpr NoiseScale() : v() {
    for (int k = 1; k < 19; ++k) v[k] = 6.0 / ct_sqrt(double(mode_b36(k)));
  }
};
__device__ constexpr NoiseScale kNoiseScale{};
static_assert(mode_parity_ok(1) && mode_parity_ok(4) && mode_parity_ok(5) && mode_parity_ok(7) && mode_parity_ok(10) &&
                  mode_parity_ok(13) && mode_parity_ok(16) && mode_parity_ok(17) && mode_parity_ok(18),
              "every mode is even or odd under c -> -c");

template <class C>
struct SiteOut {
  C rho[2];
  C j[3];  // raw momentum sum_zeta sum_i f c_i
};

template <class C>
__device__ __forceinline__ C csqrt(C v) { return sqrt(v); }

// Moments of one component from opposite-pair sums and differences.
template <class C>
__device__ __forceinline__ void moments_pairs(const C (&f)[19], C& rho, C (&j)[3]) {
  C sp[9], dp[9];
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    sp[p] = f[2 * p + 1] + f[2 * p + 2];
    dp[p] = f[2 * p + 1] - f[2 * p + 2];
  }
  rho = f[0] + (((sp[0] + sp[1]) + (sp[2] + sp[3])) + ((sp[4] + sp[5]) + (sp[6] + sp[7]))) + sp[8];
  // pair velocities (+c of each pair): x, y, z, (1,1,0), (1,-1,0), (1,0,1),
  // (1,0,-1), (0,1,1), (0,1,-1)
  j[0] = ((dp[0] + dp[3]) + (dp[4] + dp[5])) + dp[6];
  j[1] = ((dp[1] + dp[3]) - (dp[4] - dp[7])) + dp[8];
  j[2] = ((dp[2] + dp[5]) - (dp[6] - dp[7])) - dp[8];
}

// BGK relaxation of one component towards f^eq(rho, u) (Appendix, Eq. feq)
// plus, if FORCE, the paper's forcing source term with all eigenvalues
// -1/tau (Appendix, last equations), which reads
//   fpre w_i [3 (c_i - u).g + 9 (c_i.u)(c_i.g)],  fpre = 1 - omega/2.
// Opposite velocities share the even part of both terms and flip the odd
// part, so each pair costs one evaluation.
template <class C, bool FORCE>
__device__ __forceinline__ void relax(C (&f)[19], C rho, const C (&u)[3], const C (&g)[3], C om) {
  const C usq = C(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const C keep = C(1) - om;
  const C fpre = C(1) - C(0.5) * om;
  const C ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
  // rest population
  {
    const C w = weight<C>(0);
    C e = om * (w * rho * (C(1) - usq));
    if (FORCE) e += fpre * w * (C(-3) * ug);
    f[0] = keep * f[0] + e;
  }
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    const int i = 2 * p + 1;
    const int cx = D3Q19::cx[i], cy = D3Q19::cy[i], cz = D3Q19::cz[i];
    const C w = weight<C>(i);
    C cu = 0, cg = 0;
    if (cx) { cu += cx > 0 ? u[0] : -u[0]; cg += cx > 0 ? g[0] : -g[0]; }
    if (cy) { cu += cy > 0 ? u[1] : -u[1]; cg += cy > 0 ? g[1] : -g[1]; }
    if (cz) { cu += cz > 0 ? u[2] : -u[2]; cg += cz > 0 ? g[2] : -g[2]; }
    const C wr = w * rho;
    C even = om * (wr * (C(1) - usq + C(4.5) * cu * cu));
    C odd = om * (C(3) * wr * cu);
    if (FORCE) {
      const C fw = fpre * w;
      even += fw * (C(9) * cu * cg - C(3) * ug);
      odd += fw * (C(3) * cg);
    }
    f[i] = keep * f[i] + (even + odd);
    f[i + 1] = keep * f[i + 1] + (even - odd);
  }
}

// Eigenvalue of mode k under MRT: lam = {momentum, bulk, shear, kinetic}.
template <class C>
__device__ __forceinline__ C mode_lambda(int k, const C (&lam)[4]) {
  return k <= 3 ? lam[0] : (k == 4 ? lam[1] : (k <= 9 ? lam[2] : lam[3]));
}

// MRT relaxation of one component (Appendix, Eqs. collis and MODES): mode k
// relaxes with its eigenvalue lambda_k towards the mode of f^eq(rho, u), and
// the forcing source term of the Appendix is added in its general form,
//   Delta_i = 3 w_i (2 + lambda_M)/2 g.c_i
//             + 9/2 w_i [G : c_i c_i - c_s^2 tr G],
//   G = (2 + lambda_s)/2 (u g + g u - 2/3 u.g 1) + (2 + lambda_b)/3 u.g 1.
// Since the mode basis is complete and w-orthogonal, the relaxation is
// applied as f_i += w_i sum_k e_ki lambda_k (m_k - m^eq_k) / b_k.
template <class C>
__device__ __forceinline__ void relax_mrt(C (&f)[19], C rho, const C (&u)[3], const C (&g)[3], const C (&lam)[4]) {
  const C usq = C(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  C d[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const C cu = C(D3Q19::cx[i]) * u[0] + C(D3Q19::cy[i]) * u[1] + C(D3Q19::cz[i]) * u[2];
    d[i] = f[i] - weight<C>(i) * rho * (C(1) + C(3) * cu + C(4.5) * cu * cu - usq);
  }
  C a[19];
  a[0] = C(0);
#pragma unroll
  for (int k = 1; k < 19; ++k) {
    C m = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i)
      if (mode_e(k, i) != 0) m += C(mode_e(k, i)) * d[i];
    a[k] = mode_lambda<C>(k, lam) * m * (C(36) / C(mode_b36(k)));
  }
  const C ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
  const C fs = (C(2) + lam[2]) * C(0.5), fb = (C(2) + lam[1]) / C(3), fm = (C(2) + lam[0]) * C(0.5);
  C G[3][3];
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y)
      G[x][y] = fs * (u[x] * g[y] + g[x] * u[y] - (x == y ? C(2) / C(3) * ug : C(0))) + (x == y ? fb * ug : C(0));
  const C trG = G[0][0] + G[1][1] + G[2][2];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int c[3] = {D3Q19::cx[i], D3Q19::cy[i], D3Q19::cz[i]};
    C s = 0;
#pragma unroll
    for (int k = 1; k < 19; ++k)
      if (mode_e(k, i) != 0) s += C(mode_e(k, i)) * a[k];
    C gc = 0, Gcc = 0;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      gc += C(c[x]) * g[x];
#pragma unroll
      for (int y = 0; y < 3; ++y) Gcc += C(c[x] * c[y]) * G[x][y];
    }
    f[i] += weight<C>(i) * (s + C(3) * fm * gc + C(4.5) * (Gcc - trG / C(3)));
  }
}

// Macroscopic part of the collision: densities, raw momentum, forces and
// the equilibrium velocity of each component.
template <class C>
struct Macro {
  C rho[2];
  C j[3];      // raw momentum sum_zeta sum_i f c_i
  C u[2][3];   // equilibrium velocity per component
  C g[2][3];   // total force density per component
  C inv_rt;
};

// NA, NB: neighbour sums N_zeta = sum_i w_i rho_zeta(r+c_i) c_i;
// gp: total particle force density at the node
// gu (used when fs is set): the fluid solvation sums U_zeta = sum_p
// lambda_zeta S_p at the node, [2][3]; the force on component zeta is
// -rho_zeta U_zeta (Sec. 2, Eq. solvation_lambda).  A register array and a
// flag rather than a pointer that may be null: a pointer to a local array
// would put the array in scratch memory.
template <class C, int FORCING>
__device__ __forceinline__ Macro<C> macro(const C (&f)[2][19], const C (&NA)[3], const C (&NB)[3],
                                          const C (&gp)[3], const FluidConsts<C>& K, const C (&gu)[6], bool fs) {
  Macro<C> m;
  C jc[2][3];
  moments_pairs<C>(f[0], m.rho[0], jc[0]);
  moments_pairs<C>(f[1], m.rho[1], jc[1]);
#pragma unroll
  for (int a = 0; a < 3; ++a) m.j[a] = jc[0][a] + jc[1][a];
  m.inv_rt = C(1) / (m.rho[0] + m.rho[1]);
  // Shan-Chen force g_zeta = -rho_zeta sum_zeta' G N_zeta' (Sec. 2, Eq.
  // SCforce) plus the particle force split by mass fraction
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const C frac = m.rho[c] * m.inv_rt;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      m.g[c][a] = -m.rho[c] * (K.G[c][0] * NA[a] + K.G[c][1] * NB[a]) + frac * gp[a] -
                  (fs ? m.rho[c] * gu[3 * c + a] : C(0));
  }
  if (FORCING == LBMD_FORCE_PAPER) {
    // barycentric velocity with half the total force (Appendix, u and
    // momentum_definition)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const C u = (m.j[a] + C(0.5) * (m.g[0][a] + m.g[1][a])) * m.inv_rt;
      m.u[0][a] = u;
      m.u[1][a] = u;
    }
  } else {
    // velocity shift: 1/tau-weighted common velocity shifted by
    // tau_zeta g_zeta / rho_zeta
    const C den = C(1) / (m.rho[0] * K.omega[0] + m.rho[1] * K.omega[1]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const C up = (jc[0][a] * K.omega[0] + jc[1][a] * K.omega[1]) * den;
#pragma unroll
      for (int c = 0; c < 2; ++c) m.u[c][a] = up + K.tau[c] * m.g[c][a] / m.rho[c];
    }
  }
  return m;
}

// velocity seen by the particles, u_c = (j + sum_zeta g_SC,zeta / 2) / rho,
// when m was built without particle force (for the paper's forcing it is
// the equilibrium velocity itself)
template <class C, int FORCING>
__device__ __forceinline__ void coupling_velocity(const Macro<C>& m, C (&uc)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
    uc[a] = FORCING == LBMD_FORCE_PAPER ? m.u[0][a] : (m.j[a] + C(0.5) * (m.g[0][a] + m.g[1][a])) * m.inv_rt;
}

// f_i += w_i sum_k e_ki a_k over the fluctuating modes k = 1..18, written
// out at compile time: the rest population takes the even modes; each
// opposite pair (I, I + 1) takes ev + od and ev - od, ev and od the sums of
// its even and odd modes.
template <class C, int K, int I>
__device__ __forceinline__ void modes_at(const C (&a)[19], C& ev, C& od) {
  if constexpr (K < 19) {
    constexpr int e = mode_e(K, I);
    if constexpr (e != 0) {
      if constexpr (mode_odd(K))
        od += C(e) * a[K];
      else
        ev += C(e) * a[K];
    }
    modes_at<C, K + 1, I>(a, ev, od);
  }
}
template <class C>
__device__ __forceinline__ void modes_to_rest(const C (&a)[19], C& f0) {
  C ev = 0, od = 0;
  modes_at<C, 1, 0>(a, ev, od);
  f0 += weight<C>(0) * ev;
}
template <class C, int I>
__device__ __forceinline__ void modes_to_pairs(const C (&a)[19], C (&f)[19]) {
  if constexpr (I < 19) {
    C ev = 0, od = 0;
    modes_at<C, 1, I>(a, ev, od);
    f[I] += weight<C>(I) * (ev + od);
    f[I + 1] += weight<C>(I) * (ev - od);
    modes_to_pairs<C, I + 2>(a, f);
  }
}

// Relaxation of both components (and fluctuations when NOISE).
template <class C, int FORCING, bool NOISE, bool MRT = false>
__device__ __forceinline__ void relax_site(C (&f)[2][19], const Macro<C>& m, const FluidConsts<C>& K,
                                           uint32_t site) {
  if (MRT) {
    relax_mrt<C>(f[0], m.rho[0], m.u[0], m.g[0], K.lam);
    relax_mrt<C>(f[1], m.rho[1], m.u[1], m.g[1], K.lam);
  } else {
    relax<C, FORCING == LBMD_FORCE_PAPER>(f[0], m.rho[0], m.u[0], m.g[0], K.omega[0]);
    relax<C, FORCING == LBMD_FORCE_PAPER>(f[1], m.rho[1], m.u[1], m.g[1], K.omega[1]);
  }
  if (NOISE) {
    // fluctuations (Appendix, Eq. MODES): 3 shared momentum normals with
    // opposite sign for A and B, 15 per component for the bulk, shear and
    // kinetic modes; amplitude of mode k
    //   sqrt(rho (kT/c_s^2) (1 - (1 + lambda_k)^2) / b_k)
    //     = sqrt(rho) * namp[group(k)] * (6 / sqrt(36 b_k))
    // (the group factor from the host, the last one a compile-time
    // constant), mapped back with w_i e_ki
    C z[36];
#pragma unroll
    for (int b = 0; b < 9; ++b) normals4<C>(K.seed, K.step, site, b, 0, &z[4 * b]);
    const C sA = csqrt(fmax(m.rho[0], C(0))), sB = csqrt(fmax(m.rho[1], C(0)));
    const C sM = csqrt(fmax(m.rho[0] * m.rho[1] * m.inv_rt, C(0)));
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      C a[19];
#pragma unroll
      for (int k = 1; k < 19; ++k) {
        const C amp = (MRT ? K.namp[mode_group(k)] : K.namp[0]) * C(kNoiseScale.v[k]);
        if (k < 4)
          a[k] = (c == 0 ? sM : -sM) * amp * z[k - 1];
        else
          a[k] = (c == 0 ? sA : sB) * amp * z[3 + 15 * c + (k - 4)];
      }
      // back to the populations: the two velocities of an opposite pair share
      // the even modes' sum and take the odd modes' sum with opposite signs
      modes_to_rest<C>(a, f[c][0]);
      modes_to_pairs<C, 1>(a, f[c]);
    }
  }
}

// whole collision at one site (f overwritten with the post-collision values)
template <class C, int FORCING, bool NOISE>
__device__ __forceinline__ SiteOut<C> collide(C (&f)[2][19], const C (&NA)[3], const C (&NB)[3],
                                              const C (&gp)[3], const FluidConsts<C>& K, uint32_t site,
                                              const C (&gu)[6], bool fs) {
  const Macro<C> m = macro<C, FORCING>(f, NA, NB, gp, K, gu, fs);
  relax_site<C, FORCING, NOISE>(f, m, K, site);
  SiteOut<C> o;
  o.rho[0] = m.rho[0];
  o.rho[1] = m.rho[1];
  o.j[0] = m.j[0];
  o.j[1] = m.j[1];
  o.j[2] = m.j[2];
  return o;
}

}  // namespace lbmd
