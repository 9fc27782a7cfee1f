/*
 * Oracle: plain FP64 CPU statement of one time step of the two-component
 * Shan-Chen lattice Boltzmann fluid coupled to point particles
 * (arXiv 1306.0788).  TEST INFRASTRUCTURE ONLY -- see orc.h.
 *
 * The step follows the paper's definitions in this order:
 *   S1  moments rho_zeta, raw momentum                (Appendix, modes)
 *   S2  Shan-Chen force from lattice neighbour sums    (Sec. 2, Eq. SCforce)
 *   S3  velocity seen by the particles u_c            (Appendix, u definition)
 *   S4  particle half kick and drift                  (velocity Verlet, dt=1)
 *   S5  friction + solvation + random force            (Sec. 2, Eqs. NEWTON
 *       at the new positions, trilinear interpolation    and solvation_kappa)
 *   S5b fluid solvation force on the nodes of each     (Sec. 2, Eq.
 *       particle's cell, its momentum returned to the     solvation_lambda)
 *       particle
 *   S6  opposite coupling force spread onto the 8      (Sec. 2, momentum
 *       nodes                                            returned by the same
 *                                                       interpolation)
 *   S7  collision in mode space with forcing and noise (Appendix, Eqs. collis,
 *                                                       feq, MODES, forcing
 *                                                       source term)
 *   S8  streaming with periodic wrap                   (Eq. LBMIX)
 *   S9  second half kick
 *   S10 status: a non-positive or non-finite density, or a non-finite
 *       particle quantity, makes the step report ORC_EUNSTABLE (Sec. 3:
 *       negative densities mean failure of the Shan-Chen scheme).
 * Where the paper is silent the readings used are stated at each place.
 */
#include "orc.h"
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Threads: the per-site loops (moments, neighbour sums, the collision and
   streaming of every site) and the per-particle force loops are split over
   OpenMP threads; every site and particle is still computed by the same
   serial arithmetic, and the global sums and the spread onto the nodes stay
   serial in a fixed order, so any thread count gives bit-identical
   results. */
void orc_set_threads(int32_t n) { omp_set_num_threads(n > 0 ? n : 1); }
int32_t orc_get_threads(void) { return omp_get_max_threads(); }

/* D3Q19 velocities (Appendix, Eq. velo), opposite pairs adjacent.  The
   order inside the groups is not fixed by the paper; this one is used by
   every array this oracle reads or writes. */
static const int C[ORC_Q][3] = {
  { 0, 0, 0},
  { 1, 0, 0}, {-1, 0, 0}, { 0, 1, 0}, { 0,-1, 0}, { 0, 0, 1}, { 0, 0,-1},
  { 1, 1, 0}, {-1,-1, 0}, { 1,-1, 0}, {-1, 1, 0},
  { 1, 0, 1}, {-1, 0,-1}, { 1, 0,-1}, {-1, 0, 1},
  { 0, 1, 1}, { 0,-1,-1}, { 0, 1,-1}, { 0,-1, 1}};

/* weights (Appendix, Eq. weights) */
static double Wt(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

static const double CS2 = 1.0 / 3.0; /* c_s^2 of D3Q19 */

void orc_lattice(int32_t* c, double* w) {
  for (int i = 0; i < ORC_Q; i++) {
    for (int a = 0; a < 3; a++) c[3 * i + a] = C[i][a];
    w[i] = Wt(i);
  }
}

/* Mode basis: polynomials of the velocities, orthogonal under the weighted
   product sum_i w_i e_ki e_li = b_k delta_kl (Appendix: the basis vectors of
   mode space come from orthogonalising polynomials of c_i).  The polynomial
   set is the usual D3Q19 one of the fluctuating-LB literature:
     k=0 mass; 1-3 momentum; 4 bulk; 5-9 shear; 10-18 kinetic (ghost). */
static double mode_poly(int k, const int* c) {
  double x = c[0], y = c[1], z = c[2];
  double c2 = x * x + y * y + z * z;
  switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1.0;
    case 5: return 3.0 * x * x - c2;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return x * z;
    case 10: return (3.0 * c2 - 5.0) * x;
    case 11: return (3.0 * c2 - 5.0) * y;
    case 12: return (3.0 * c2 - 5.0) * z;
    case 13: return (y * y - z * z) * x;
    case 14: return (z * z - x * x) * y;
    case 15: return (x * x - y * y) * z;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * x * x - c2);
    case 18: return (2.0 * c2 - 3.0) * (y * y - z * z);
  }
  return 0.0;
}

void orc_mode_basis(double* e, double* b) {
  for (int k = 0; k < ORC_Q; k++) {
    b[k] = 0.0;
    for (int i = 0; i < ORC_Q; i++) {
      e[k * ORC_Q + i] = mode_poly(k, C[i]);
      b[k] += Wt(i) * e[k * ORC_Q + i] * e[k * ORC_Q + i];
    }
  }
}

/* Equilibrium (Appendix, Eq. feq).  The identity in the second-order term
   is read as c_s^2 times the identity: with it the second moment is the
   ideal-gas pressure plus rho u u, as the momentum flux of the Chapman-
   Enskog section requires (the printed form drops the c_s^2). */
void orc_equilibrium(double rho, const double* u, double* feq) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < ORC_Q; i++) {
    double uc = u[0] * C[i][0] + u[1] * C[i][1] + u[2] * C[i][2];
    double uu_ccmI = uc * uc - CS2 * uu; /* uu:(c c - c_s^2 1) */
    feq[i] = Wt(i) * rho * (1.0 + uc / CS2 + uu_ccmI / (2.0 * CS2 * CS2));
  }
}

/* Forcing source term (Appendix, last equations): a first-order part along
   g.c_i scaled by (2+lambda_M)/2 and a second-order part built from the
   tensor G(u, g) with the shear and bulk eigenvalues.  Time step 1. */
void orc_forcing_term(double lam_mom, double lam_shear, double lam_bulk,
                      const double* u, const double* g, double* dg) {
  double ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
  double Gt[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      double d = (a == b) ? 1.0 : 0.0;
      Gt[a][b] = 0.5 * (2.0 + lam_shear) * (u[a] * g[b] + g[a] * u[b] - (2.0 / 3.0) * ug * d) +
                 (2.0 + lam_bulk) / 3.0 * ug * d;
    }
  for (int i = 0; i < ORC_Q; i++) {
    double gc = g[0] * C[i][0] + g[1] * C[i][1] + g[2] * C[i][2];
    double GccmI = 0.0; /* G:(c c - c_s^2 1) */
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++)
        GccmI += Gt[a][b] * (C[i][a] * C[i][b] - (a == b ? CS2 : 0.0));
    dg[i] = Wt(i) / CS2 * 0.5 * (2.0 + lam_mom) * gc + Wt(i) / CS2 * (GccmI / (2.0 * CS2));
  }
}

/* Philox4x32-10 counter-based generator, from its published definition
   (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,
   3", SC'11): ten rounds of two 32x32->64 multiplications whose high halves
   are xored with the other counter words and the round key; the key is
   bumped by two Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Box-Muller transform of two 32-bit words into two standard normals. */
void orc_box_muller(uint32_t a, uint32_t b, double* z0, double* z1) {
  const double two32 = 4294967296.0;
  double u1 = ((double)a + 0.5) / two32;
  double u2 = ((double)b + 0.5) / two32;
  double r = sqrt(-2.0 * log(u1));
  double th = 2.0 * M_PI * u2;
  *z0 = r * cos(th);
  *z1 = r * sin(th);
}

/* Normals for one site or particle: counter = (index, step low word,
   block | tag<<16, step high word), key = seed.  Block j gives normals
   4j..4j+3 from the word pairs (0,1) and (2,3). */
void orc_site_normals(uint64_t seed, int64_t step, int64_t index, int32_t tag,
                      int32_t nblocks, double* z) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int j = 0; j < nblocks; j++) {
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)step, (uint32_t)j | ((uint32_t)tag << 16),
                       (uint32_t)((uint64_t)step >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    orc_box_muller(o[0], o[1], &z[4 * j + 0], &z[4 * j + 1]);
    orc_box_muller(o[2], o[3], &z[4 * j + 2], &z[4 * j + 3]);
  }
}

/* ------------------------------------------------------------------ */
static int64_t nsites(const orc_params* P) { return (int64_t)P->nx * P->ny * P->nz; }
static int pmod(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }
static int64_t site_of(const orc_params* P, int x, int y, int z) {
  return ((int64_t)pmod(z, P->nz) * P->ny + pmod(y, P->ny)) * P->nx + pmod(x, P->nx);
}
static void coords_of(const orc_params* P, int64_t s, int* x, int* y, int* z) {
  *x = (int)(s % P->nx);
  *y = (int)((s / P->nx) % P->ny);
  *z = (int)(s / ((int64_t)P->nx * P->ny));
}

/* wrap a coordinate into [0, L) */
static double wrap(double x, double L) {
  x -= L * floor(x / L);
  if (x >= L) x -= L;
  if (x < 0.0) x += L;
  return x;
}

void orc_init_populations(const orc_params* P, const double* rho, double* f) {
  int64_t N = nsites(P);
  for (int c = 0; c < 2; c++)
    for (int i = 0; i < ORC_Q; i++)
      for (int64_t s = 0; s < N; s++) f[((int64_t)c * ORC_Q + i) * N + s] = Wt(i) * rho[c * N + s];
}

/* S1: rho_zeta = sum_i f_zeta i, raw momentum sum_zeta sum_i f c_i. */
void orc_moments(const orc_params* P, const double* f, double* rho, double* j, double* jc) {
  int64_t N = nsites(P);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; s++) {
    double jt[3] = {0, 0, 0};
    for (int c = 0; c < 2; c++) {
      double r = 0.0, jj[3] = {0, 0, 0};
      for (int i = 0; i < ORC_Q; i++) {
        double fi = f[((int64_t)c * ORC_Q + i) * N + s];
        r += fi;
        for (int a = 0; a < 3; a++) jj[a] += fi * C[i][a];
      }
      rho[c * N + s] = r;
      for (int a = 0; a < 3; a++) {
        if (jc) jc[((int64_t)c * 3 + a) * N + s] = jj[a];
        jt[a] += jj[a];
      }
    }
    for (int a = 0; a < 3; a++) j[a * N + s] = jt[a];
  }
}

/* S2: N_zeta(r) = sum_i w_i rho_zeta(r + c_i) c_i.  The Shan-Chen force
   (Sec. 2, Eq. SCforce) is -rho_zeta sum_zeta' g N_zeta', i.e. the link
   vector r'-r is taken as w_i c_i with proportionality constant 1. */
void orc_neighbour_sums(const orc_params* P, const double* rho, double* Ns) {
  int64_t N = nsites(P);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; s++) {
    int x, y, z;
    coords_of(P, s, &x, &y, &z);
    for (int c = 0; c < 2; c++) {
      double acc[3] = {0, 0, 0};
      for (int i = 1; i < ORC_Q; i++) {
        double r = rho[c * N + site_of(P, x + C[i][0], y + C[i][1], z + C[i][2])];
        for (int a = 0; a < 3; a++) acc[a] += Wt(i) * r * C[i][a];
      }
      for (int a = 0; a < 3; a++) Ns[((int64_t)c * 3 + a) * N + s] = acc[a];
    }
  }
}

/* trilinear weights: nodes at integer coordinates, the particle in the cell
   whose lowest corner is floor(x); node k = ox + 2 oy + 4 oz. */
void orc_interp_weights(const double* x, int32_t nx, int32_t ny, int32_t nz, int64_t* node,
                        double* W) {
  int L[3] = {nx, ny, nz};
  int i0[3];
  double d[3];
  for (int a = 0; a < 3; a++) {
    double fl = floor(x[a]);
    i0[a] = (int)fl;
    d[a] = x[a] - fl;
  }
  for (int k = 0; k < 8; k++) {
    int o[3] = {k & 1, (k >> 1) & 1, (k >> 2) & 1};
    double w = 1.0;
    int n[3];
    for (int a = 0; a < 3; a++) {
      w *= o[a] ? d[a] : 1.0 - d[a];
      n[a] = pmod(i0[a] + o[a], L[a]);
    }
    W[k] = w;
    node[k] = ((int64_t)n[2] * ny + n[1]) * nx + n[0];
  }
}

void orc_solvation_fluid_force(const orc_params* P, const double* rho, int64_t np, const double* x,
                               const int32_t* type, double* fs, double* back) {
  int64_t N = nsites(P);
  int L[3] = {P->nx, P->ny, P->nz};
  for (int64_t p = 0; p < np; p++) {
    int t = type ? type[p] : 0;
    double lam[2] = {P->lambda_fs[t][0], P->lambda_fs[t][1]};
    double b[3] = {0.0, 0.0, 0.0};
    double fl[3];
    for (int a = 0; a < 3; a++) fl[a] = floor(x[3 * p + a]);
    for (int k = 0; k < 8; k++) {
      int o[3] = {k & 1, (k >> 1) & 1, (k >> 2) & 1};
      double d[3];
      int n[3];
      for (int a = 0; a < 3; a++) {
        d[a] = x[3 * p + a] - (fl[a] + o[a]); /* from the vertex to the particle */
        n[a] = pmod((int)fl[a] + o[a], L[a]);
      }
      int64_t site = ((int64_t)n[2] * P->ny + n[1]) * P->nx + n[0];
      /* links pointing into the half space of the particle, each weighted
         by (r' - r)/|r' - r|^2 */
      double S[3] = {0.0, 0.0, 0.0};
      for (int i = 1; i < ORC_Q; i++) {
        double dot = d[0] * C[i][0] + d[1] * C[i][1] + d[2] * C[i][2];
        if (dot > 0.0) {
          double c2 = C[i][0] * C[i][0] + C[i][1] * C[i][1] + C[i][2] * C[i][2];
          for (int a = 0; a < 3; a++) S[a] += C[i][a] / c2;
        }
      }
      for (int c = 0; c < 2; c++)
        for (int a = 0; a < 3; a++) {
          double force = -lam[c] * rho[c * N + site] * S[a];
          fs[((int64_t)c * 3 + a) * N + site] += force;
          b[a] -= force;
        }
    }
    for (int a = 0; a < 3; a++) back[3 * p + a] = b[a];
  }
}

/* Pair potentials: 0 = WCA (Sec. 2.. examples, with the usual +eps shift),
   1 = screened Debye-Hueckel, 2 = FENE bond.  qq = product of charges. */
double orc_pair_energy(const orc_params* P, int32_t kind, double r, double qq) {
  if (kind == 0) {
    double rc = pow(2.0, 1.0 / 6.0) * P->wca_sigma;
    if (r >= rc) return 0.0;
    double s6 = pow(P->wca_sigma / r, 6);
    return 4.0 * P->wca_eps * (s6 * s6 - s6) + P->wca_eps;
  } else if (kind == 1) {
    if (r >= P->dh_rc) return 0.0;
    return qq * P->dh_lB * exp(-P->dh_kappa * r) / r;
  } else {
    double q = r / P->fene_R0;
    if (q >= 1.0) return NAN;
    return -0.5 * P->fene_k * P->fene_R0 * P->fene_R0 * log(1.0 - q * q);
  }
}

/* radial force -dU/dr (positive = repulsive) */
double orc_pair_force(const orc_params* P, int32_t kind, double r, double qq) {
  if (kind == 0) {
    double rc = pow(2.0, 1.0 / 6.0) * P->wca_sigma;
    if (r >= rc) return 0.0;
    double s6 = pow(P->wca_sigma / r, 6);
    return 24.0 * P->wca_eps * (2.0 * s6 * s6 - s6) / r;
  } else if (kind == 1) {
    if (r >= P->dh_rc) return 0.0;
    return qq * P->dh_lB * exp(-P->dh_kappa * r) * (1.0 + P->dh_kappa * r) / (r * r);
  } else {
    double q = r / P->fene_R0;
    if (q >= 1.0) return NAN;
    return -P->fene_k * r / (1.0 - q * q);
  }
}

static void min_image(const orc_params* P, const double* xi, const double* xj, double* d) {
  double L[3] = {P->nx, P->ny, P->nz};
  for (int a = 0; a < 3; a++) {
    double t = xj[a] - xi[a];
    d[a] = t - L[a] * floor(t / L[a] + 0.5);
  }
}

/* force on i from j through potential `kind`, added into Fi */
static void add_pair(const orc_params* P, int kind, const double* xi, const double* xj, double qq,
                     double* Fi) {
  double d[3];
  min_image(P, xi, xj, d);
  double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double fr = orc_pair_force(P, kind, r, qq);
  if (fr == 0.0) return;
  for (int a = 0; a < 3; a++) Fi[a] -= fr * d[a] / r;
}

static double qq_of(const orc_params* P, const int32_t* type, int64_t i, int64_t j) {
  return P->charge[type ? type[i] : 0] * P->charge[type ? type[j] : 0];
}

int orc_conservative_force_one(const orc_params* P, int64_t np, const double* x, const int32_t* type,
                               int64_t nbonds, const int32_t* bonds, int64_t p, double* Fp) {
  Fp[0] = Fp[1] = Fp[2] = 0.0;
  for (int64_t q = 0; q < np; q++) {
    if (q == p) continue;
    if (P->wca_on) add_pair(P, 0, &x[3 * p], &x[3 * q], 0.0, Fp);
    if (P->dh_on) add_pair(P, 1, &x[3 * p], &x[3 * q], qq_of(P, type, p, q), Fp);
  }
  if (P->fene_on)
    for (int64_t b = 0; b < nbonds; b++) {
      int64_t i = bonds[2 * b], j = bonds[2 * b + 1];
      if (i == p) add_pair(P, 2, &x[3 * i], &x[3 * j], 0.0, Fp);
      if (j == p) add_pair(P, 2, &x[3 * j], &x[3 * i], 0.0, Fp);
    }
  return (isfinite(Fp[0]) && isfinite(Fp[1]) && isfinite(Fp[2])) ? ORC_OK : ORC_EUNSTABLE;
}

int orc_conservative_forces(const orc_params* P, int64_t np, const double* x, const int32_t* type,
                            int64_t nbonds, const int32_t* bonds, double* F) {
  int st = ORC_OK;
#pragma omp parallel for schedule(dynamic, 64) reduction(min : st)
  for (int64_t p = 0; p < np; p++)
    if (orc_conservative_force_one(P, np, x, type, nbonds, bonds, p, &F[3 * p]) != ORC_OK)
      st = ORC_EUNSTABLE;
  return st;
}

/* relaxation eigenvalue of mode k for component c */
static double lambda_of(const orc_params* P, int c, int k) {
  if (k == 0) return 0.0;
  if (!P->mrt) return -1.0 / P->tau[c];
  if (k <= 3) return P->lambda_mom;
  if (k == 4) return P->lambda_bulk;
  if (k <= 9) return P->lambda_shear;
  return P->lambda_ghost;
}

static int check_params(const orc_params* P) {
  if (P->nx < 1 || P->ny < 1 || P->nz < 1) return ORC_EINVAL;
  if (!P->mrt && (P->tau[0] <= 0.5 || P->tau[1] <= 0.5)) return ORC_EINVAL;
  if (P->forcing == ORC_FORCE_PAPER && !P->mrt && P->tau[0] != P->tau[1]) return ORC_EINVAL;
  if (P->forcing == ORC_FORCE_SHIFT && P->kT != 0.0) return ORC_EINVAL;
  if (P->forcing == ORC_FORCE_SHIFT && P->mrt) return ORC_EINVAL;
  if (P->kT < 0.0) return ORC_EINVAL;
  return ORC_OK;
}

/* S7 for one site: collision of both components in mode space.
   fin  [2][19] post-streaming populations at the site
   gsc  [2][3]  Shan-Chen force per component, gP [3] particle force (total)
   out  [2][19] post-collision populations */
static double E[ORC_Q][ORC_Q], B[ORC_Q];
static void basis_init(void) {
#pragma omp critical(orc_basis)
  {
    static int ready = 0;
    if (!ready) {
      orc_mode_basis(&E[0][0], B);
      ready = 1;
    }
  }
}

static void collide_site(const orc_params* P, int64_t step, int64_t site, const double* fin,
                         const double* gsc, const double* gP, const double* gfs, double* out) {
  double rho[2], jc[2][3];
  for (int c = 0; c < 2; c++) {
    rho[c] = 0.0;
    jc[c][0] = jc[c][1] = jc[c][2] = 0.0;
    for (int i = 0; i < ORC_Q; i++) {
      rho[c] += fin[c * ORC_Q + i];
      for (int a = 0; a < 3; a++) jc[c][a] += fin[c * ORC_Q + i] * C[i][a];
    }
  }
  double rt = rho[0] + rho[1];
  /* particle back-reaction split between the components by mass fraction
     (the paper does not say which component receives it); the fluid
     solvation force (if any) acts on its own component */
  double g[2][3];
  for (int c = 0; c < 2; c++)
    for (int a = 0; a < 3; a++) g[c][a] = gsc[3 * c + a] + rho[c] / rt * gP[a] + (gfs ? gfs[3 * c + a] : 0.0);

  /* equilibrium velocity per component */
  double ueq[2][3];
  if (P->forcing == ORC_FORCE_PAPER) {
    /* barycentric velocity with half the total force (Appendix, u and
       momentum_definition) */
    for (int a = 0; a < 3; a++) {
      double u = (jc[0][a] + jc[1][a] + 0.5 * (g[0][a] + g[1][a])) / rt;
      ueq[0][a] = ueq[1][a] = u;
    }
  } else {
    /* velocity shift: common velocity weighted by 1/tau, then shifted by
       tau_zeta g_zeta / rho_zeta per component */
    double den = rho[0] / P->tau[0] + rho[1] / P->tau[1];
    for (int a = 0; a < 3; a++) {
      double up = (jc[0][a] / P->tau[0] + jc[1][a] / P->tau[1]) / den;
      for (int c = 0; c < 2; c++) ueq[c][a] = up + P->tau[c] * g[c][a] / rho[c];
    }
  }

  /* noise draws (only if kT > 0): 3 shared momentum normals with opposite
     sign for the two components, then 15 per component for modes 4..18 */
  double z[36];
  int noisy = P->kT > 0.0;
  if (noisy) orc_site_normals(P->seed, step, site, 0, 9, z);

  for (int c = 0; c < 2; c++) {
    double feq[ORC_Q], dg[ORC_Q];
    orc_equilibrium(rho[c], ueq[c], feq);
    if (P->forcing == ORC_FORCE_PAPER)
      orc_forcing_term(lambda_of(P, c, 1), lambda_of(P, c, 5), lambda_of(P, c, 4), ueq[c], g[c], dg);
    else
      for (int i = 0; i < ORC_Q; i++) dg[i] = 0.0;
    double ms[ORC_Q];
    for (int k = 0; k < ORC_Q; k++) {
      double m = 0.0, meq = 0.0, mg = 0.0;
      for (int i = 0; i < ORC_Q; i++) {
        m += E[k][i] * fin[c * ORC_Q + i];
        meq += E[k][i] * feq[i];
        mg += E[k][i] * dg[i];
      }
      double lam = lambda_of(P, c, k);
      ms[k] = meq + (1.0 + lam) * (m - meq) + mg;
      if (noisy && k > 0) {
        /* amplitude from the equilibrium variance rho (kT/c_s^2) b_k of a
           mode and its relaxation factor (1+lambda)^2 (the amplitudes are
           deferred by the paper to the fluctuating-LB literature) */
        double relax = 1.0 - (1.0 + lam) * (1.0 + lam);
        if (k <= 3) {
          double mu = rho[0] * rho[1] / rt;
          double phi = sqrt(fmax(mu, 0.0) * (P->kT / CS2) * B[k] * relax);
          ms[k] += (c == 0 ? 1.0 : -1.0) * phi * z[k - 1];
        } else {
          double phi = sqrt(fmax(rho[c], 0.0) * (P->kT / CS2) * B[k] * relax);
          ms[k] += phi * z[3 + 15 * c + (k - 4)];
        }
      }
    }
    for (int i = 0; i < ORC_Q; i++) {
      double s = 0.0;
      for (int k = 0; k < ORC_Q; k++) s += E[k][i] * ms[k] / B[k];
      out[c * ORC_Q + i] = Wt(i) * s;
    }
  }
}

void orc_node_fields(const orc_params* P, const double* f, int64_t site, double* uc, double* grad) {
  int64_t N = nsites(P);
  int x, y, z;
  coords_of(P, site, &x, &y, &z);
  double rho[2], j[3] = {0, 0, 0}, Ns[2][3];
  for (int c = 0; c < 2; c++) {
    rho[c] = 0.0;
    for (int i = 0; i < ORC_Q; i++) {
      double fi = f[((int64_t)c * ORC_Q + i) * N + site];
      rho[c] += fi;
      for (int a = 0; a < 3; a++) j[a] += fi * C[i][a];
    }
    for (int a = 0; a < 3; a++) Ns[c][a] = 0.0;
    for (int i = 1; i < ORC_Q; i++) {
      int64_t s2 = site_of(P, x + C[i][0], y + C[i][1], z + C[i][2]);
      double r = 0.0;
      for (int q = 0; q < ORC_Q; q++) r += f[((int64_t)c * ORC_Q + q) * N + s2];
      for (int a = 0; a < 3; a++) Ns[c][a] += Wt(i) * r * C[i][a];
    }
  }
  double rt = rho[0] + rho[1];
  for (int a = 0; a < 3; a++) {
    double gsum = 0.0;
    for (int c = 0; c < 2; c++) {
      double gsc = -rho[c] * (P->G[c][0] * Ns[0][a] + P->G[c][1] * Ns[1][a]);
      gsum += gsc;
      grad[3 * c + a] = Ns[c][a] / CS2;
    }
    uc[a] = (j[a] + 0.5 * gsum) / rt;
  }
}

void orc_coupling_force_one(const orc_params* P, int64_t step, const double* f, const double* xp,
                            const double* vp, int32_t type, int64_t p, double* Fc) {
  int64_t node[8];
  double W[8], up[3] = {0, 0, 0}, gr[2][3] = {{0, 0, 0}, {0, 0, 0}};
  orc_interp_weights(xp, P->nx, P->ny, P->nz, node, W);
  for (int k = 0; k < 8; k++) {
    double uc[3], grad[6];
    orc_node_fields(P, f, node[k], uc, grad);
    for (int a = 0; a < 3; a++) {
      up[a] += W[k] * uc[a];
      for (int c = 0; c < 2; c++) gr[c][a] += W[k] * grad[3 * c + a];
    }
  }
  double R[4] = {0, 0, 0, 0};
  if (P->kT > 0.0) {
    orc_site_normals(P->seed, step, p, 1, 1, R);
    for (int a = 0; a < 3; a++) R[a] *= sqrt(2.0 * P->kT * P->gamma);
  }
  for (int a = 0; a < 3; a++)
    Fc[a] = -P->gamma * (vp[a] - up[a]) - (P->kappa[type][0] * gr[0][a] + P->kappa[type][1] * gr[1][a]) + R[a];
}

void orc_particle_force_at(const orc_params* P, int64_t step, const double* f, int64_t np, const double* x,
                           const double* v, const int32_t* type, int64_t site, double* gP) {
  gP[0] = gP[1] = gP[2] = 0.0;
  for (int64_t p = 0; p < np; p++) {
    int64_t node[8];
    double W[8];
    orc_interp_weights(&x[3 * p], P->nx, P->ny, P->nz, node, W);
    for (int k = 0; k < 8; k++) {
      if (node[k] != site) continue;
      double Fc[3];
      orc_coupling_force_one(P, step, f, &x[3 * p], &v[3 * p], type ? type[p] : 0, p, Fc);
      for (int a = 0; a < 3; a++) gP[a] -= W[k] * Fc[a];
    }
  }
}

int orc_site_collide(const orc_params* P, int64_t step, const double* f, int64_t site,
                     const double* gP, double* out) {
  if (check_params(P) != ORC_OK) return ORC_EINVAL;
  int64_t N = nsites(P);
  int x, y, z;
  coords_of(P, site, &x, &y, &z);
  double fin[2 * ORC_Q], rho[2], Ns[2][3], gsc[6];
  for (int c = 0; c < 2; c++) {
    rho[c] = 0.0;
    for (int i = 0; i < ORC_Q; i++) {
      fin[c * ORC_Q + i] = f[((int64_t)c * ORC_Q + i) * N + site];
      rho[c] += fin[c * ORC_Q + i];
    }
    for (int a = 0; a < 3; a++) Ns[c][a] = 0.0;
    for (int i = 1; i < ORC_Q; i++) {
      int64_t s2 = site_of(P, x + C[i][0], y + C[i][1], z + C[i][2]);
      double r = 0.0;
      for (int q = 0; q < ORC_Q; q++) r += f[((int64_t)c * ORC_Q + q) * N + s2];
      for (int a = 0; a < 3; a++) Ns[c][a] += Wt(i) * r * C[i][a];
    }
  }
  for (int c = 0; c < 2; c++)
    for (int a = 0; a < 3; a++) gsc[3 * c + a] = -rho[c] * (P->G[c][0] * Ns[0][a] + P->G[c][1] * Ns[1][a]);
  basis_init();
  collide_site(P, step, site, fin, gsc, gP, NULL, out);
  return ORC_OK;
}

int orc_step(const orc_params* P, int64_t step, double* f, int64_t np, double* x, double* v,
             double* F, double* Fc, const int32_t* type, int64_t nbonds, const int32_t* bonds,
             double* red) {
  if (check_params(P) != ORC_OK) return ORC_EINVAL;
  int64_t N = nsites(P);
  int status = ORC_OK;
  double* rho = malloc(sizeof(double) * 2 * N);
  double* j = malloc(sizeof(double) * 3 * N);
  double* Ns = malloc(sizeof(double) * 6 * N);
  double* gsc = malloc(sizeof(double) * 6 * N);
  double* uc = malloc(sizeof(double) * 3 * N);
  double* gP = calloc(3 * N, sizeof(double));
  double* gfs = calloc(6 * N, sizeof(double));
  double* back = calloc(3 * (np > 0 ? np : 1), sizeof(double));
  double* fnew = malloc(sizeof(double) * 2 * ORC_Q * N);

  /* S1 */
  orc_moments(P, f, rho, j, NULL);
  double sr[2] = {0, 0}, sj[3] = {0, 0, 0};
  for (int64_t s = 0; s < N; s++) {
    for (int c = 0; c < 2; c++) {
      double r = rho[c * N + s];
      sr[c] += r;
      if (!(r > 0.0) || !isfinite(r)) status = ORC_EUNSTABLE;
    }
    for (int a = 0; a < 3; a++) {
      sj[a] += j[a * N + s];
      if (!isfinite(j[a * N + s])) status = ORC_EUNSTABLE;
    }
  }
  if (red) {
    red[0] = sr[0]; red[1] = sr[1];
    red[2] = sj[0]; red[3] = sj[1]; red[4] = sj[2];
  }
  /* S2 */
  orc_neighbour_sums(P, rho, Ns);
  for (int c = 0; c < 2; c++)
    for (int a = 0; a < 3; a++)
#pragma omp parallel for schedule(static)
      for (int64_t s = 0; s < N; s++)
        gsc[((int64_t)c * 3 + a) * N + s] =
            -rho[c * N + s] * (P->G[c][0] * Ns[(0 * 3 + a) * N + s] + P->G[c][1] * Ns[(1 * 3 + a) * N + s]);
  /* S3 */
  for (int a = 0; a < 3; a++)
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; s++)
      uc[a * N + s] = (j[a * N + s] + 0.5 * (gsc[(0 * 3 + a) * N + s] + gsc[(1 * 3 + a) * N + s])) /
                      (rho[s] + rho[N + s]);
  /* S4 */
  double L[3] = {P->nx, P->ny, P->nz};
  for (int64_t p = 0; p < np; p++) {
    double m = P->mass[type ? type[p] : 0];
    for (int a = 0; a < 3; a++) {
      v[3 * p + a] += 0.5 * F[3 * p + a] / m;
      x[3 * p + a] = wrap(x[3 * p + a] + v[3 * p + a], L[a]);
    }
  }
  /* S5 */
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; p++) {
    int t = type ? type[p] : 0;
    int64_t node[8];
    double W[8], up[3] = {0, 0, 0}, gr[2][3] = {{0, 0, 0}, {0, 0, 0}};
    orc_interp_weights(&x[3 * p], P->nx, P->ny, P->nz, node, W);
    for (int k = 0; k < 8; k++)
      for (int a = 0; a < 3; a++) {
        up[a] += W[k] * uc[a * N + node[k]];
        for (int c = 0; c < 2; c++) gr[c][a] += W[k] * Ns[((int64_t)c * 3 + a) * N + node[k]] / CS2;
      }
    double R[4] = {0, 0, 0, 0};
    if (P->kT > 0.0) {
      orc_site_normals(P->seed, step, p, 1, 1, R);
      for (int a = 0; a < 3; a++) R[a] *= sqrt(2.0 * P->kT * P->gamma);
    }
    for (int a = 0; a < 3; a++)
      Fc[3 * p + a] = -P->gamma * (v[3 * p + a] - up[a]) -
                      (P->kappa[t][0] * gr[0][a] + P->kappa[t][1] * gr[1][a]) + R[a];
  }
  /* S6: the interpolated coupling force goes back through the same
     weights */
  for (int64_t p = 0; p < np; p++) {
    int64_t node[8];
    double W[8];
    orc_interp_weights(&x[3 * p], P->nx, P->ny, P->nz, node, W);
    for (int k = 0; k < 8; k++)
      for (int a = 0; a < 3; a++) gP[a * N + node[k]] -= W[k] * Fc[3 * p + a];
  }
  /* S5b: fluid solvation force at step n's densities; the particle gets
     back what it gave, so Fc becomes the total force from the fluid */
  orc_solvation_fluid_force(P, rho, np, x, type, gfs, back);
  for (int64_t p = 0; p < 3 * np; p++) Fc[p] += back[p];
  if (np > 0) {
    if (orc_conservative_forces(P, np, x, type, nbonds, bonds, F) != ORC_OK) status = ORC_EUNSTABLE;
    for (int64_t p = 0; p < 3 * np; p++) F[p] += Fc[p];
  }
  /* S7 + S8 (streaming is a permutation: every site writes its own
     targets) */
  basis_init();
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; s++) {
    double fin[2 * ORC_Q], out[2 * ORC_Q], gs[6], gp[3], gf[6];
    for (int c = 0; c < 2; c++)
      for (int i = 0; i < ORC_Q; i++) fin[c * ORC_Q + i] = f[((int64_t)c * ORC_Q + i) * N + s];
    for (int q = 0; q < 6; q++) gs[q] = gsc[(int64_t)q * N + s];
    for (int a = 0; a < 3; a++) gp[a] = gP[a * N + s];
    for (int q = 0; q < 6; q++) gf[q] = gfs[(int64_t)q * N + s];
    collide_site(P, step, s, fin, gs, gp, gf, out);
    int xx, yy, zz;
    coords_of(P, s, &xx, &yy, &zz);
    for (int c = 0; c < 2; c++)
      for (int i = 0; i < ORC_Q; i++)
        fnew[((int64_t)c * ORC_Q + i) * N + site_of(P, xx + C[i][0], yy + C[i][1], zz + C[i][2])] =
            out[c * ORC_Q + i];
  }
  memcpy(f, fnew, sizeof(double) * 2 * ORC_Q * N);
  /* S9 */
  for (int64_t p = 0; p < np; p++) {
    double m = P->mass[type ? type[p] : 0];
    for (int a = 0; a < 3; a++) {
      v[3 * p + a] += 0.5 * F[3 * p + a] / m;
      if (!isfinite(x[3 * p + a]) || !isfinite(v[3 * p + a])) status = ORC_EUNSTABLE;
    }
  }
  free(rho); free(j); free(Ns); free(gsc); free(uc); free(gP); free(gfs); free(back); free(fnew);
  return status;
}
