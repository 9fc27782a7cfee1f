/*
 * Oracle for the two-component Shan-Chen lattice Boltzmann fluid coupled to
 * off-lattice point particles (Sega, Sbragaglia, Kantorovich, Ivanov,
 * arXiv 1306.0788).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, FP64 CPU statement of
 * what one time step computes.  It is used by the tests, by the package's
 * smoke check and by the benchmark's CPU baseline leg, and by nothing else.
 * It shares no code, header, table or constant with the GPU library: every
 * table below is written out here again on purpose.
 *
 * Units: lattice spacing 1, time step 1 (the paper's tau is the time step).
 * Populations are stored [component][i][z][y][x], x fastest, in the velocity
 * order listed in orc.c (rest, the six axis links, then the twelve diagonal
 * links, opposite pairs adjacent).
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#define ORC_Q 19
#define ORC_MAXTYPES 8

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EUNSTABLE = -4 };
enum { ORC_FORCE_PAPER = 0, ORC_FORCE_SHIFT = 1 };

typedef struct {
  int32_t nx, ny, nz;
  int32_t forcing;        /* ORC_FORCE_PAPER: Appendix forcing source term;
                             ORC_FORCE_SHIFT: Shan-Chen velocity shift      */
  int32_t mrt;            /* 0: every non-conserved mode relaxes with -1/tau
                             1: use lambda_* below (paper's MRT form)       */
  int32_t pad0;
  double tau[2];          /* relaxation time per component (BGK)            */
  double lambda_bulk, lambda_shear, lambda_mom, lambda_ghost; /* if mrt=1   */
  double G[2][2];         /* g_{zeta zeta'} of the Shan-Chen force          */
  double gamma;           /* particle friction                              */
  double kT;              /* thermal energy; 0 => deterministic             */
  uint64_t seed;          /* Philox key                                     */
  int32_t ntypes, pad1;
  double kappa[ORC_MAXTYPES][2]; /* solvation kappa_A, kappa_B per type     */
  double mass[ORC_MAXTYPES];
  double charge[ORC_MAXTYPES];
  int32_t wca_on, fene_on, dh_on, pad2;
  double wca_sigma, wca_eps;
  double fene_k, fene_R0;
  double dh_kappa, dh_rc, dh_lB;
  double lambda_fs[ORC_MAXTYPES][2]; /* fluid solvation lambda_A, lambda_B per
                                        type (Sec. 2, Eq. solvation_lambda)  */
} orc_params;

/* ---- tables and single-site pieces (exposed for the pins) ---- */
void orc_lattice(int32_t* c /*[19][3]*/, double* w /*[19]*/);
void orc_mode_basis(double* e /*[19][19] e[k][i]*/, double* b /*[19]*/);
void orc_equilibrium(double rho, const double* u, double* feq /*[19]*/);
void orc_forcing_term(double lam_mom, double lam_shear, double lam_bulk,
                      const double* u, const double* g, double* dg /*[19]*/);
void orc_philox4x32_10(const uint32_t* ctr /*[4]*/, const uint32_t* key /*[2]*/,
                       uint32_t* out /*[4]*/);
void orc_box_muller(uint32_t a, uint32_t b, double* z0, double* z1);
void orc_site_normals(uint64_t seed, int64_t step, int64_t index, int32_t tag,
                      int32_t nblocks, double* z /*[4*nblocks]*/);
void orc_interp_weights(const double* x, int32_t nx, int32_t ny, int32_t nz,
                        int64_t* node /*[8]*/, double* W /*[8]*/);
double orc_pair_energy(const orc_params* P, int32_t kind, double r, double qq);
double orc_pair_force(const orc_params* P, int32_t kind, double r, double qq);

/* OpenMP threads of the per-site and per-particle loops (results do not
   depend on the count). */
void orc_set_threads(int32_t n);
int32_t orc_get_threads(void);

/* ---- whole-lattice pieces ---- */
/* moments: rho [2][N], j (raw, both components summed) [3][N],
   jc (raw per component) [2][3][N] (may be NULL) */
void orc_moments(const orc_params* P, const double* f, double* rho, double* j,
                 double* jc);
/* neighbour sums N_zeta(r) = sum_i w_i rho_zeta(r+c_i) c_i  -> [2][3][N] */
void orc_neighbour_sums(const orc_params* P, const double* rho, double* Nsum);

/* ---- one full time step ----
 * f     [2][19][N]  post-streaming populations at step n, replaced by n+1
 * x,v   [np][3]     positions / velocities at n, replaced by n+1
 * F     [np][3]     total force at n (input), force at n+1 (output)
 * Fc    [np][3]     coupling part of the force at n+1 (output)
 * red   [5]         sum rho_A, sum rho_B, sum of raw fluid momentum (3) at n
 * bonds [nbonds][2] FENE bonds
 * Returns ORC_OK, ORC_EINVAL or ORC_EUNSTABLE.                              */
int orc_step(const orc_params* P, int64_t step, double* f, int64_t np,
             double* x, double* v, double* F, double* Fc, const int32_t* type,
             int64_t nbonds, const int32_t* bonds, double* red);

/* Initial populations f = w_i rho_zeta(r) (fluid at rest). */
void orc_init_populations(const orc_params* P, const double* rho, double* f);

/* Conservative particle forces only (pair potentials + bonds), all pairs
   with the minimum image convention.  F [np][3] is overwritten. */
int orc_conservative_forces(const orc_params* P, int64_t np, const double* x,
                            const int32_t* type, int64_t nbonds,
                            const int32_t* bonds, double* F);
/* Same, for one particle p only (sampled checks at large sizes). */
int orc_conservative_force_one(const orc_params* P, int64_t np, const double* x,
                               const int32_t* type, int64_t nbonds,
                               const int32_t* bonds, int64_t p, double* Fp);

/* Post-collision (pre-streaming) populations at one site r, from the full
 * post-streaming state f at step n and the particle back-reaction force
 * density gP [3] at r.  Used for sampled comparisons on large lattices.     */
int orc_site_collide(const orc_params* P, int64_t step, const double* f,
                     int64_t site, const double* gP, double* out /*[2][19]*/);
/* Coupling force (friction + solvation + random) on particle p at position
 * xp with velocity vp (after the step's half kick and drift), from the
 * post-streaming state f at step n.                                        */
void orc_coupling_force_one(const orc_params* P, int64_t step, const double* f, const double* xp,
                            const double* vp, int32_t type, int64_t p, double* Fc /*[3]*/);
/* Particle force density at one node: -sum_p W_p(site) F_coup,p over the
 * particles whose 8 nodes include the site (positions/velocities after the
 * half kick and drift).                                                    */
void orc_particle_force_at(const orc_params* P, int64_t step, const double* f, int64_t np,
                           const double* x, const double* v, const int32_t* type, int64_t site,
                           double* gP /*[3]*/);
/* Fluid solvation force (Sec. 2, Eq. solvation_lambda).  Each particle acts
 * on the 8 vertices r of its lattice cell: at r, with d = x_p - r, it adds
 * -lambda_zeta(type) rho_zeta(r) sum_j c_j / |c_j|^2 over the D3Q19 links j
 * whose direction makes an angle in [0, 90) degrees with d (Theta read as
 * 0 < cos <= 1, i.e. d . c_j > 0).  The momentum it gives the fluid is
 * returned to the particle (back [np][3] = minus its total over the 8 nodes
 * and both components).  rho: [2][N]; fs: [2][3][N] is accumulated into.   */
void orc_solvation_fluid_force(const orc_params* P, const double* rho, int64_t np, const double* x,
                               const int32_t* type, double* fs, double* back);
/* u_c and grad rho_zeta at one node (the quantities the particles see).    */
void orc_node_fields(const orc_params* P, const double* f, int64_t site,
                     double* uc /*[3]*/, double* grad /*[2][3]*/);
#endif
