/*
 * lbmd -- two-component Shan-Chen lattice Boltzmann fluid coupled to
 * off-lattice point particles, on one AMD MI355X (gfx950).
 *
 * Method: Sega, Sbragaglia, Kantorovich, Ivanov, arXiv 1306.0788.
 *   fluid      Sec. 2 (Eqs. SCforce, LBMIX) and the Appendix (Eqs. feq,
 *              weights, velo, collis, MODES, momentum_definition and the
 *              forcing source term), D3Q19, periodic box, BGK relaxation
 *              (every non-conserved mode relaxes with -1/tau);
 *   particles  Sec. 2 (Eqs. NEWTON and solvation_kappa): friction against
 *              the trilinearly interpolated fluid velocity, solvation force
 *              -sum_zeta kappa_zeta grad rho_zeta, random force of variance
 *              2 kT gamma, and the opposite force spread back onto the 8
 *              surrounding nodes so that total momentum is conserved.
 *
 * Units: lattice spacing 1, time step 1 (the paper's tau is the time step;
 * here tau[] is the BGK relaxation time of each component).
 *
 * Layouts (all host arrays are float64, C order):
 *   site index   s = (z*ny + y)*nx + x, x fastest; N = nx*ny*nz
 *   densities    [2][N]            component A then B
 *   velocity     [3][N]            u_c = (j + g_SC/2)/rho, the velocity the
 *                                  particles see (Appendix, u definition)
 *   populations  [2][19][N]        post-streaming populations f_zeta,i(s) in
 *                                  the velocity order: 0 rest; 1..6 = +x,-x,
 *                                  +y,-y,+z,-z; 7..18 = (+,+,0),(-,-,0),
 *                                  (+,-,0),(-,+,0),(+,0,+),(-,0,-),(+,0,-),
 *                                  (-,0,+),(0,+,+),(0,-,-),(0,+,-),(0,-,+)
 *   particles    [n][3]            positions in [0,L) per axis, velocities,
 *                                  forces
 *
 * Ownership: the library owns all device memory it allocates (hipMalloc).
 * Host arrays passed in are copied before the call returns; the caller keeps
 * them.  Output arrays belong to the caller.
 *
 * Errors: every call returns LBMD_OK (0) or a negative code.  Parameter
 * errors are reported synchronously and leave the handle unchanged.  A
 * numerical failure (a density <= 0 or a non-finite density, momentum or
 * particle quantity -- Sec. 3: negative densities mean failure of the
 * Shan-Chen scheme) is latched on the device and returned as
 * LBMD_EUNSTABLE by the next lbmd_sync / lbmd_get_* / lbmd_reductions call
 * (and by lbmd_step when check_every > 0); lbmd_last_error names the first
 * failing step.  Once latched, the state stays readable but further
 * lbmd_step calls return LBMD_ESTATE.
 *
 * Threading: one handle = one HIP stream; calls on one handle must not
 * overlap.  Different handles are independent.
 */
#ifndef LBMD_H
#define LBMD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbmd_ctx* lbmd_handle;

#define LBMD_OK 0
#define LBMD_EINVAL (-1)    /* invalid argument                         */
#define LBMD_ENOMEM (-2)    /* device allocation failed                 */
#define LBMD_EDEVICE (-3)   /* HIP runtime error                        */
#define LBMD_EUNSTABLE (-4) /* numerical failure latched on the device  */
#define LBMD_ESTATE (-5)    /* call not valid in the handle's state     */

/* storage precision of the populations.  FP64 and FP32 store f and compute
   in the same type.  FP16DEV and BF16DEV store the deviation f_i - w_i rho0
   from the rest equilibrium of density rho0 (same rho0 for both components)
   as IEEE binary16 or bfloat16 and do all arithmetic, the density field and
   the particle coupling in FP32; rounding the stored deviation is not
   mass-conserving (the drift is visible in lbmd_reductions).  Global sums
   are FP64 in every mode. */
#define LBMD_FP64 0
#define LBMD_FP32 1
#define LBMD_FP16DEV 2
#define LBMD_BF16DEV 3

/* forcing scheme */
#define LBMD_FORCE_PAPER 0 /* Appendix forcing source term with the half-force
                              barycentric velocity; needs tau[0] == tau[1]   */
#define LBMD_FORCE_SHIFT 1 /* Shan-Chen velocity shift of the equilibrium
                              velocity (u' + tau_zeta g_zeta / rho_zeta); kT
                              must be 0                                       */

/* fluid kernel organisation (same results up to rounding order) */
#define LBMD_KERNEL_FUSED 0   /* one pass: density halo in LDS + collide +
                                 stream, then a sparse re-collision of the
                                 nodes the particles touch (best with few
                                 particles)                                   */
#define LBMD_KERNEL_TWOPASS 1 /* a streaming density pass (density field,
                                 momentum at the touched nodes), then collide +
                                 stream with the particle force applied
                                 in-line                                      */
#define LBMD_KERNEL_AUTO 2    /* fused with fewer than one touched node per
                                 2,048 sites; otherwise (and always with MRT) push
                                 for a deterministic fluid in FP32 or FP64,
                                 two-pass with thermal noise or on 16-bit
                                 storage                                     */
#define LBMD_KERNEL_PUSH 3    /* one pass over the populations per step: the
                                 collide + stream pass also accumulates the
                                 next step's densities and momentum of every
                                 site from the values it writes (the pulled
                                 sums of step n+1, Eq. LBMIX), which the next
                                 step's Shan-Chen force and particle coupling
                                 read; the particle force is applied in-line.
                                 Keeps a [3][5][N] moment field.              */

/* lbmd_get_fields masks; outputs are concatenated in this order */
#define LBMD_RHO 1u /* [2][N] */
#define LBMD_U 2u   /* [3][N] */
#define LBMD_POP 4u /* [2][19][N] */

/* pair potentials for lbmd_set_pair_potential */
#define LBMD_PAIR_WCA 0  /* params {sigma, eps}: 4 eps[(s/r)^12-(s/r)^6]+eps,
                            r < 2^(1/6) sigma                                 */
#define LBMD_PAIR_DH 1   /* params {kappa_D, r_c, l_B}: q_i q_j l_B e^{-kappa r}
                            / r, r < r_c                                       */
#define LBMD_BOND_FENE 2 /* params {k, R0}: -k R0^2/2 ln(1-(r/R0)^2) on bonds */

#define LBMD_MAX_TYPES 8

typedef struct {
  int32_t nx, ny, nz;  /* periodic lattice, each >= 1                       */
  int32_t precision;   /* LBMD_FP64, _FP32, _FP16DEV or _BF16DEV            */
  int32_t forcing;     /* LBMD_FORCE_PAPER or LBMD_FORCE_SHIFT              */
  int32_t kernel;      /* LBMD_KERNEL_FUSED, _TWOPASS or _AUTO              */
  double tau[2];       /* BGK relaxation time per component, > 1/2          */
  double G[2][2];      /* coupling g_{zeta zeta'} of the Shan-Chen force
                          (Sec. 2, Eq. SCforce) with psi = rho; G[0][1] ==
                          G[1][0] conserves momentum                         */
  double gamma;        /* particle friction (Eq. NEWTON)                    */
  double kappa[2];     /* solvation kappa_A, kappa_B of particle type 0
                          (Eq. solvation_kappa)                             */
  double mass;         /* particle mass of type 0 (> 0)                     */
  double kT;           /* thermal energy; 0 = deterministic                 */
  uint64_t seed;       /* Philox4x32-10 key for fluid and particle noise    */
  int32_t check_every; /* lbmd_step polls the status word every this many
                          steps (0 = never; errors surface at sync/get)     */
  int32_t reserved;    /* must be 0                                         */
  double rho0;         /* reference density of the deviation storage (> 0,
                          finite) for FP16DEV / BF16DEV; ignored otherwise  */
} lbmd_params;

/* Create a simulation.  rho_init: host [2][N] initial densities, or NULL for
   1.0 everywhere; the fluid starts at rest, f = w_i rho_zeta (Appendix,
   Eq. feq with u = 0).  hip_stream: a hipStream_t to run on (e.g. torch's
   current stream), or NULL for a stream owned by the library.  On success
   *out receives the handle.  Errors: LBMD_EINVAL (bad parameters, tau <= 1/2,
   unequal tau with LBMD_FORCE_PAPER, kT > 0 with LBMD_FORCE_SHIFT, kT < 0),
   LBMD_ENOMEM, LBMD_EDEVICE. */
int lbmd_create(const lbmd_params* p, const double* rho_init, void* hip_stream, lbmd_handle* out);

/* Free every device allocation of the handle (waits for its stream). */
int lbmd_destroy(lbmd_handle h);

/* Replace the particles (Sec. 2, Eq. NEWTON).  pos: host [n][3] (wrapped into
   the box); vel: host [n][3] or NULL (zero); type: host [n] in [0, ntypes)
   or NULL (type 0).  Forces from the previous step are reset to zero.
   n = 0 removes all particles.  Errors: LBMD_EINVAL (non-finite values, bad
   type), LBMD_ENOMEM. */
int lbmd_set_particles(lbmd_handle h, int64_t n, const double* pos, const double* vel,
                       const int32_t* type);

/* Per-type solvation constants kappa [ntypes][2] (Eq. solvation_kappa), masses
   [ntypes] (> 0) and charges [ntypes] (NULL = 0), ntypes <= LBMD_MAX_TYPES.
   Type 0 initially takes kappa/mass from lbmd_params. */
int lbmd_set_particle_types(lbmd_handle h, int32_t ntypes, const double* kappa, const double* mass,
                            const double* charge);

/* Multiple-relaxation-time collision (Appendix, Eqs. collis and MODES; the
   forcing source term in its general form with lambda_M, lambda_s,
   lambda_b): enable != 0 relaxes the momentum modes of each component with
   lambda_mom, the bulk mode with lambda_bulk, the five shear modes with
   lambda_shear and the nine kinetic modes with lambda_ghost (each in
   (-2, 0); BGK is every eigenvalue -1/tau), in place of the BGK relaxation
   with tau[].  Fluctuations (kT > 0) take each mode's own eigenvalue.  Needs
   LBMD_FORCE_PAPER; the step then uses the two-pass or the push
   organisation (LBMD_KERNEL_AUTO: push without noise in FP32 or FP64,
   two-pass with noise or on 16-bit storage; a
   kernel explicitly set to LBMD_KERNEL_FUSED is refused).  enable = 0
   returns to BGK.  Errors: LBMD_EINVAL, LBMD_ESTATE (in a batch). */
int lbmd_set_mrt(lbmd_handle h, int32_t enable, double lambda_bulk, double lambda_shear, double lambda_mom,
                 double lambda_ghost);

/* Fluid solvation force (Sec. 2, Eq. solvation_lambda): lambda [ntypes][2]
   = (lambda_A, lambda_B) per particle type (types >= ntypes get 0; ntypes =
   0 switches the force off).  Each particle acts on the 8 vertices r of its
   lattice cell with -lambda_zeta rho_zeta(r) sum_j c_j/|c_j|^2 over the
   D3Q19 links j with (x_p - r) . c_j > 0, and receives the opposite of the
   total, so momentum is conserved; lbmd_get_particles' fcoup then includes
   that return.  Allocates 8 values per site on first use.  Errors:
   LBMD_EINVAL, LBMD_ENOMEM, LBMD_EDEVICE, LBMD_ESTATE (in a batch). */
int lbmd_set_solvation_lambda(lbmd_handle h, int32_t ntypes, const double* lambda);

/* Switch a conservative particle interaction on (params != NULL) or off
   (params == NULL).  The WCA form is the one the paper uses for excluded
   volume, with the usual +eps shift; the screened Debye-Hueckel form is the
   paper's short-range electrostatics.  Cut-offs must be below half the
   smallest box edge.  Errors: LBMD_EINVAL. */
int lbmd_set_pair_potential(lbmd_handle h, int32_t kind, const double* params);

/* FENE bonds: pairs [nb][2] of particle indices (host, copied).  Each
   particle may take part in at most 8 bonds.  Errors: LBMD_EINVAL. */
int lbmd_set_bonds(lbmd_handle h, int64_t nb, const int32_t* pairs);

/* Enqueue nsteps time steps on the handle's stream and return (asynchronous
   unless check_every > 0).  Each step: particle half kick and drift, fluid
   moments and Shan-Chen force, coupling forces at the new positions, the
   opposite force spread onto the nodes, collision with forcing (and noise if
   kT > 0), streaming, second half kick.  Errors: LBMD_ESTATE after a
   latched failure, LBMD_EUNSTABLE when a poll finds one, LBMD_EDEVICE. */
int lbmd_step(lbmd_handle h, int64_t nsteps);

/* Wait for the handle's stream; returns the latched status. */
int lbmd_sync(lbmd_handle h);

/* Write the fields selected by mask (LBMD_RHO | LBMD_U | LBMD_POP) of the
   current state, concatenated in that order, as float64 into out: a host
   pointer (out_is_device = 0; the call waits) or a device pointer on the same
   device (out_is_device = 1; enqueued on the handle's stream).  u needs the
   Shan-Chen force and so reads the density halo.  Returns the latched
   status. */
int lbmd_get_fields(lbmd_handle h, uint32_t mask, double* out, int32_t out_is_device);

/* lbmd_get_fields without any allocation, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc): same arguments, same results.  Its
   device intermediates -- the density field the export reads for the
   Shan-Chen force of u, and for a host out the float64 staging of the
   fields -- live in a static array of LBMD_NOALLOC_SCRATCH_BYTES that the
   library holds on each GPU it runs on until the process ends; the call
   makes no hipMalloc or hipFree.  Requests needing more (2 N arithmetic
   values for the density field, rounded up to 256 bytes, plus 8 bytes per
   output value for a host out) fail with LBMD_EINVAL.  Every call on one
   GPU uses that GPU's array: calls that overlap on one GPU (from different
   handles or threads) race and must be serialised by the caller. */
#define LBMD_NOALLOC_SCRATCH_BYTES (64u << 20)
int lbmd_get_fields_noalloc(lbmd_handle h, uint32_t mask, double* out, int32_t out_is_device);

/* Host copies of the particle state (any pointer may be NULL): positions,
   velocities, total forces F(n) and their coupling part (friction +
   solvation + random), each [n][3].  Waits.  Returns the latched status. */
int lbmd_get_particles(lbmd_handle h, double* pos, double* vel, double* force, double* fcoup);

/* Replace the populations with host [2][19][N] post-streaming values
   (resume, fault injection).  Errors: LBMD_EINVAL on a NULL pointer. */
int lbmd_set_populations(lbmd_handle h, const double* pop);

/* Checkpoint and resume.  The dynamic state of a simulation is its
   post-streaming populations (Appendix: f_i(r, t) is the whole fluid state),
   its particles' positions, velocities, total and coupling forces (velocity
   Verlet needs F(n) to take step n) and types, and the step index, from which
   every random draw of a step follows (the Philox counter holds the step:
   Appendix, Eq. MODES noise; Sec. 2, Eq. NEWTON random force).  Parameters,
   particle types, potentials, bonds, MRT, lambda and tiling belong to the
   handle and are not part of the state.

   lbmd_get_state writes the state into the host buffer buf as an opaque,
   versioned blob (the populations in their stored form, so a resume is exact
   in every precision).  With buf == NULL it only sets *bytes to the size
   needed.  If *bytes is too small it sets *bytes to the size needed and
   returns LBMD_EINVAL.  On success *bytes receives the size written.  Waits
   for the stream.  Returns the latched status (the state is written either
   way).

   lbmd_set_state replaces the handle's state with a blob from lbmd_get_state
   of a handle with the same lattice size, precision (and rho0 for deviation
   storage); a different particle count is applied as by lbmd_set_particles
   (bonds then dropped).  The step index, the device status latch and the
   sums are reset to the blob's step; captured graphs are dropped.  Taking K
   steps after a restore gives the same result as taking them on the handle
   the state came from (bit for bit where the step is deterministic; the
   spread's float atomics can change the order of additions).  Errors:
   LBMD_EINVAL (NULL, foreign or truncated blob, size or precision mismatch,
   bad type), LBMD_ESTATE (in a batch), LBMD_ENOMEM, LBMD_EDEVICE. */
int lbmd_get_state(lbmd_handle h, void* buf, size_t* bytes);
int lbmd_set_state(lbmd_handle h, const void* buf, size_t bytes);

/* Conservation sums of the state at the start of the most recent step, in
   float64: out[0..1] = sum rho_A, sum rho_B; out[2..4] = raw fluid momentum
   sum_zeta,i f c_i; out[5..7] = sum_p (m v_p + F_coup,p / 2).  With a
   symmetric G and a force-free box out[2..4] + out[5..7] is conserved
   exactly (up to rounding).  *step_out (may be NULL) receives the index of
   that step, -1 before the first step.  Waits.  Returns the latched status. */
int lbmd_reductions(lbmd_handle h, double* out, int64_t* step_out);

/* Number of steps taken so far. */
int64_t lbmd_get_step(lbmd_handle h);

/* Message of the last error on the handle (static storage of the handle). */
const char* lbmd_last_error(lbmd_handle h);

/* Launch configuration of the z-march fluid kernels: rows per block (tile_y
   in {2, 4, 8, 16}), z planes marched per block (tile_z >= 1), and flags:
   LBMD_TILE_HOLD keeps the next plane's populations in registers in the
   fused kernel (else they are read again from cache), LBMD_TILE_XCD orders
   the blocks so that tiles sharing border rows run on the same XCD,
   LBMD_TILE_NT marks the population stores non-temporal.  Same results;
   only speed changes.  Without this call the library uses 4 rows x 16
   planes (HOLD | NT) for the fused organisation and 16 rows x 64 planes
   (XCD | NT) for the two-pass one.  Errors: LBMD_EINVAL. */
#define LBMD_TILE_HOLD 1
#define LBMD_TILE_XCD 2
#define LBMD_TILE_NT 4
int lbmd_set_tiling(lbmd_handle h, int32_t tile_y, int32_t tile_z, int32_t flags);

/* Timing of the collide-stream kernel (the fused kernel, or the collide
   kernel of the two-pass organisation): enable = 1 clears the record and
   brackets every later launch with HIP events on the handle's stream;
   enable = 0 stops.  Either way *total_ms (may be NULL) receives the summed
   duration of the recorded launches and *launches (may be NULL) their
   number.  Waits.  Errors: LBMD_EDEVICE. */
int lbmd_kernel_timing(lbmd_handle h, int32_t enable, double* total_ms, int64_t* launches);

/* Memory ceiling of the collide-stream access pattern: times reps launches
   of a pass that reads every site's 38 pulled populations (in the handle's
   storage type) and writes them unchanged, with no arithmetic, one site per
   thread; *ms receives the average duration of one pass.  Only the scratch
   population buffer (the destination of the next step) is written: the
   state is unchanged.  Waits.  Errors: LBMD_EINVAL (reps < 1, NULL ms),
   LBMD_ESTATE (attached to a batch), LBMD_EDEVICE. */
int lbmd_stream_ceiling(lbmd_handle h, int32_t reps, double* ms);

/* Organisation the next step will use: LBMD_KERNEL_FUSED or
   LBMD_KERNEL_TWOPASS or LBMD_KERNEL_PUSH (resolves LBMD_KERNEL_AUTO);
   negative on a NULL handle. */
int lbmd_organisation(lbmd_handle h);

/* Replay of captured step sequences (default off).  With enable != 0,
   lbmd_step advances two steps at a time by launching a HIP graph captured
   from the step's own launch sequence (one graph per ping-pong parity,
   captured on first use, dropped when particles, types, potentials, bonds
   or the tiling change); an odd remainder, and any step while kernel
   timing is on, is launched kernel by kernel.  Results are identical to
   the eager launches.  Waits for the handle's stream.  The caller's stream
   must not be under capture by someone else.  Errors: LBMD_EINVAL,
   LBMD_EDEVICE. */
int lbmd_set_graph(lbmd_handle h, int32_t enable);

/* Tiling autotuner.  Times the fluid passes of the organisation the next
   step would use, reps times per candidate tiling (rows per tile, planes per
   z chunk, HOLD and XCD flags; non-temporal stores on) in each of two sweeps
   over the candidates, on the current state without advancing it, and keeps
   the fastest (each candidate timed by the better of its two sweeps) as if
   set by lbmd_set_tiling.
   cache_path (may be NULL): a text file of "nx ny nz precision organisation
   forcing noise tile_y tile_z flags ms" lines; an existing entry for the
   same key is applied without timing, a new result is appended.  chosen
   (may be NULL) receives {tile_y, tile_z, flags}; best_ms (may be NULL) the
   time of one pass pair in ms.  Waits.  Errors: LBMD_EINVAL (reps < 1),
   LBMD_ESTATE (failure latched), LBMD_EDEVICE. */
int lbmd_autotune(lbmd_handle h, int32_t reps, const char* cache_path, int32_t* chosen, double* best_ms);

/* ---- multi-lattice batches (serving many independent simulations) ----

   A batch advances every attached handle by one launch sequence per step:
   six kernels (particle half kick and drift, fused density + collision +
   streaming pass, coupling forces and spread, re-collision of the touched
   nodes, second half kick, FP64 sums) whose blocks walk the lattice tiles,
   particle blocks and touched-node blocks of all attached jobs together, so
   jobs of uneven size share the device; the sequence is captured once in a
   HIP graph and replayed, and jobs join and leave by rewriting the device
   job table.  Each job stops advancing at its own target step or at its own
   numerical failure, without affecting the others; its results are those
   of lbmd_step with the fused organisation (bit for bit without particles;
   with particles up to the order of the float additions of the spread).
   Jobs must be FP32, use LBMD_FORCE_PAPER, have no pair potentials or bonds
   and all have kT > 0 or all kT = 0 (the batch's noise setting). */
typedef struct lbmd_batch_s* lbmd_batch;

/* Create a batch of at most max_jobs slots (1..4096) on the current device.
   noise: 1 for jobs with kT > 0, 0 for deterministic jobs.  hip_stream as
   for lbmd_create.  Errors: LBMD_EINVAL, LBMD_ENOMEM, LBMD_EDEVICE. */
int lbmd_batch_create(int32_t max_jobs, int32_t noise, void* hip_stream, lbmd_batch* out);

/* Detach every job (their handles stay valid) and free the batch. */
int lbmd_batch_destroy(lbmd_batch b);

/* Attach handle h to a free slot (*slot receives it); the batch will advance
   it nsteps steps from its current step.  While attached, calls on h other
   than lbmd_last_error return LBMD_ESTATE.  Errors: LBMD_EINVAL (the job
   does not meet the batch's conditions), LBMD_ESTATE (no free slot, h in a
   batch or latched), LBMD_EDEVICE. */
int lbmd_batch_attach(lbmd_batch b, lbmd_handle h, int64_t nsteps, int32_t* slot);

/* Detach the job in slot (waits for the batch's stream); its handle resumes
   at the step the batch reached.  Errors: LBMD_EINVAL, LBMD_EDEVICE. */
int lbmd_batch_detach(lbmd_batch b, int32_t slot);

/* Enqueue nsteps batch steps (jobs past their target or failed stay put).
   Does not wait.  Errors: LBMD_EINVAL, LBMD_EDEVICE. */
int lbmd_batch_step(lbmd_batch b, int64_t nsteps);

/* Wait for the batch's stream and report, per slot (arrays of max_jobs):
   steps[s] = the job's step (-1 if empty), state[s] = 0 empty, 1 running,
   2 reached its target, 3 numerical failure (details through lbmd_sync on
   the handle after detaching).  Either array may be NULL. */
int lbmd_batch_poll(lbmd_batch b, int64_t* steps, int32_t* state);

/* Message of the batch's last error. */
const char* lbmd_batch_last_error(lbmd_batch b);

#ifdef __cplusplus
}
#endif
#endif
