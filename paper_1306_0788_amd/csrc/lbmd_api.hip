// C-ABI entry points of the lbmd library (declared in include/lbmd.h).
// Host-side runtime: validation, device allocation, step sequencing on one
// HIP stream, the device status latch and host transfers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lbmd_internal.h"

using namespace lbmd;

namespace {

int fail(lbmd_ctx* h, int code, const char* msg) {
  if (h) h->err = msg;
  return code;
}

int hip_fail(lbmd_ctx* h, hipError_t e, const char* where) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
  if (h) h->err = buf;
  return e == hipErrorOutOfMemory ? LBMD_ENOMEM : LBMD_EDEVICE;
}

#define HIPCHECK(h, expr)                              \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(h, e_, #expr); \
  } while (0)

template <class T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) return hipSuccess;
  return hipMalloc((void**)p, n * sizeof(T));
}

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

// the populations were replaced from outside a step: derived fields kept
// between steps are stale
void state_changed(lbmd_ctx* h) { h->push_step = -1; }

// moment field of the push organisation and its x-boundary side buffers
// (allocated on first use): R[3][5][N], H[2][tiles_x][2][5][nz][ny]
int ensure_push_field(lbmd_ctx* h) {
  if (h->R && h->H) return LBMD_OK;
  const size_t tiles_x = size_t(h->p.nx + 63) / 64;
  if (!h->R) HIPCHECK(h, hipMalloc(&h->R, size_t(3) * 5 * size_t(h->N) * h->c_bytes));
  if (!h->H) HIPCHECK(h, hipMalloc(&h->H, size_t(2) * tiles_x * 2 * 5 * size_t(h->p.nz) * h->p.ny * h->c_bytes));
  h->push_step = -1;
  return LBMD_OK;
}

// the push organisation's moments of the current step, computed from the
// populations when the field does not hold them
int push_ready(lbmd_ctx* h) {
  if (int rc = ensure_push_field(h)) return rc;
  if (h->push_step != h->step) {
    HIPCHECK(h, push_init(h));
    h->push_step = h->step;
  }
  return LBMD_OK;
}

// drop the captured step sequences (the launch sequence changed)
void graph_invalidate(lbmd_ctx* h) {
  for (int c = 0; c < 2; ++c)
    if (h->gexec[c]) {
      (void)hipGraphExecDestroy(h->gexec[c]);
      h->gexec[c] = nullptr;
    }
}

bool finite_all(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// bytes per stored population
static size_t storage_bytes(int precision) {
  return precision == LBMD_FP64 ? 8 : (precision == LBMD_FP32 ? 4 : 2);
}

int validate(const lbmd_params* p, std::string& why) {
  if (!p) return why = "params is NULL", LBMD_EINVAL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return why = "lattice size must be >= 1", LBMD_EINVAL;
  const double n = double(p->nx) * p->ny * p->nz;
  if (n > 2147483647.0) return why = "lattice has more than 2^31-1 sites", LBMD_EINVAL;
  // kernels address the 19 arrays of a component through one buffer
  // resource (32-bit byte range)
  if (p->precision != LBMD_FP64 && p->precision != LBMD_FP32 && p->precision != LBMD_FP16DEV &&
      p->precision != LBMD_BF16DEV)
    return why = "unknown precision", LBMD_EINVAL;
  if (19.0 * n * double(storage_bytes(p->precision)) >= 4294967296.0)
    return why = "the 19 population arrays of a component must stay below 4 GiB", LBMD_EINVAL;
  if ((p->precision == LBMD_FP16DEV || p->precision == LBMD_BF16DEV) && !(p->rho0 > 0 && std::isfinite(p->rho0)))
    return why = "deviation storage needs a finite rho0 > 0", LBMD_EINVAL;
  if (p->forcing != LBMD_FORCE_PAPER && p->forcing != LBMD_FORCE_SHIFT) return why = "unknown forcing", LBMD_EINVAL;
  if (p->kernel != LBMD_KERNEL_FUSED && p->kernel != LBMD_KERNEL_TWOPASS && p->kernel != LBMD_KERNEL_AUTO &&
      p->kernel != LBMD_KERNEL_PUSH)
    return why = "unknown kernel", LBMD_EINVAL;
  for (int c = 0; c < 2; ++c)
    if (!(p->tau[c] > 0.5) || !std::isfinite(p->tau[c])) return why = "tau must be > 1/2", LBMD_EINVAL;
  if (p->forcing == LBMD_FORCE_PAPER && p->tau[0] != p->tau[1])
    return why = "the paper's forcing needs the same relaxation for both components", LBMD_EINVAL;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      if (!std::isfinite(p->G[a][b])) return why = "G must be finite", LBMD_EINVAL;
  if (!std::isfinite(p->gamma) || p->gamma < 0) return why = "gamma must be finite and >= 0", LBMD_EINVAL;
  if (!std::isfinite(p->kappa[0]) || !std::isfinite(p->kappa[1])) return why = "kappa must be finite", LBMD_EINVAL;
  if (!(p->mass > 0) || !std::isfinite(p->mass)) return why = "mass must be > 0", LBMD_EINVAL;
  if (!(p->kT >= 0) || !std::isfinite(p->kT)) return why = "kT must be finite and >= 0", LBMD_EINVAL;
  if (p->kT > 0 && p->forcing == LBMD_FORCE_SHIFT) return why = "fluctuations need the paper's forcing", LBMD_EINVAL;
  if (p->check_every < 0 || p->reserved != 0) return why = "bad check_every/reserved", LBMD_EINVAL;
  return LBMD_OK;
}

// read and latch the device status (synchronises the stream)
int poll_status(lbmd_ctx* h) {
  if (h->latched) return LBMD_EUNSTABLE;
  uint32_t st = 0;
  long long bad = 0;
  HIPCHECK(h, hipMemcpyAsync(&st, h->status, sizeof st, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipMemcpyAsync(&bad, h->bad_step, sizeof bad, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  if (st) {
    h->latched = true;
    char buf[200];
    snprintf(buf, sizeof buf, "numerical failure at step %lld (%s%s)", bad, (st & 1u) ? "fluid density <= 0 or non-finite" : "",
             (st & 2u) ? ((st & 1u) ? ", non-finite particle state" : "non-finite particle state") : "");
    h->err = buf;
    return LBMD_EUNSTABLE;
  }
  return LBMD_OK;
}

void free_particles(lbmd_ctx* h) {
  dfree(h->x);
  dfree(h->v);
  dfree(h->F);
  dfree(h->Fc);
  dfree(h->Fcons);
  dfree(h->type);
  dfree(h->cell_of);
  dfree(h->rank_of);
  dfree(h->cell_perm);
  dfree(h->xs);
  dfree(h->flag_list);
  dfree(h->red_part);
  h->np_cap = 0;
  h->flag_cap = 0;
  h->red_part_cap = 0;
}

void free_bonds(lbmd_ctx* h) {
  dfree(h->bond_start);
  dfree(h->bond_nbr);
  h->nbonds = 0;
}

// (re)build the cell grid for the current cut-off.  Particles are sorted by
// cell every step whether or not a pair potential is on: the coupling kernel
// then takes them in spatial order, so that neighbouring lanes read and
// update nearby nodes.
int setup_cells(lbmd_ctx* h) {
  dfree(h->cell_count);
  dfree(h->cell_start);
  dfree(h->scan_block);
  h->rcut = 0.0;
  if (h->pair.wca_on) h->rcut = std::max(h->rcut, std::sqrt(h->pair.wca_rc2));
  if (h->pair.dh_on) h->rcut = std::max(h->rcut, h->pair.dh_rc);
  const int L[3] = {h->p.nx, h->p.ny, h->p.nz};
  // cell edge >= the cut-off, and no smaller than half the mean particle
  // spacing (about one particle per 8 cells: few candidates in the 27-cell
  // scan while the scan of the counts stays short; measured against one
  // particle per cell: the bead-chain workload's step 2.43 -> 2.31 ms)
  double edge = h->rcut;
  if (h->np > 0) edge = std::max(edge, 0.5 * std::cbrt(double(h->N) / double(h->np)));
  h->ncells = 1;
  for (int a = 0; a < 3; ++a) {
    int n = edge > 0 ? int(std::floor(L[a] / edge)) : 1;
    h->ncell[a] = n >= 3 ? n : 1;  // fewer than 3 cells would alias neighbours
    h->ncells *= h->ncell[a];
  }
  if (h->np == 0) return LBMD_OK;
  HIPCHECK(h, dalloc(&h->cell_count, h->ncells + 1));
  HIPCHECK(h, dalloc(&h->cell_start, h->ncells + 1));
  HIPCHECK(h, dalloc(&h->scan_block, (h->ncells + 1 + 1023) / 1024 + 1));
  HIPCHECK(h, hipMemsetAsync(h->cell_count, 0, (h->ncells + 1) * sizeof(int32_t), h->stream));
  return LBMD_OK;
}

int ensure_coupling_buffers(lbmd_ctx* h) {
  if (h->mask) return LBMD_OK;
  const size_t words = (h->N + 31) / 32;
  HIPCHECK(h, dalloc(&h->mask, words));
  HIPCHECK(h, hipMemsetAsync(h->mask, 0, words * sizeof(uint32_t), h->stream));
  HIPCHECK(h, hipMalloc(&h->rec, 16 * h->N * h->c_bytes));
  HIPCHECK(h, hipMalloc(&h->gP, 4 * h->N * h->c_bytes));
  HIPCHECK(h, hipMemsetAsync(h->gP, 0, 4 * h->N * h->c_bytes, h->stream));
  HIPCHECK(h, hipMemsetAsync(h->rec, 0, 16 * h->N * h->c_bytes, h->stream));
  return LBMD_OK;
}

int ensure_staging(lbmd_ctx* h, size_t n) {
  if (h->export_cap >= n) return LBMD_OK;
  dfree(h->export_tmp);
  h->export_cap = 0;
  HIPCHECK(h, dalloc(&h->export_tmp, n));
  h->export_cap = n;
  return LBMD_OK;
}

}  // namespace

namespace lbmd {
hipError_t prof_begin(lbmd_ctx* h) {
  if (!h->prof_on) return hipSuccess;
  if (2 * h->prof_n + 2 > h->prof_ev.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      if (hipError_t r = hipEventCreate(&e)) return r;
      h->prof_ev.push_back(e);
    }
  }
  return hipEventRecord(h->prof_ev[2 * h->prof_n], h->stream);
}
hipError_t prof_end(lbmd_ctx* h) {
  if (!h->prof_on) return hipSuccess;
  hipError_t r = hipEventRecord(h->prof_ev[2 * h->prof_n + 1], h->stream);
  h->prof_n += 1;
  return r;
}
}  // namespace lbmd

namespace {

// Launch sequence of one step (see lbmd_step); flips nothing.
int enqueue_step(lbmd_ctx* h) {
  const bool parts = h->np > 0;
  if (parts) {
    HIPCHECK(h, particles_begin(h));
    HIPCHECK(h, particles_mark_sorted(h));
  } else {
    h->red_part_used = 0;
  }
  HIPCHECK(h, fluid_pass_a(h));
  if (parts) {
    HIPCHECK(h, particles_pairs(h));
    HIPCHECK(h, particles_forces(h));
    // the pair forces (side stream, beside the coupling) are joined before
    // the collide-stream pass, which then has the chip to itself
    HIPCHECK(h, particles_join_pairs(h));
  }
  HIPCHECK(h, fluid_pass_b(h));
  if (parts) HIPCHECK(h, particles_end(h));
  HIPCHECK(h, finalize_step(h));
  return LBMD_OK;
}

// Capture two steps from the current ping-pong parity into an executable
// graph.  Every step-dependent quantity is read by the kernels from the
// device step counter, so the graph replays any pair of steps.  The second
// stream (pair forces) joins the capture through its events.
int capture_two_steps(lbmd_ctx* h) {
  const int c0 = h->cur;
  HIPCHECK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  int rc = LBMD_OK;
  for (int k = 0; k < 2 && rc == LBMD_OK; ++k) {
    rc = enqueue_step(h);
    h->cur = 1 - h->cur;
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->stream, &g);
  h->cur = c0;
  if (rc != LBMD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return hip_fail(h, ei, "hipGraphInstantiate");
  h->gexec[c0] = x;
  return LBMD_OK;
}

// Tiling search.  Times the two fluid passes of the current organisation
// (pass a + pass b, the kernels that carry the lattice traffic) for every
// candidate tiling on the current state, without advancing it: outside a
// step the touched-node mask, the node forces and the compact node list are
// empty, so the passes only rewrite the scratch population buffer, the
// density field and the reduction partials.  The fastest tiling is kept
// (lbmd_set_tiling semantics) and, with a cache file, recorded under the key
// (lattice, precision, organisation, forcing, noise); a later call with the
// same key reads it back instead of timing.
int autotune(lbmd_ctx* h, int reps, const char* cache_path, int32_t* chosen, double* best_ms) {
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  const int org = organisation_of(h);
  char key[160];
  snprintf(key, sizeof key, "%d %d %d %d %d %d %d", h->p.nx, h->p.ny, h->p.nz, h->p.precision, org, h->p.forcing,
           h->p.kT > 0 ? 1 : 0);
  auto report = [&](int ty, int tz, int flags, double ms) {
    if (chosen) {
      chosen[0] = ty;
      chosen[1] = tz;
      chosen[2] = flags;
    }
    if (best_ms) *best_ms = ms;
  };
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "r")) {
      char line[256];
      int found = 0, ty = 0, tz = 0, fl = 0;
      double ms = 0;
      const size_t kl = strlen(key);
      while (fgets(line, sizeof line, f))
        if (strncmp(line, key, kl) == 0 && line[kl] == ' ' &&
            sscanf(line + kl, " %d %d %d %lf", &ty, &tz, &fl, &ms) == 4)
          found = 1;  // the last entry for the key wins
      fclose(f);
      if (found && lbmd_set_tiling(h, ty, tz, fl) == LBMD_OK) {
        report(ty, tz, fl, ms);
        return LBMD_OK;
      }
    }
  }
  struct Cand {
    int ty, tz, flags;
  };
  std::vector<Cand> cands;
  const bool fused = org == LBMD_KERNEL_FUSED;
  // short z chunks give a small lattice enough blocks for the chip (32^3 at
  // 4 rows x 16 planes is 16 blocks); long ones spread the three-plane start
  // of a march over more planes on a large lattice
  const int tys_f[] = {2, 4, 8}, tys_t[] = {4, 8, 16};
  const int tzs_f[] = {4, 8, 16, 32}, tzs_t[] = {4, 8, 16, 32, 64, 128};
  for (int a = 0; a < 3; ++a) {
    const int ty = fused ? tys_f[a] : tys_t[a];
    if (ty > std::max(2, h->p.ny) && ty != 2) continue;
    if (org == LBMD_KERNEL_PUSH && ty > push_rows_max(h)) continue;
    const int ntz = fused ? 4 : 6;
    for (int b = 0; b < ntz; ++b) {
      const int tz = std::min(fused ? tzs_f[b] : tzs_t[b], h->p.nz);
      for (int xcd = 0; xcd < 2; ++xcd)
        for (int hold = 0; hold < (fused ? 2 : 1); ++hold) {
          const Cand c{ty, tz, LBMD_TILE_NT | (xcd ? LBMD_TILE_XCD : 0) | (hold ? LBMD_TILE_HOLD : 0)};
          bool dup = false;
          for (const Cand& d : cands) dup = dup || (d.ty == c.ty && d.tz == c.tz && d.flags == c.flags);
          if (!dup) cands.push_back(c);
        }
    }
  }
  if (org == LBMD_KERNEL_PUSH)
    if (int rc = push_ready(h)) return rc;
  const bool prof = h->prof_on;
  h->prof_on = false;
  hipEvent_t e0, e1;
  HIPCHECK(h, hipEventCreate(&e0));
  HIPCHECK(h, hipEventCreate(&e1));
  double best = 1e300;
  Cand win = cands.front();
  int rc = LBMD_OK;
  // two sweeps over the candidates, each candidate's time the smaller of
  // its two, so that neither the order of the candidates nor one disturbed
  // measurement decides between tilings a few percent apart
  std::vector<double> times(cands.size(), 1e300);
  for (int sweep = 0; sweep < 2 && rc == LBMD_OK; ++sweep)
    for (size_t i = 0; i < cands.size(); ++i) {
      const Cand& c = cands[i];
      lbmd_set_tiling(h, c.ty, c.tz, c.flags);
      hipError_t e = fluid_pass_a(h);
      if (e == hipSuccess) e = fluid_pass_b(h);
      if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = fluid_pass_a(h);
        if (e == hipSuccess) e = fluid_pass_b(h);
      }
      if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        rc = hip_fail(h, e, "autotune");
        break;
      }
      times[i] = std::min(times[i], double(ms) / reps);
    }
  for (size_t i = 0; rc == LBMD_OK && i < cands.size(); ++i)
    if (times[i] < best) {
      best = times[i];
      win = cands[i];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->prof_on = prof;
  if (rc != LBMD_OK) return rc;
  lbmd_set_tiling(h, win.ty, win.tz, win.flags);
  report(win.ty, win.tz, win.flags, best);
  if (cache_path)
    if (FILE* f = fopen(cache_path, "a")) {
      fprintf(f, "%s %d %d %d %.6f\n", key, win.ty, win.tz, win.flags, best);
      fclose(f);
    }
  return LBMD_OK;
}

}  // namespace

namespace {
// Device scratch of lbmd_get_fields_noalloc: one array per GPU, part of the
// library's code object, so that the call allocates nothing.  Host code must
// never pass `scratch` itself to a kernel (in host code it is only a handle
// of the symbol): the device address comes from hipGetSymbolAddress, once
// per device, with that device current.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of this handle's GPU's scratch array
int static_scratch(lbmd_ctx* h, void** out) {
  if (h->device < 0 || h->device >= kMaxDevices) return fail(h, LBMD_EDEVICE, "static scratch: device index");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[h->device]) {
    int prev = 0;
    HIPCHECK(h, hipGetDevice(&prev));
    if (prev != h->device) HIPCHECK(h, hipSetDevice(h->device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != h->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(h, e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(h, LBMD_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[h->device] = p;
  }
  *out = g_scratch_ptr[h->device];
  return LBMD_OK;
}
}  // namespace

namespace {
// Checkpoint blob: this header, then the stored populations of the current
// buffer as raw storage words [2][19][N] (pull layout), then the particles'
// x, v, F, F_coup ([n][3] float64 each) and types ([n] int32).
struct StateHeader {
  char magic[8];
  int32_t version, precision;
  int32_t nx, ny, nz, pad;
  int64_t np, step;
  double rho0;
};
constexpr char kStateMagic[8] = {'L', 'B', 'M', 'D', 'S', 'T', 'A', 'T'};
constexpr int32_t kStateVersion = 1;

size_t state_bytes(const lbmd_ctx* h, int64_t np) {
  return sizeof(StateHeader) + size_t(2) * 19 * size_t(h->N) * h->s_bytes + size_t(np) * (4 * 3 * sizeof(double) + sizeof(int32_t));
}
}  // namespace

extern "C" {

int lbmd_create(const lbmd_params* p, const double* rho_init, void* hip_stream, lbmd_handle* out) {
  if (!out) return LBMD_EINVAL;
  *out = nullptr;
  std::string why;
  if (int rc = validate(p, why)) {
    fprintf(stderr, "lbmd_create: %s\n", why.c_str());
    return rc;
  }
  if (rho_init && !finite_all(rho_init, size_t(2) * p->nx * p->ny * p->nz)) return LBMD_EINVAL;
  lbmd_ctx* h = new (std::nothrow) lbmd_ctx();
  if (!h) return LBMD_ENOMEM;
  h->p = *p;
  h->N = int64_t(p->nx) * p->ny * p->nz;
  h->s_bytes = storage_bytes(p->precision);
  h->c_bytes = p->precision == LBMD_FP64 ? 8 : 4;
  h->types.ntypes = 1;
  for (int t = 0; t < LBMD_MAX_TYPES; ++t) {
    h->types.kappa[t][0] = p->kappa[0];
    h->types.kappa[t][1] = p->kappa[1];
    h->types.mass[t] = p->mass;
    h->types.charge[t] = 0.0;
  }
  std::memset(&h->pair, 0, sizeof h->pair);
  auto bail = [&](int rc) {
    lbmd_destroy(h);
    return rc;
  };
  if (hipGetDevice(&h->device) != hipSuccess) return bail(LBMD_EDEVICE);
  if (hip_stream) {
    h->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return bail(LBMD_EDEVICE);
    h->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_sorted, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_pairs, hipEventDisableTiming) != hipSuccess)
    return bail(LBMD_EDEVICE);
  const size_t pop = size_t(2) * 19 * h->N * h->s_bytes;
  for (int b = 0; b < 2; ++b)
    if (hipMalloc(&h->f[b], pop) != hipSuccess) return bail(LBMD_ENOMEM);
  if (hipMalloc(&h->rho, 2 * h->N * h->c_bytes) != hipSuccess) return bail(LBMD_ENOMEM);
  // reduction partials: the largest launch is the two-row fused tiling with
  // one plane per block, or the two-pass collide grid
  const int64_t tiles_x = (p->nx + 63) / 64;
  // partials of the tiled passes (at least 2 rows per tile) and of the flat
  // density pass (512 sites per block)
  h->red_fluid_cap = std::max<int64_t>(tiles_x * ((p->ny + 1) / 2) * p->nz, (h->N + 511) / 512);
  if (dalloc(&h->red_fluid, 5 * h->red_fluid_cap) != hipSuccess) return bail(LBMD_ENOMEM);
  if (dalloc(&h->red_out, 8) != hipSuccess || dalloc(&h->status, 1) != hipSuccess ||
      dalloc(&h->bad_step, 1) != hipSuccess || dalloc(&h->nflag, 1) != hipSuccess ||
      dalloc(&h->step_dev, 1) != hipSuccess)
    return bail(LBMD_ENOMEM);
  const long long never = 0x7fffffffffffffffLL;
  if (hipMemsetAsync(h->red_out, 0, 8 * sizeof(double), h->stream) != hipSuccess ||
      hipMemsetAsync(h->status, 0, sizeof(uint32_t), h->stream) != hipSuccess ||
      hipMemcpyAsync(h->bad_step, &never, sizeof never, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipMemsetAsync(h->nflag, 0, sizeof(int32_t), h->stream) != hipSuccess ||
      hipMemsetAsync(h->step_dev, 0, sizeof(int64_t), h->stream) != hipSuccess)
    return bail(LBMD_EDEVICE);
  double* rho_dev = nullptr;
  if (rho_init) {
    if (dalloc(&rho_dev, 2 * h->N) != hipSuccess) return bail(LBMD_ENOMEM);
    if (hipMemcpyAsync(rho_dev, rho_init, 2 * h->N * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess)
      return bail(LBMD_EDEVICE);
  }
  if (fluid_init(h, rho_dev) != hipSuccess) return bail(LBMD_EDEVICE);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(LBMD_EDEVICE);
  dfree(rho_dev);
  h->tile_y = p->ny >= 8 ? 8 : (p->ny >= 4 ? 4 : 2);
  h->tile_z = std::max(1, std::min(p->nz, 16));
  *out = h;
  return LBMD_OK;
}

int lbmd_destroy(lbmd_handle h) {
  if (!h) return LBMD_EINVAL;
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (int b = 0; b < 2; ++b)
    if (h->f[b]) (void)hipFree(h->f[b]);
  if (h->rho) (void)hipFree(h->rho);
  if (h->R) (void)hipFree(h->R);
  if (h->H) (void)hipFree(h->H);
  if (h->rec) (void)hipFree(h->rec);
  if (h->gP) (void)hipFree(h->gP);
  if (h->gS) (void)hipFree(h->gS);
  dfree(h->mask);
  free_particles(h);
  free_bonds(h);
  dfree(h->cell_count);
  dfree(h->cell_start);
  dfree(h->scan_block);
  dfree(h->red_fluid);
  dfree(h->red_out);
  dfree(h->status);
  dfree(h->bad_step);
  dfree(h->nflag);
  dfree(h->step_dev);
  graph_invalidate(h);
  dfree(h->export_tmp);
  for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
  if (h->side) (void)hipStreamSynchronize(h->side);
  if (h->ev_sorted) (void)hipEventDestroy(h->ev_sorted);
  if (h->ev_pairs) (void)hipEventDestroy(h->ev_pairs);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return LBMD_OK;
}

int lbmd_set_particles(lbmd_handle h, int64_t n, const double* pos, const double* vel, const int32_t* type) {
  if (!h || n < 0 || (n > 0 && !pos)) return fail(h, LBMD_EINVAL, "set_particles: bad arguments");
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  graph_invalidate(h);
  if (n > (int64_t(1) << 28)) return fail(h, LBMD_EINVAL, "set_particles: too many particles");
  if (!finite_all(pos, 3 * n) || (vel && !finite_all(vel, 3 * n)))
    return fail(h, LBMD_EINVAL, "set_particles: non-finite input");
  std::vector<double> x(3 * n), v(3 * n, 0.0);
  std::vector<int32_t> t(n, 0);
  const double L[3] = {double(h->p.nx), double(h->p.ny), double(h->p.nz)};
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      double q = pos[3 * i + a];
      q -= L[a] * std::floor(q / L[a]);
      if (q >= L[a]) q -= L[a];
      if (q < 0) q += L[a];
      x[3 * i + a] = q;
      if (vel) v[3 * i + a] = vel[3 * i + a];
    }
  if (type)
    for (int64_t i = 0; i < n; ++i) {
      if (type[i] < 0 || type[i] >= h->types.ntypes) return fail(h, LBMD_EINVAL, "set_particles: bad type");
      t[i] = type[i];
    }
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  if (n != h->np) free_bonds(h);
  if (n > h->np_cap) {
    free_particles(h);
    HIPCHECK(h, dalloc(&h->x, 3 * n));
    HIPCHECK(h, dalloc(&h->v, 3 * n));
    HIPCHECK(h, dalloc(&h->F, 3 * n));
    HIPCHECK(h, dalloc(&h->Fc, 3 * n));
    HIPCHECK(h, dalloc(&h->Fcons, 3 * n));
    HIPCHECK(h, dalloc(&h->type, n));
    HIPCHECK(h, dalloc(&h->cell_of, n));
    HIPCHECK(h, dalloc(&h->rank_of, n));
    HIPCHECK(h, dalloc(&h->cell_perm, n));
    HIPCHECK(h, dalloc(&h->xs, 4 * n));
    HIPCHECK(h, dalloc(&h->flag_list, 8 * n));
    HIPCHECK(h, dalloc(&h->red_part, 3 * ((n + 255) / 256)));
    h->np_cap = n;
    h->flag_cap = 8 * n;
    h->red_part_cap = (n + 255) / 256;
  }
  const bool regrid = n != h->np;
  h->np = n;
  h->red_part_used = 0;
  if (regrid)
    if (int rc = setup_cells(h)) return rc;
  if (n > 0) {
    if (int rc = ensure_coupling_buffers(h)) return rc;
    HIPCHECK(h, hipMemcpyAsync(h->x, x.data(), 3 * n * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPCHECK(h, hipMemcpyAsync(h->v, v.data(), 3 * n * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPCHECK(h, hipMemcpyAsync(h->type, t.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
    HIPCHECK(h, hipMemsetAsync(h->F, 0, 3 * n * sizeof(double), h->stream));
    HIPCHECK(h, hipMemsetAsync(h->Fc, 0, 3 * n * sizeof(double), h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
  }
  return LBMD_OK;
}

int lbmd_set_particle_types(lbmd_handle h, int32_t ntypes, const double* kappa, const double* mass,
                            const double* charge) {
  if (h && h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  if (h) graph_invalidate(h);
  if (!h || ntypes < 1 || ntypes > LBMD_MAX_TYPES || !kappa || !mass)
    return fail(h, LBMD_EINVAL, "set_particle_types: bad arguments");
  for (int t = 0; t < ntypes; ++t)
    if (!(mass[t] > 0) || !std::isfinite(mass[t]) || !std::isfinite(kappa[2 * t]) || !std::isfinite(kappa[2 * t + 1]) ||
        (charge && !std::isfinite(charge[t])))
      return fail(h, LBMD_EINVAL, "set_particle_types: bad values");
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  h->types.ntypes = ntypes;
  for (int t = 0; t < ntypes; ++t) {
    h->types.kappa[t][0] = kappa[2 * t];
    h->types.kappa[t][1] = kappa[2 * t + 1];
    h->types.mass[t] = mass[t];
    h->types.charge[t] = charge ? charge[t] : 0.0;
  }
  return LBMD_OK;
}

int lbmd_set_mrt(lbmd_handle h, int32_t enable, double lambda_bulk, double lambda_shear, double lambda_mom,
                 double lambda_ghost) {
  if (h && h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  if (!h) return LBMD_EINVAL;
  if (enable) {
    const double l[4] = {lambda_mom, lambda_bulk, lambda_shear, lambda_ghost};
    for (double v : l)
      if (!(v > -2.0 && v < 0.0)) return fail(h, LBMD_EINVAL, "set_mrt: every eigenvalue must lie in (-2, 0)");
    if (h->p.forcing != LBMD_FORCE_PAPER) return fail(h, LBMD_EINVAL, "set_mrt: needs the paper's forcing");
    if (h->p.kernel == LBMD_KERNEL_FUSED) return fail(h, LBMD_EINVAL, "set_mrt: MRT runs in the two-pass or push organisation");
  }
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  graph_invalidate(h);
  h->mrt = enable != 0;
  h->mrt_lam[0] = lambda_mom;
  h->mrt_lam[1] = lambda_bulk;
  h->mrt_lam[2] = lambda_shear;
  h->mrt_lam[3] = lambda_ghost;
  return LBMD_OK;
}

int lbmd_set_solvation_lambda(lbmd_handle h, int32_t ntypes, const double* lambda) {
  if (h && h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  if (!h || ntypes < 0 || ntypes > LBMD_MAX_TYPES || (ntypes > 0 && !lambda))
    return fail(h, LBMD_EINVAL, "set_solvation_lambda: bad arguments");
  for (int t = 0; t < 2 * ntypes; ++t)
    if (!std::isfinite(lambda[t])) return fail(h, LBMD_EINVAL, "set_solvation_lambda: non-finite lambda");
  graph_invalidate(h);
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  int on = 0;
  for (int t = 0; t < LBMD_MAX_TYPES; ++t)
    for (int c = 0; c < 2; ++c) {
      h->types.lambda[t][c] = t < ntypes ? lambda[2 * t + c] : 0.0;
      on |= h->types.lambda[t][c] != 0.0;
    }
  h->types.lambda_on = on;
  if (on && !h->gS) {
    HIPCHECK(h, hipMalloc(&h->gS, 8 * h->N * h->c_bytes));
    HIPCHECK(h, hipMemsetAsync(h->gS, 0, 8 * h->N * h->c_bytes, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
  } else if (!on && h->gS) {
    (void)hipFree(h->gS);
    h->gS = nullptr;
  }
  return LBMD_OK;
}

int lbmd_set_pair_potential(lbmd_handle h, int32_t kind, const double* q) {
  if (h && h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  if (h) graph_invalidate(h);
  if (!h) return LBMD_EINVAL;
  const double half = 0.5 * std::min({h->p.nx, h->p.ny, h->p.nz});
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  switch (kind) {
    case LBMD_PAIR_WCA:
      if (!q) {
        h->pair.wca_on = 0;
        break;
      }
      if (!(q[0] > 0) || !(q[1] >= 0) || !std::isfinite(q[0]) || !std::isfinite(q[1]))
        return fail(h, LBMD_EINVAL, "WCA: sigma > 0, eps >= 0");
      if (std::pow(2.0, 1.0 / 6.0) * q[0] >= half) return fail(h, LBMD_EINVAL, "WCA cut-off >= half the box");
      h->pair.wca_on = 1;
      h->pair.wca_sigma = q[0];
      h->pair.wca_eps = q[1];
      h->pair.wca_rc2 = std::pow(2.0, 1.0 / 3.0) * q[0] * q[0];
      break;
    case LBMD_PAIR_DH:
      if (!q) {
        h->pair.dh_on = 0;
        break;
      }
      if (!(q[0] >= 0) || !(q[1] > 0) || !std::isfinite(q[0]) || !std::isfinite(q[1]) || !std::isfinite(q[2]))
        return fail(h, LBMD_EINVAL, "DH: kappa_D >= 0, r_c > 0");
      if (q[1] >= half) return fail(h, LBMD_EINVAL, "DH cut-off >= half the box");
      h->pair.dh_on = 1;
      h->pair.dh_kappa = q[0];
      h->pair.dh_rc = q[1];
      h->pair.dh_lB = q[2];
      break;
    case LBMD_BOND_FENE:
      if (!q) {
        h->pair.fene_on = 0;
        break;
      }
      if (!(q[0] >= 0) || !(q[1] > 0) || !std::isfinite(q[0]) || !std::isfinite(q[1]))
        return fail(h, LBMD_EINVAL, "FENE: k >= 0, R0 > 0");
      if (q[1] >= half) return fail(h, LBMD_EINVAL, "FENE R0 >= half the box");
      h->pair.fene_on = 1;
      h->pair.fene_k = q[0];
      h->pair.fene_R0 = q[1];
      break;
    default:
      return fail(h, LBMD_EINVAL, "unknown potential kind");
  }
  return setup_cells(h);
}

int lbmd_set_bonds(lbmd_handle h, int64_t nb, const int32_t* pairs) {
  if (h && h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  if (h) graph_invalidate(h);
  if (!h || nb < 0 || (nb > 0 && !pairs)) return fail(h, LBMD_EINVAL, "set_bonds: bad arguments");
  std::vector<int32_t> deg(h->np + 1, 0);
  for (int64_t b = 0; b < nb; ++b) {
    const int32_t i = pairs[2 * b], j = pairs[2 * b + 1];
    if (i < 0 || j < 0 || i >= h->np || j >= h->np || i == j) return fail(h, LBMD_EINVAL, "set_bonds: bad index");
    if (++deg[i] > 8 || ++deg[j] > 8) return fail(h, LBMD_EINVAL, "set_bonds: more than 8 bonds on a particle");
  }
  std::vector<int32_t> start(h->np + 1, 0), nbr(2 * nb);
  for (int64_t i = 0; i < h->np; ++i) start[i + 1] = start[i] + deg[i];
  std::vector<int32_t> fill(start.begin(), start.end() - 1);
  for (int64_t b = 0; b < nb; ++b) {
    const int32_t i = pairs[2 * b], j = pairs[2 * b + 1];
    nbr[fill[i]++] = j;
    nbr[fill[j]++] = i;
  }
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  free_bonds(h);
  if (nb == 0) return LBMD_OK;
  HIPCHECK(h, dalloc(&h->bond_start, h->np + 1));
  HIPCHECK(h, dalloc(&h->bond_nbr, 2 * nb));
  HIPCHECK(h, hipMemcpyAsync(h->bond_start, start.data(), (h->np + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                             h->stream));
  HIPCHECK(h, hipMemcpyAsync(h->bond_nbr, nbr.data(), 2 * nb * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  h->nbonds = nb;
  return LBMD_OK;
}

int lbmd_step(lbmd_handle h, int64_t nsteps) {
  if (!h || nsteps < 0) return fail(h, LBMD_EINVAL, "step: bad arguments");
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  if (h->latched) return fail(h, LBMD_ESTATE, "step: a numerical failure is latched");
  const bool push = organisation_of(h) == LBMD_KERNEL_PUSH;
  int64_t k = 0;
  while (k < nsteps) {
    // the push organisation reads this step's moments from its field
    if (push)
      if (int rc = push_ready(h)) return rc;
    // two steps at a time from a captured graph (the ping-pong parity
    // returns), else one step launched kernel by kernel
    int64_t done = 1;
    if (h->use_graph && !h->prof_on && nsteps - k >= 2) {
      if (!h->gexec[h->cur]) {
        if (int rc = capture_two_steps(h)) return rc;
      }
      HIPCHECK(h, hipGraphLaunch(h->gexec[h->cur], h->stream));
      done = 2;
    } else {
      if (int rc = enqueue_step(h)) return rc;
      h->cur = 1 - h->cur;
    }
    const int64_t before = h->step;
    if (push) h->push_step = h->step + done;
    h->step += done;
    k += done;
    if (h->p.check_every > 0 && h->step / h->p.check_every != before / h->p.check_every)
      if (int rc = poll_status(h)) return rc;
  }
  return LBMD_OK;
}

int lbmd_sync(lbmd_handle h) {
  if (!h) return LBMD_EINVAL;
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  return poll_status(h);
}

int lbmd_get_fields(lbmd_handle h, uint32_t mask, double* out, int32_t out_is_device) {
  if (!h || !out || mask == 0 || (mask & ~(LBMD_RHO | LBMD_U | LBMD_POP)))
    return fail(h, LBMD_EINVAL, "get_fields: bad arguments");
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  size_t n = 0;
  if (mask & LBMD_RHO) n += 2 * h->N;
  if (mask & LBMD_U) n += 3 * h->N;
  if (mask & LBMD_POP) n += 38 * h->N;
  double* dst = out;
  if (!out_is_device) {
    if (int rc = ensure_staging(h, n)) return rc;
    dst = h->export_tmp;
  }
  HIPCHECK(h, fluid_export(h, mask, dst, h->rho));
  if (!out_is_device) {
    HIPCHECK(h, hipMemcpyAsync(out, dst, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
  }
  return out_is_device ? LBMD_OK : poll_status(h);
}

int lbmd_get_fields_noalloc(lbmd_handle h, uint32_t mask, double* out, int32_t out_is_device) {
  if (!h || !out || mask == 0 || (mask & ~(LBMD_RHO | LBMD_U | LBMD_POP)))
    return fail(h, LBMD_EINVAL, "get_fields_noalloc: bad arguments");
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  size_t n = 0;
  if (mask & LBMD_RHO) n += 2 * h->N;
  if (mask & LBMD_U) n += 3 * h->N;
  if (mask & LBMD_POP) n += 38 * h->N;
  // scratch layout: the density field [2][N], then (host output) the float64
  // staging of the fields
  const size_t field = (size_t(2) * h->N * h->c_bytes + 255) & ~size_t(255);
  const size_t need = field + (out_is_device ? 0 : n * sizeof(double));
  if (need > kStaticScratchBytes) {
    char buf[200];
    snprintf(buf, sizeof buf, "get_fields_noalloc: needs %zu bytes of scratch, more than the static %zu", need,
             kStaticScratchBytes);
    return fail(h, LBMD_EINVAL, buf);
  }
  void* base = nullptr;
  if (int rc = static_scratch(h, &base)) return rc;
  double* dst = out_is_device ? out : reinterpret_cast<double*>(static_cast<char*>(base) + field);
  HIPCHECK(h, fluid_export(h, mask, dst, base));
  if (!out_is_device) {
    HIPCHECK(h, hipMemcpyAsync(out, dst, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
  }
  return out_is_device ? LBMD_OK : poll_status(h);
}

int lbmd_get_particles(lbmd_handle h, double* pos, double* vel, double* force, double* fcoup) {
  if (!h) return LBMD_EINVAL;
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  const size_t b = 3 * h->np * sizeof(double);
  if (h->np > 0) {
    if (pos) HIPCHECK(h, hipMemcpyAsync(pos, h->x, b, hipMemcpyDeviceToHost, h->stream));
    if (vel) HIPCHECK(h, hipMemcpyAsync(vel, h->v, b, hipMemcpyDeviceToHost, h->stream));
    if (force) HIPCHECK(h, hipMemcpyAsync(force, h->F, b, hipMemcpyDeviceToHost, h->stream));
    if (fcoup) HIPCHECK(h, hipMemcpyAsync(fcoup, h->Fc, b, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
  }
  return poll_status(h);
}

int lbmd_set_populations(lbmd_handle h, const double* pop) {
  if (!h || !pop) return fail(h, LBMD_EINVAL, "set_populations: NULL");
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  if (int rc = ensure_staging(h, 38 * h->N)) return rc;
  HIPCHECK(h, hipMemcpyAsync(h->export_tmp, pop, 38 * h->N * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(h, fluid_import(h, h->export_tmp));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  state_changed(h);
  return LBMD_OK;
}


int lbmd_get_state(lbmd_handle h, void* buf, size_t* bytes) {
  if (!h || !bytes) return fail(h, LBMD_EINVAL, "get_state: NULL argument");
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  const size_t need = state_bytes(h, h->np);
  if (!buf) {
    *bytes = need;
    return LBMD_OK;
  }
  if (*bytes < need) {
    *bytes = need;
    return fail(h, LBMD_EINVAL, "get_state: buffer too small");
  }
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  StateHeader hd;
  std::memset(&hd, 0, sizeof hd);
  std::memcpy(hd.magic, kStateMagic, sizeof hd.magic);
  hd.version = kStateVersion;
  hd.precision = h->p.precision;
  hd.nx = h->p.nx;
  hd.ny = h->p.ny;
  hd.nz = h->p.nz;
  hd.np = h->np;
  hd.step = h->step;
  hd.rho0 = h->p.rho0;
  char* o = static_cast<char*>(buf);
  std::memcpy(o, &hd, sizeof hd);
  o += sizeof hd;
  const size_t pop = size_t(2) * 19 * size_t(h->N) * h->s_bytes;
  HIPCHECK(h, hipMemcpyAsync(o, h->f[h->cur], pop, hipMemcpyDeviceToHost, h->stream));
  o += pop;
  const size_t vb = 3 * size_t(h->np) * sizeof(double);
  if (h->np > 0) {
    const double* src[4] = {h->x, h->v, h->F, h->Fc};
    for (const double* d : src) {
      HIPCHECK(h, hipMemcpyAsync(o, d, vb, hipMemcpyDeviceToHost, h->stream));
      o += vb;
    }
    HIPCHECK(h, hipMemcpyAsync(o, h->type, size_t(h->np) * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  *bytes = need;
  return poll_status(h);
}

int lbmd_set_state(lbmd_handle h, const void* buf, size_t bytes) {
  if (!h || !buf) return fail(h, LBMD_EINVAL, "set_state: NULL argument");
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  if (bytes < sizeof(StateHeader)) return fail(h, LBMD_EINVAL, "set_state: not a state blob");
  StateHeader hd;
  std::memcpy(&hd, buf, sizeof hd);
  if (std::memcmp(hd.magic, kStateMagic, sizeof hd.magic) != 0 || hd.version != kStateVersion)
    return fail(h, LBMD_EINVAL, "set_state: not a state blob of this version");
  if (hd.nx != h->p.nx || hd.ny != h->p.ny || hd.nz != h->p.nz || hd.precision != h->p.precision)
    return fail(h, LBMD_EINVAL, "set_state: lattice size or precision differs from the handle's");
  if ((h->p.precision == LBMD_FP16DEV || h->p.precision == LBMD_BF16DEV) && hd.rho0 != h->p.rho0)
    return fail(h, LBMD_EINVAL, "set_state: deviation storage with another rho0");
  if (hd.np < 0 || hd.np > (int64_t(1) << 28) || hd.step < 0 || bytes < state_bytes(h, hd.np))
    return fail(h, LBMD_EINVAL, "set_state: truncated or inconsistent blob");
  const char* in = static_cast<const char*>(buf) + sizeof hd;
  const size_t pop = size_t(2) * 19 * size_t(h->N) * h->s_bytes;
  const char* pops = in;
  in += pop;
  const size_t vb = 3 * size_t(hd.np) * sizeof(double);
  const double* x = reinterpret_cast<const double*>(in);
  const double* v = reinterpret_cast<const double*>(in + vb);
  const double* F = reinterpret_cast<const double*>(in + 2 * vb);
  const double* Fc = reinterpret_cast<const double*>(in + 3 * vb);
  const int32_t* type = reinterpret_cast<const int32_t*>(in + 4 * vb);
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  graph_invalidate(h);
  // particles: a different count goes through lbmd_set_particles (which
  // keeps bonds only for an unchanged count); F and F_coup are then restored
  if (hd.np != h->np) {
    const bool was_latched = h->latched;
    h->latched = false;
    const int rc = lbmd_set_particles(h, hd.np, x, v, type);
    h->latched = was_latched;
    if (rc != LBMD_OK) return rc;
  } else if (hd.np > 0) {
    for (int64_t i = 0; i < hd.np; ++i)
      if (type[i] < 0 || type[i] >= h->types.ntypes) return fail(h, LBMD_EINVAL, "set_state: bad particle type");
    HIPCHECK(h, hipMemcpyAsync(h->x, x, vb, hipMemcpyHostToDevice, h->stream));
    HIPCHECK(h, hipMemcpyAsync(h->v, v, vb, hipMemcpyHostToDevice, h->stream));
    HIPCHECK(h, hipMemcpyAsync(h->type, type, size_t(hd.np) * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  }
  if (hd.np > 0) {
    HIPCHECK(h, hipMemcpyAsync(h->F, F, vb, hipMemcpyHostToDevice, h->stream));
    HIPCHECK(h, hipMemcpyAsync(h->Fc, Fc, vb, hipMemcpyHostToDevice, h->stream));
  }
  HIPCHECK(h, hipMemcpyAsync(h->f[h->cur], pops, pop, hipMemcpyHostToDevice, h->stream));
  // step index (host count and the device counter the kernels read), a
  // clear status latch and empty sums
  const long long never = 0x7fffffffffffffffLL;
  const int64_t step = hd.step;
  HIPCHECK(h, hipMemcpyAsync(h->step_dev, &step, sizeof step, hipMemcpyHostToDevice, h->stream));
  HIPCHECK(h, hipMemsetAsync(h->status, 0, sizeof(uint32_t), h->stream));
  HIPCHECK(h, hipMemcpyAsync(h->bad_step, &never, sizeof never, hipMemcpyHostToDevice, h->stream));
  HIPCHECK(h, hipMemsetAsync(h->red_out, 0, 8 * sizeof(double), h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  h->step = step;
  h->latched = false;
  h->err.clear();
  state_changed(h);
  return LBMD_OK;
}

int lbmd_reductions(lbmd_handle h, double* out, int64_t* step_out) {
  if (!h || !out) return LBMD_EINVAL;
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  HIPCHECK(h, hipMemcpyAsync(out, h->red_out, 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  if (step_out) *step_out = h->step - 1;
  return poll_status(h);
}

int64_t lbmd_get_step(lbmd_handle h) { return h ? h->step : -1; }

const char* lbmd_last_error(lbmd_handle h) { return h ? h->err.c_str() : "NULL handle"; }

int lbmd_set_tiling(lbmd_handle h, int32_t tile_y, int32_t tile_z, int32_t flags) {
  if (h && h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  if (!h || !(tile_y == 2 || tile_y == 4 || tile_y == 8 || tile_y == 16) || tile_z < 1 || (flags & ~7))
    return fail(h, LBMD_EINVAL, "set_tiling: tile_y in {2,4,8,16}, tile_z >= 1, flags in 0..7");
  h->tile_y = tile_y;
  h->tile_z = tile_z;
  h->hold = flags & LBMD_TILE_HOLD ? 1 : 0;
  h->xcd = flags & LBMD_TILE_XCD ? 1 : 0;
  h->nt = flags & LBMD_TILE_NT ? 1 : 0;
  h->tiling_set = true;
  h->push_step = -1;  // the push pass clears the face sites of its tiling
  graph_invalidate(h);
  return LBMD_OK;
}

int lbmd_organisation(lbmd_handle h) { return h ? organisation_of(h) : LBMD_EINVAL; }

int lbmd_kernel_timing(lbmd_handle h, int32_t enable, double* total_ms, int64_t* launches) {
  if (!h) return LBMD_EINVAL;
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  double tot = 0.0;
  for (size_t k = 0; k < h->prof_n; ++k) {
    float ms = 0.0f;
    HIPCHECK(h, hipEventElapsedTime(&ms, h->prof_ev[2 * k], h->prof_ev[2 * k + 1]));
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = int64_t(h->prof_n);
  if (enable) h->prof_n = 0;
  h->prof_on = enable != 0;
  return LBMD_OK;
}

int lbmd_stream_ceiling(lbmd_handle h, int32_t reps, double* ms) {
  if (!h || reps < 1 || !ms) return fail(h, LBMD_EINVAL, "stream_ceiling: bad arguments");
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  HIPCHECK(h, fluid_pull_copy(h));  // first touch outside the timing
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHECK(h, hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = fluid_pull_copy(h);
  if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(h, e, "stream_ceiling");
  *ms = double(t) / reps;
  return LBMD_OK;
}

int lbmd_set_graph(lbmd_handle h, int32_t enable) {
  if (!h) return LBMD_EINVAL;
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  h->use_graph = enable != 0;
  if (!h->use_graph) graph_invalidate(h);
  return LBMD_OK;
}

int lbmd_autotune(lbmd_handle h, int32_t reps, const char* cache_path, int32_t* chosen, double* best_ms) {
  if (!h || reps < 1) return fail(h, LBMD_EINVAL, "autotune: bad arguments");
  if (h->batch) return fail(h, LBMD_ESTATE, "the handle is attached to a batch");
  if (h->latched) return fail(h, LBMD_ESTATE, "autotune: a numerical failure is latched");
  return autotune(h, reps, cache_path, chosen, best_ms);
}

}  // extern "C"
