// Multi-lattice batches (C ABI in include/lbmd.h): independent simulations,
// each created as an ordinary handle, advanced together by one launch
// sequence per step whose kernels walk the work of all attached jobs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "lbmd_internal.h"

using namespace lbmd;

struct lbmd_batch_s {
  int max_jobs = 0;
  bool noise = false;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<lbmd_ctx*> job;      // per slot; nullptr = free
  std::vector<int64_t> target;     // per slot: step at which the job stops
  std::vector<int> row_slot;       // table row -> slot
  BatchJob* tab_host = nullptr;    // pinned
  BatchHeader* hdr_host = nullptr; // pinned
  BatchJob* tab = nullptr;         // device
  BatchHeader* hdr = nullptr;      // device
  int64_t* gather = nullptr;       // device [2 max_jobs]
  int64_t* gather_host = nullptr;  // pinned
  bool dirty = true;
  hipGraphExec_t gexec = nullptr;
  std::string err;
};

namespace {

int bfail(lbmd_batch_s* b, int code, const char* msg) {
  if (b) b->err = msg;
  return code;
}

#define BHIP(b, expr)                                            \
  do {                                                           \
    hipError_t e_ = (expr);                                      \
    if (e_ != hipSuccess) return bfail(b, LBMD_EDEVICE, #expr);  \
  } while (0)

// Rebuild the job table from the occupied slots (in slot order) and upload
// it.  The stream is idle here, so the pinned copies can be rewritten.  The z
// chunk is common to the table: 16 planes (long z marches; the three-plane
// start of a march is paid once per chunk) unless the tiles would then not
// fill the fused kernel's grid, in which case it is halved (down to 2) --
// a lone small lattice gets the parallelism, a full table the long marches.
// The fused pass gives the same results for any chunk.
int upload(lbmd_batch_s* b) {
  BHIP(b, hipStreamSynchronize(b->stream));
  b->row_slot.clear();
  int tz = 16;
  for (; tz > 2; tz /= 2) {
    int64_t t = 0;
    for (int s = 0; s < b->max_jobs; ++s)
      if (const lbmd_ctx* h = b->job[s]) {
        const int z = std::min(tz, h->p.nz);
        t += int64_t((h->p.nx + 63) / 64) * ((h->p.ny + BATCH_TY - 1) / BATCH_TY) * ((h->p.nz + z - 1) / z);
      }
    if (t >= BATCH_FLUID_GRID) break;
  }
  int64_t tiles = 0, pblk = 0, fix = 0, cmp = 0;
  for (int s = 0; s < b->max_jobs; ++s) {
    lbmd_ctx* h = b->job[s];
    if (!h) continue;
    BatchJob& J = b->tab_host[b->row_slot.size()];
    std::memset(&J, 0, sizeof J);
    batch_fill_fluid(h, J, tz);
    if (h->np > 0) batch_fill_particles(h, J);
    J.target = b->target[s];
    J.tile_begin = tiles;
    J.pblk_begin = pblk;
    J.fix_begin = fix;
    J.cmp_begin = cmp;
    tiles += J.nblk;
    pblk += J.npblk;
    fix += J.nfixblk;
    cmp += J.ncmpblk;
    b->row_slot.push_back(s);
  }
  b->hdr_host->njobs = int32_t(b->row_slot.size());
  b->hdr_host->ntiles = tiles;
  b->hdr_host->npblk = pblk;
  b->hdr_host->nfixblk = fix;
  b->hdr_host->ncmpblk = cmp;
  if (!b->row_slot.empty())
    BHIP(b, hipMemcpyAsync(b->tab, b->tab_host, b->row_slot.size() * sizeof(BatchJob), hipMemcpyHostToDevice,
                           b->stream));
  BHIP(b, hipMemcpyAsync(b->hdr, b->hdr_host, sizeof(BatchHeader), hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  b->dirty = false;
  return LBMD_OK;
}

int enqueue_batch_step(lbmd_batch_s* b) {
  BHIP(b, batch_particles_begin(b->stream, b->tab, b->hdr));
  BHIP(b, batch_fluid_pass(b->stream, b->tab, b->hdr, b->noise));
  BHIP(b, batch_particles_couple(b->stream, b->tab, b->hdr));
  BHIP(b, batch_fluid_fix(b->stream, b->tab, b->hdr, b->noise));
  BHIP(b, batch_particles_end(b->stream, b->tab, b->hdr));
  BHIP(b, batch_finalize(b->stream, b->tab, b->hdr, b->max_jobs));
  return LBMD_OK;
}

int capture(lbmd_batch_s* b) {
  BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_batch_step(b);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc != LBMD_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc != LBMD_OK ? rc : bfail(b, LBMD_EDEVICE, "hipStreamEndCapture");
  }
  const hipError_t ei = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return bfail(b, LBMD_EDEVICE, "hipGraphInstantiate");
  return LBMD_OK;
}

void release_job(lbmd_batch_s* b, int slot) {
  lbmd_ctx* h = b->job[slot];
  // the host's step count and ping-pong parity follow the device counter
  int64_t st = h->step;
  if (hipMemcpy(&st, h->step_dev, sizeof st, hipMemcpyDeviceToHost) == hipSuccess) {
    h->step = st;
    h->cur = int(st & 1);
  }
  h->batch = nullptr;
  b->job[slot] = nullptr;
  b->dirty = true;
}

}  // namespace

extern "C" {

int lbmd_batch_create(int32_t max_jobs, int32_t noise, void* hip_stream, lbmd_batch* out) {
  if (!out || max_jobs < 1 || max_jobs > 4096) return LBMD_EINVAL;
  *out = nullptr;
  lbmd_batch_s* b = new (std::nothrow) lbmd_batch_s();
  if (!b) return LBMD_ENOMEM;
  b->max_jobs = max_jobs;
  b->noise = noise != 0;
  b->job.assign(max_jobs, nullptr);
  b->target.assign(max_jobs, 0);
  auto bail = [&](int rc) {
    lbmd_batch_destroy(b);
    return rc;
  };
  if (hipGetDevice(&b->device) != hipSuccess) return bail(LBMD_EDEVICE);
  if (hip_stream) {
    b->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) return bail(LBMD_EDEVICE);
    b->own_stream = true;
  }
  if (hipHostMalloc((void**)&b->tab_host, max_jobs * sizeof(BatchJob), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->hdr_host, sizeof(BatchHeader), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->gather_host, 2 * max_jobs * sizeof(int64_t), hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void**)&b->tab, max_jobs * sizeof(BatchJob)) != hipSuccess ||
      hipMalloc((void**)&b->hdr, sizeof(BatchHeader)) != hipSuccess ||
      hipMalloc((void**)&b->gather, 2 * max_jobs * sizeof(int64_t)) != hipSuccess)
    return bail(LBMD_ENOMEM);
  std::memset(b->hdr_host, 0, sizeof(BatchHeader));
  if (upload(b) != LBMD_OK) return bail(LBMD_EDEVICE);
  *out = b;
  return LBMD_OK;
}

int lbmd_batch_destroy(lbmd_batch b) {
  if (!b) return LBMD_EINVAL;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (int s = 0; s < b->max_jobs; ++s)
    if (b->job[s]) release_job(b, s);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->tab_host) (void)hipHostFree(b->tab_host);
  if (b->hdr_host) (void)hipHostFree(b->hdr_host);
  if (b->gather_host) (void)hipHostFree(b->gather_host);
  if (b->tab) (void)hipFree(b->tab);
  if (b->hdr) (void)hipFree(b->hdr);
  if (b->gather) (void)hipFree(b->gather);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return LBMD_OK;
}

int lbmd_batch_attach(lbmd_batch b, lbmd_handle h, int64_t nsteps, int32_t* slot) {
  if (!b || !h || nsteps < 0) return LBMD_EINVAL;
  if (h->batch) return bfail(b, LBMD_ESTATE, "attach: the handle is already in a batch");
  if (h->latched) return bfail(b, LBMD_ESTATE, "attach: the handle has a latched failure");
  if (h->p.precision != LBMD_FP32 || h->p.forcing != LBMD_FORCE_PAPER || (h->p.kT > 0.0) != b->noise)
    return bfail(b, LBMD_EINVAL, "attach: a batch runs FP32 populations, the paper's forcing and one noise setting");
  if (h->mrt) return bfail(b, LBMD_EINVAL, "attach: batch jobs use the BGK collision");
  if (h->pair.wca_on || h->pair.dh_on || h->pair.fene_on || h->nbonds > 0)
    return bfail(b, LBMD_EINVAL, "attach: batch jobs have no pair potentials or bonds");
  if (h->device != b->device) return bfail(b, LBMD_EINVAL, "attach: the handle lives on another device");
  int s = 0;
  while (s < b->max_jobs && b->job[s]) ++s;
  if (s == b->max_jobs) return bfail(b, LBMD_ESTATE, "attach: no free slot");
  BHIP(b, hipStreamSynchronize(h->stream));
  b->job[s] = h;
  b->target[s] = h->step + nsteps;
  h->batch = b;
  h->push_step = -1;  // the batch advances the populations, not the moment field
  b->dirty = true;
  if (slot) *slot = s;
  return LBMD_OK;
}

int lbmd_batch_detach(lbmd_batch b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->max_jobs || !b->job[slot]) return LBMD_EINVAL;
  BHIP(b, hipStreamSynchronize(b->stream));
  release_job(b, slot);
  return LBMD_OK;
}

int lbmd_batch_step(lbmd_batch b, int64_t nsteps) {
  if (!b || nsteps < 0) return LBMD_EINVAL;
  if (b->dirty)
    if (int rc = upload(b)) return rc;
  if (b->row_slot.empty() || nsteps == 0) return LBMD_OK;
  if (!b->gexec)
    if (int rc = capture(b)) return rc;
  for (int64_t k = 0; k < nsteps; ++k) BHIP(b, hipGraphLaunch(b->gexec, b->stream));
  return LBMD_OK;
}

int lbmd_batch_poll(lbmd_batch b, int64_t* steps, int32_t* state) {
  if (!b) return LBMD_EINVAL;
  if (b->dirty)
    if (int rc = upload(b)) return rc;
  BHIP(b, batch_gather(b->stream, b->tab, b->hdr, b->max_jobs, b->gather));
  BHIP(b, hipMemcpyAsync(b->gather_host, b->gather, 2 * b->max_jobs * sizeof(int64_t), hipMemcpyDeviceToHost,
                         b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  for (int s = 0; s < b->max_jobs; ++s) {
    if (steps) steps[s] = -1;
    if (state) state[s] = 0;
  }
  for (size_t r = 0; r < b->row_slot.size(); ++r) {
    const int s = b->row_slot[r];
    const int64_t st = b->gather_host[2 * r], status = b->gather_host[2 * r + 1];
    if (steps) steps[s] = st;
    if (state) state[s] = status != 0 ? 3 : (st >= b->target[s] ? 2 : 1);
  }
  return LBMD_OK;
}

const char* lbmd_batch_last_error(lbmd_batch b) { return b ? b->err.c_str() : "NULL batch"; }

}  // extern "C"
