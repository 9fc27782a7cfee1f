"""Serving independent simulations with continuous batching.

A request loop admits jobs (lattice, G, particles, step count) as they
arrive, in arrival order, whenever a batch slot is free and the job's device
footprint fits the memory budget; admitted jobs keep their lattices and
particles resident and advance together in the multi-lattice batch
(lbmd_batch_*: one launch sequence per step for all jobs, captured in a HIP
graph); a job leaves the batch, and frees its memory, when it reaches its
step count or fails numerically, and queued jobs take its place.  The same
jobs can be run one by one on the single-job path for comparison.

Time-to-completion of a job = completion time - arrival time (queueing,
set-up, stepping).  Aggregate MLUPS = lattice site updates of all completed
steps / (last completion - first arrival).
"""
import threading
import time
from collections import deque

import numpy as np

from . import lbmd

# device bytes per site: two population buffers (2 x 38 x 4), the density
# field (2 x 4), node records (16 x 4), node forces (4 x 4), touched-node mask
BYTES_PER_SITE = 2 * 38 * 4 + 2 * 4 + 16 * 4 + 4 * 4 + 1 / 8
BYTES_PER_PARTICLE = 4 * 3 * 8 + 4 + 8 * 4 + 64


def footprint(job):
    """Device bytes a job holds while resident."""
    return int(np.prod(job["shape"]) * BYTES_PER_SITE + len(job["x"]) * BYTES_PER_PARTICLE)


def make_sim(job, kernel=lbmd.KERNEL_AUTO, check_every=0):
    sim = lbmd.Sim(job["shape"], precision=lbmd.FP32, forcing=lbmd.FORCE_PAPER, kernel=kernel,
                   G=((0.0, job["G"]), (job["G"], 0.0)), gamma=job["gamma"], kappa=job["kappa"],
                   mass=job["mass"], kT=job.get("kT", 0.0), seed=job.get("seed", 0), rho_init=job["rho"],
                   check_every=check_every)
    if len(job["x"]):
        sim.set_particles(job["x"])
    return sim


def serve_batched(jobs, arrivals, max_jobs=32, mem_budget=64 << 30, chunk=10, log=None):
    """Continuous batching.  Returns one record per job: arrival, admitted,
    done (s from the start), steps completed, failed flag."""
    n = len(jobs)
    rec = [dict(arrival=float(arrivals[i]), admitted=None, done=None, steps=0, failed=False) for i in range(n)]
    pending = deque(range(n))
    queue = deque()
    batch = lbmd.Batch(max_jobs=max_jobs, noise=False)
    active = {}  # slot -> (job index, sim, bytes)
    used = 0
    finished = 0
    t0 = time.perf_counter()
    try:
        while finished < n:
            now = time.perf_counter() - t0
            while pending and arrivals[pending[0]] <= now:
                queue.append(pending.popleft())
            # the device first: a chunk of steps for the resident jobs ...
            if active:
                batch.step(chunk)
            # ... while the host sets up the jobs it can admit (their set-up
            # runs on their own streams) ...
            new = []
            while queue and len(active) + len(new) < max_jobs and used + footprint(jobs[queue[0]]) <= mem_budget:
                i = queue.popleft()
                new.append((i, make_sim(jobs[i], kernel=lbmd.KERNEL_FUSED)))
                used += footprint(jobs[i])
            if queue and not active and not new:
                raise RuntimeError("job %d does not fit the memory budget" % queue[0])
            # ... then waits for the chunk and retires finished jobs
            if active:
                steps, state = batch.poll()
                t = time.perf_counter() - t0
                for slot in list(active):
                    if state[slot] in (lbmd.DONE, lbmd.FAILED):
                        i, sim, b = active.pop(slot)
                        batch.detach(slot)
                        rec[i]["done"] = t
                        rec[i]["steps"] = int(steps[slot])
                        rec[i]["failed"] = state[slot] == lbmd.FAILED
                        sim.close()
                        used -= b
                        finished += 1
                        if log:
                            log("job %d (%s) %s at %.3f s" % (i, jobs[i]["shape"][0],
                                                             "failed" if rec[i]["failed"] else "done", t))
            for i, sim in new:
                slot = batch.attach(sim, jobs[i]["steps"])
                active[slot] = (i, sim, footprint(jobs[i]))
                rec[i]["admitted"] = time.perf_counter() - t0
            if not active and pending:
                time.sleep(max(0.0, min(0.01, arrivals[pending[0]] - (time.perf_counter() - t0))))
    finally:
        batch.close()
    return rec


def serve_batched_classes(jobs, arrivals, bounds=(64 ** 3,), max_jobs=32, mem_budget=64 << 30, chunk=10,
                          log=None):
    """Continuous batching by size class: the jobs are split by lattice size
    (class c takes the jobs with bounds[c-1] < sites <= bounds[c], the last
    class the rest), and each class is served by its own batch on its own
    stream, driven by its own host thread (the library calls release the
    interpreter lock while they wait).  A small job then advances at the pace
    of the small jobs' batch step instead of that of the largest box resident.
    Admission order, the memory budget and the records are shared; slots are
    split evenly between the classes.  Returns the records of serve_batched."""
    n = len(jobs)
    ncls = len(bounds) + 1

    def cls(i):
        sites = int(np.prod(jobs[i]["shape"]))
        for c, b in enumerate(bounds):
            if sites <= b:
                return c
        return ncls - 1

    for i in range(n):
        if footprint(jobs[i]) > mem_budget:
            raise RuntimeError("job %d does not fit the memory budget" % i)
    lbmd.load()  # the library is loaded once, before the workers start
    rec = [dict(arrival=float(arrivals[i]), admitted=None, done=None, steps=0, failed=False) for i in range(n)]
    pending = deque(range(n))
    queues = [deque() for _ in range(ncls)]
    slots = [max(1, max_jobs // ncls)] * ncls
    shared = {"used": 0, "finished": 0}
    lock = threading.Lock()
    errors = []
    t0 = time.perf_counter()

    def arrived():
        now = time.perf_counter() - t0
        while pending and arrivals[pending[0]] <= now:
            i = pending.popleft()
            queues[cls(i)].append(i)

    def worker(c):
        batch = lbmd.Batch(max_jobs=slots[c], noise=False)
        active = {}
        try:
            while True:
                with lock:
                    arrived()
                    if shared["finished"] == n:
                        break
                if active:
                    batch.step(chunk)
                take = []
                with lock:
                    while (queues[c] and len(active) + len(take) < slots[c] and
                           shared["used"] + footprint(jobs[queues[c][0]]) <= mem_budget):
                        i = queues[c].popleft()
                        take.append(i)
                        shared["used"] += footprint(jobs[i])
                new = [(i, make_sim(jobs[i], kernel=lbmd.KERNEL_FUSED)) for i in take]
                if active:
                    steps, state = batch.poll()
                    t = time.perf_counter() - t0
                    for slot in list(active):
                        if state[slot] in (lbmd.DONE, lbmd.FAILED):
                            i, sim, b = active.pop(slot)
                            batch.detach(slot)
                            rec[i]["done"] = t
                            rec[i]["steps"] = int(steps[slot])
                            rec[i]["failed"] = state[slot] == lbmd.FAILED
                            sim.close()
                            with lock:
                                shared["used"] -= b
                                shared["finished"] += 1
                            if log:
                                log("job %d (%s) %s at %.3f s" % (i, jobs[i]["shape"][0],
                                                                 "failed" if rec[i]["failed"] else "done", t))
                for i, sim in new:
                    slot = batch.attach(sim, jobs[i]["steps"])
                    active[slot] = (i, sim, footprint(jobs[i]))
                    rec[i]["admitted"] = time.perf_counter() - t0
                if not active:
                    with lock:
                        nxt = arrivals[pending[0]] - (time.perf_counter() - t0) if pending else 0.002
                    time.sleep(max(0.0005, min(0.005, nxt)))
        except Exception as e:  # surfaced by the caller after the join
            errors.append(e)
            with lock:
                shared["finished"] = n  # let the other threads end
        finally:
            batch.close()

    threads = [threading.Thread(target=worker, args=(c,)) for c in range(ncls)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    if errors:
        raise errors[0]
    return rec


def serve_one_by_one(jobs, arrivals, check_every=10, log=None):
    """The same stream served one job at a time on the single-job path
    (default organisation and tiling, graph replay)."""
    n = len(jobs)
    rec = [dict(arrival=float(arrivals[i]), admitted=None, done=None, steps=0, failed=False) for i in range(n)]
    t0 = time.perf_counter()
    for i in range(n):
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        rec[i]["admitted"] = time.perf_counter() - t0
        sim = make_sim(jobs[i], check_every=check_every)
        sim.set_graph(True)
        rc = sim.step_rc(jobs[i]["steps"])
        st = sim.sync()
        rec[i]["failed"] = rc != lbmd.OK or st != lbmd.OK
        rec[i]["steps"] = int(jobs[i]["steps"]) if not rec[i]["failed"] else _failed_step(sim)
        rec[i]["done"] = time.perf_counter() - t0
        sim.close()
        if log:
            log("job %d (%s) %s at %.3f s" % (i, jobs[i]["shape"][0], "failed" if rec[i]["failed"] else "done",
                                             rec[i]["done"]))
    return rec


def _failed_step(sim):
    msg = sim.last_error()
    try:
        return int(msg.split("step ")[1].split()[0])
    except (IndexError, ValueError):
        return 0


def summarize(jobs, rec):
    """Latency percentiles over the completed jobs, throughput over all
    lattice-site updates done, and where the failed jobs lie in G_AB (the
    failure is the model's: a density reaches zero)."""
    done = [r for r in rec if not r["failed"]]
    lat = np.array([r["done"] - r["arrival"] for r in done])
    sites = sum(int(np.prod(jobs[i]["shape"])) * rec[i]["steps"] for i in range(len(jobs)))
    span = max(r["done"] for r in rec) - min(r["arrival"] for r in rec)
    out = {"jobs": len(jobs), "completed": len(done), "failed": len(rec) - len(done),
           "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
           "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
           "aggregate_MLUPS": sites / span / 1e6, "makespan_s": span}
    G = np.array([j["G"] for j in jobs])
    failed = np.array([r["failed"] for r in rec])
    if failed.any():
        edges = np.round(np.arange(1.6, 2.21, 0.1), 2)
        bins = []
        for lo, hi in zip(edges[:-1], edges[1:]):
            sel = (G >= lo) & (G < hi + (1e-9 if hi >= 2.2 else 0.0))
            bins.append({"G": [float(lo), float(hi)], "jobs": int(sel.sum()), "failed": int((failed & sel).sum())})
        out["failures"] = {
            "cause": "a density reached zero, the model's own failure at these inputs: small droplets "
                     "compressed above their coexistence density at larger G_AB, and dense solvated "
                     "particles at any G_AB (the FP64 CPU oracle fails the same jobs; "
                     "tests/test_oracle_serving_jobs.py)",
            "G_min_failed": float(G[failed].min()),
            "G_max_completed": float(G[~failed].max()) if (~failed).any() else None,
            "median_failed_step": float(np.median([r["steps"] for r in np.array(rec)[failed]])),
            "by_G": bins}
    return out
