"""Throughput of the coupled Shan-Chen LB + particle step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2_256]

Prints one JSON line.  A step is one pass of the whole path: particle half
kick and drift, density and Shan-Chen force, coupling forces at the nodes,
spread, collision with forcing (and fluctuations when kT > 0), streaming,
second half kick and the FP64 conservation sums.  Inputs are resident on the
device before the timed region starts.

value            lattice updates per second (MLUPS) over the timed K steps
roofline         the fused collide-stream kernel: algorithmic bytes per launch
                 (38 populations read + 38 written per site) over its average
                 launch duration, from HIP events on the stream it runs on
cpu_baseline     the FP64 oracle on the host cores (one thread and all usable
                 cores), on a 64^3 box of the same workload (same densities
                 recipe, same particle number density), and the full 32^3 FP64
                 workload of 100 steps
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
PROFILE_DIR = os.path.join(ROOT, "profiles")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lbmd_fluid.hip", "lbmd_push.hip", "lbmd_stencil.h", "lbmd_site.h", "lbmd_internal.h"):
        with open(os.path.join(ROOT, "paper_1306_0788_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name, workload):
    """HBM bytes per launch of the timed kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(PROFILE_DIR, "%s_%s_counters.md" % (kernel_name, workload))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel source hash:\s*([0-9a-f]+)", txt)
    t = re.search(r"HBM bytes per launch \(scaled\):\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != kernel_source_hash():
        return None
    return float(t.group(1))


PRECISIONS = {"fp64": 0, "fp32": 1, "fp16dev": 2, "bf16dev": 3}
STORAGE_BYTES = {"fp64": 8, "fp32": 4, "fp16dev": 2, "bf16dev": 2}


def kernel_bytes_per_site(kname, prec_name):
    """Algorithmic HBM bytes per site of one launch of the collide-stream
    kernel: the 38 pulled populations read and 38 written, plus, for the
    two-pass collide kernel, the two densities of the density field it reads,
    and for the push kernel the two densities of the moment field it reads
    and the five moments of the next step it writes (arithmetic type)."""
    pops = 76 * STORAGE_BYTES[prec_name]
    c = 8 if prec_name == "fp64" else 4
    return pops + {"k_fused": 0, "k_collide": 2 * c, "k_push": 7 * c}[kname]


def setup(workload, stream, kernel, tiling, precision=None):
    """The workload's simulation on the given stream; precision (a key of
    PRECISIONS) replaces the workload's storage precision if given."""
    from paper_1306_0788_amd import lbmd, workloads
    w = workloads.WORKLOADS[workload]
    shape = w["shape"]
    rho = workloads.initial_densities(shape, w["seed"]).reshape(2, -1)
    x, bonds = workloads.particles_for(w)
    prec = PRECISIONS[precision or w["precision"]]
    forcing = lbmd.FORCE_SHIFT if w["forcing"] == "shift" else lbmd.FORCE_PAPER
    sim = lbmd.Sim(shape, precision=prec, forcing=forcing, kernel=kernel, tau=w["tau"], G=w["G"],
                   gamma=w["gamma"], kappa=w["kappa"][0], mass=w["mass"][0], kT=w["kT"], seed=w["seed"],
                   rho_init=rho, stream=stream)
    sim.set_particle_types(w["kappa"], w["mass"], w["charge"])
    if w["wca"]:
        sim.set_pair_potential(lbmd.PAIR_WCA, w["wca"])
    if w["dh"]:
        sim.set_pair_potential(lbmd.PAIR_DH, w["dh"])
    if w["fene"]:
        sim.set_pair_potential(lbmd.BOND_FENE, w["fene"])
    sim.set_particles(x)
    if bonds is not None:
        sim.set_bonds(bonds)
    if tiling:
        sim.set_tiling(*tiling)
    return sim, w, len(x)


def host_cpu():
    """Model name and logical CPU counts of this host."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def _oracle_sim(w, shape, forcing=None):
    import oracle
    from paper_1306_0788_amd import workloads
    rho = workloads.initial_densities(shape, w["seed"]).reshape(2, -1)
    x, bonds = workloads.particles_for(w, shape)
    forcing = forcing or w["forcing"]
    P = oracle.make_params(shape, tau=w["tau"], G=w["G"],
                           forcing=oracle.FORCE_SHIFT if forcing == "shift" else oracle.FORCE_PAPER,
                           gamma=w["gamma"], kT=w["kT"], seed=w["seed"], kappa=w["kappa"], mass=w["mass"],
                           charge=w["charge"], wca=w["wca"], fene=w["fene"], dh=w["dh"])
    return oracle.Sim(P, rho, x, None, None, bonds), len(x)


def _oracle_mlups(w, shape, threads, target_s):
    """MLUPS of the oracle on `shape` with `threads` OpenMP threads over as
    many steps as fit in about target_s (at least 2)."""
    import oracle
    oracle.set_threads(threads)
    s, npart = _oracle_sim(w, shape)
    t0 = time.perf_counter()
    s.step(1)
    t1 = time.perf_counter()
    n = max(1, int(target_s / max(t1 - t0, 1e-3)) - 1)
    s.step(n)
    t2 = time.perf_counter()
    steps = n + 1
    return int(np.prod(shape)) * steps / (t2 - t0) / 1e6, steps, npart


def cpu_baseline(workload, target_s=10.0):
    """The FP64 oracle as it stands, timed on this host's cores: on a 64^3 box
    of the benchmarked workload (same density recipe, same particle number
    density) with one thread and with every usable core (its OpenMP loops
    give bit-identical results for any thread count), and the full 32^3
    FP64 workload (64 particles, 100 steps) on every core.  value = the
    all-core MLUPS of the 64^3 sample."""
    import oracle
    from paper_1306_0788_amd import workloads
    w = workloads.WORKLOADS[workload]
    model, ncpu, usable = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or usable
    shape = (64, 64, 64)
    one, steps1, npart = _oracle_mlups(w, shape, 1, target_s)
    print("bench: CPU oracle 1 thread %.3f MLUPS" % one, file=sys.stderr, flush=True)
    allc, stepsN, _ = _oracle_mlups(w, shape, threads, target_s)
    print("bench: CPU oracle %d threads %.3f MLUPS" % (threads, allc), file=sys.stderr, flush=True)
    # the 32^3 FP64 workload in full; its velocity-shift forcing reaches zero
    # density at step 35 from this start, so the 100 steps run with the
    # paper's forcing (as the parity tests' 100-step runs do)
    oracle.set_threads(threads)
    c1 = workloads.WORKLOADS["c1"]
    s, n1 = _oracle_sim(c1, c1["shape"], forcing="paper")
    t0 = time.perf_counter()
    st = s.step(c1["steps"])
    t_c1 = time.perf_counter() - t0
    oracle.set_threads(1)
    return {"value": round(allc, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "FP64 oracle, %d OpenMP threads, %d steps of a 64^3 box of workload %s (%d particles)"
                      % (threads, stepsN, workload, npart),
            "single_thread_MLUPS": round(one, 4), "single_thread_steps": steps1,
            "host": {"cpu_model": model, "nproc": ncpu, "usable_cpus": usable},
            "c1_full": {"lattice": list(c1["shape"]), "particles": n1, "steps": c1["steps"],
                        "forcing": "paper", "threads": threads, "seconds": round(t_c1, 3),
                        "MLUPS": round(int(np.prod(c1["shape"])) * c1["steps"] / t_c1 / 1e6, 4),
                        "status": "ok" if st == oracle.OK else "unstable"}}


def copy_calibration():
    """A plain elementwise copy kernel (torch.mul by 1) over 2 GiB of float32:
    the reference for scaling the FETCH_SIZE / WRITE_SIZE counters and for the
    copy bandwidth this device reaches in practice."""
    import torch
    torch.cuda.set_device(0)
    n = 512 * 1024 * 1024
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    print(json.dumps({"copy_kernel_bytes_read": n * 4, "copy_kernel_bytes_written": n * 4,
                      "ms": round(ms, 4), "GBs_read_plus_write": round(2 * n * 4 / ms / 1e6, 1)}), flush=True)


def interface(phi, shape):
    """Interface of phi = rho_A - rho_B on the periodic lattice (the locus
    rho_A = rho_B): per axis, the links across which phi changes sign and the
    linear zero crossing along each (fraction of the link from its lower
    site).  Returns {axis: (link mask, crossing)}."""
    nx, ny, nz = shape
    f = phi.reshape(nz, ny, nx)
    out = {}
    for ax, npax in (("x", 2), ("y", 1), ("z", 0)):
        g = np.roll(f, -1, axis=npax)
        m = (f > 0) != (g > 0)
        t = np.where(m, f / np.where(m, f - g, 1.0), 0.0)
        out[ax] = (m, t)
    return out


def accuracy_study(workload, steps):
    """Error of each storage form against the FP64 step after `steps` steps of
    the workload (same seeded inputs): density of A, coupling velocity u_c,
    interface area (links across which rho_A - rho_B changes sign) and
    position (zero crossing along the links both runs cut), and the mass
    drift of each component from the device FP64 sums."""
    import torch
    from paper_1306_0788_amd import lbmd
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    res = {}
    ref = None
    for prec in ("fp64", "fp32", "fp16dev", "bf16dev"):
        print("accuracy: %s %s, %d steps" % (workload, prec, steps), file=sys.stderr, flush=True)
        sim, w, npart = setup(workload, stream.cuda_stream, lbmd.KERNEL_AUTO, None, prec)
        sim.step(1)
        r0, _ = sim.reductions()
        sim.step(steps - 1)
        rc = sim.sync()
        if rc != lbmd.OK:
            res[prec] = {"failed": sim.last_error()}
            sim.close()
            continue
        r1, _ = sim.reductions()
        fields = sim.get_fields(lbmd.RHO | lbmd.U)
        sim.close()
        N = int(np.prod(w["shape"]))
        rho = fields[:2 * N].reshape(2, N)
        u = fields[2 * N:].reshape(3, N)
        itf = interface(rho[0] - rho[1], w["shape"])
        area = int(sum(int(m.sum()) for m, _ in itf.values()))
        drift = [float(abs(r1[c] - r0[c]) / r0[c]) for c in range(2)]
        if ref is None:
            ref = (rho, u, itf, area)
            res[prec] = {"interface_links": area, "mass_drift": drift}
            continue
        rr, ur, itr, ar = ref
        both = [(m & itr[ax][0], t, itr[ax][1]) for ax, (m, t) in itf.items()]
        nboth = sum(int(b.sum()) for b, _, _ in both)
        pos_err = sum(float(np.abs(t[b] - tr[b]).sum()) for b, t, tr in both) / max(nboth, 1)
        dr = rho[0] - rr[0]
        du = u - ur
        res[prec] = {"rho_A_max_abs_err": float(np.abs(dr).max()), "rho_A_rms_err": float(np.sqrt(np.mean(dr ** 2))),
                     "u_max_abs_err": float(np.abs(du).max()), "u_rms_err": float(np.sqrt(np.mean(du ** 2))),
                     "u_max_abs_ref": float(np.abs(ur).max()),
                     "interface_links": area, "interface_links_rel_diff": (area - ar) / max(ar, 1),
                     "interface_position_mean_abs_diff": pos_err, "mass_drift": drift}
        del rho, u, itf
    print(json.dumps({"accuracy": workload, "steps": steps, "reference": "fp64 GPU step (parity-tested "
                      "against the FP64 oracle)", "results": res}), flush=True)


def _emulsion(args):
    from paper_1306_0788_amd import workloads
    return workloads.emulsion_job(*args)


def serving(njobs, rate, seed, max_jobs, mem_gib, one_by_one, jobs, single_batch=False):
    """The serving workload: a Poisson stream of emulsion jobs served with
    continuous batching (and, if asked, one job at a time)."""
    from paper_1306_0788_amd import serve, workloads
    arrivals = workloads.poisson_arrivals(njobs, rate, seed)
    print("serve: %d jobs at %.0f/s, continuous batching (%d slots, %d GiB)" % (njobs, rate, max_jobs, mem_gib),
          file=sys.stderr, flush=True)
    count = [0]

    def progress(msg):
        count[0] += 1
        if count[0] % 64 == 0:
            print("serve: %d jobs finished (%s)" % (count[0], msg), file=sys.stderr, flush=True)

    rb = serve.serve_batched_classes(jobs, arrivals, bounds=(64 ** 3,), max_jobs=max_jobs,
                                     mem_budget=mem_gib << 30, chunk=10, log=progress)
    out = {"jobs": njobs, "arrival_rate_per_s": rate, "steps_per_job": jobs[0]["steps"],
           "lattice_sites_mean": float(np.mean([np.prod(j["shape"]) for j in jobs])),
           "slots": max_jobs, "memory_budget_GiB": mem_gib,
           "batched": dict(serve.summarize(jobs, rb), size_classes="<= 64^3 sites, larger: one batch each")}
    if single_batch:
        print("serve: the same stream in one batch for all sizes", file=sys.stderr, flush=True)
        count[0] = 0
        r1 = serve.serve_batched(jobs, arrivals, max_jobs=max_jobs, mem_budget=mem_gib << 30, chunk=10, log=progress)
        out["batched_one_class"] = serve.summarize(jobs, r1)
    if one_by_one:
        print("serve: the same stream one job at a time", file=sys.stderr, flush=True)
        count[0] = 0
        rs = serve.serve_one_by_one(jobs, arrivals, log=progress)
        out["one_by_one"] = serve.summarize(jobs, rs)
        fb = [r["failed"] for r in rb]
        fs = [r["failed"] for r in rs]
        out["same_failures"] = fb == fs
    return out


def run_workload(name, stream, kernel, tiling, precision, autotune, cache, graph, warmup, steps):
    """Set up workload `name` on `stream`, tune its tiling (unless told not
    to), take `warmup` untimed steps, then time `steps` steps between HIP
    events on the stream, with the collide-stream kernel's launches timed
    by events of their own (eager launches; with graph replay those are
    taken over the warm-up instead).  Returns the measurements, or None after
    a numerical failure."""
    import torch
    from paper_1306_0788_amd import lbmd
    print("bench: setting up %s" % name, file=sys.stderr, flush=True)
    sim, w, npart = setup(name, stream.cuda_stream, kernel, tiling, precision)
    sim_org = sim.organisation()
    tuned = None
    if autotune:
        print("bench: autotuning the tiling", file=sys.stderr, flush=True)
        tuned = sim.autotune(reps=5, cache_path=cache)
    if graph:
        sim.set_graph(True)
    N = int(np.prod(w["shape"]))
    prec_name = precision or w["precision"]
    s_bytes = STORAGE_BYTES[prec_name]
    label = name if prec_name == w["precision"] else "%s_%s" % (name, prec_name)
    print("bench: %s warmup %d steps" % (name, warmup), file=sys.stderr, flush=True)
    first = min(2, warmup)
    sim.step(first)
    if graph:
        sim.kernel_timing(True)
    sim.step(warmup - first)
    torch.cuda.synchronize()
    if graph:
        kms, launches = sim.kernel_timing(False)
    assert sim.sync() == lbmd.OK, sim.last_error()
    if not graph:
        sim.kernel_timing(True)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    sim.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    if not graph:
        kms, launches = sim.kernel_timing(False)
    st = sim.sync()
    if st != lbmd.OK:
        print("bench: %s numerical failure: %s" % (name, sim.last_error()), file=sys.stderr)
        sim.close()
        return None
    print("bench: %s timed %d steps in %.3f ms" % (name, steps, ms), file=sys.stderr, flush=True)
    kname = {lbmd.KERNEL_FUSED: "k_fused", lbmd.KERNEL_TWOPASS: "k_collide", lbmd.KERNEL_PUSH: "k_push"}[sim_org]
    # the same bytes moved by a pass with no arithmetic (one site per
    # thread): what this access pattern reaches on the device
    ceil_gbs = 76 * s_bytes * N / (sim.stream_ceiling(10) * 1e-3) / 1e9
    sim.close()
    del sim
    return dict(ms=ms, N=N, npart=npart, w=w, prec=prec_name, s_bytes=s_bytes, label=label, org=sim_org,
                tuned=tuned, kname=kname, kernel_ms=kms / max(launches, 1), ceiling_gbs=ceil_gbs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the G_AB = 1.8 workloads drive a density to zero at a known step from
    # the uniform start ("onset"); the default window stays inside it
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2_256")
    ap.add_argument("--kernel", choices=["auto", "fused", "twopass", "push"], default="auto")
    ap.add_argument("--precision", choices=sorted(PRECISIONS), default=None,
                    help="population storage (default: the workload's); fp16dev / bf16dev store f - w rho0")
    ap.add_argument("--tiling", type=int, nargs=2, default=None, metavar=("TILE_Y", "TILE_Z"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="advance the timed steps by replaying the step captured as a HIP graph (the kernel's "
                         "roofline time is then taken over eager warm-up steps, not the timed region)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the library's default tiling instead of running its autotuner before the "
                         "untimed warm-up")
    ap.add_argument("--autotune-cache", default=None, metavar="PATH",
                    help="tiling cache file: a run that finds its key there skips the timing (profiling runs use "
                         "the tiling an earlier run chose, without the candidates' launches in their traces)")
    ap.add_argument("--also", nargs="*", default=["c3"], metavar="WORKLOAD",
                    help="further workloads timed the same way and reported as keys of the line (default: the "
                         "256^3 bead-spring workload c3)")
    ap.add_argument("--serve-jobs", type=int, default=512, help="jobs in the served Poisson stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="arrivals per second")
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-mem-gib", type=int, default=64)
    ap.add_argument("--serve-one-by-one", action="store_true",
                    help="also serve the stream one job at a time for comparison")
    ap.add_argument("--serve-one-batch", action="store_true",
                    help="also serve the stream with one batch for all sizes (no size classes)")
    ap.add_argument("--serve-only", action="store_true", help="only the serving workload")
    ap.add_argument("--accuracy", type=int, default=None, metavar="STEPS",
                    help="instead of timing: error of every storage form against the FP64 step after STEPS steps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 2 GiB copy kernel used to calibrate the byte counters")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.accuracy is not None:
        accuracy_study(args.workload, args.accuracy)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: lbmd runs on one GPU only (the step would shard by z-slabs across GPUs, "
              "which is not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    jobs = None
    if args.serve_jobs > 0:
        # inputs of the served stream, generated before the GPU is touched
        import multiprocessing as mp
        print("bench: generating %d serving jobs" % args.serve_jobs, file=sys.stderr, flush=True)
        with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
            jobs = pool.map(_emulsion, [(5, i) for i in range(args.serve_jobs)], chunksize=4)

    from paper_1306_0788_amd import workloads
    onset = workloads.WORKLOADS[args.workload].get("onset")
    if args.steps is None:
        args.steps = 90 if onset is None else min(90, onset - 5 - args.warmup)
    if onset is not None and args.warmup + args.steps >= onset:
        print("bench.py: workload %s reaches zero density at step %d; warmup + steps must stay below it"
              % (args.workload, onset), file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1306_0788_amd import lbmd
    assert torch.cuda.is_available(), "no GPU visible"
    if args.serve_only:
        torch.cuda.set_device(0)
        print(json.dumps({"served": serving(args.serve_jobs, args.serve_rate, 5, args.serve_slots,
                                            args.serve_mem_gib, args.serve_one_by_one, jobs,
                                            args.serve_one_batch)}), flush=True)
        return
    torch.cuda.set_device(0)
    # a dedicated stream (the current one may be the null stream, handle 0,
    # which the library would replace by a stream of its own)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    kernel = {"auto": lbmd.KERNEL_AUTO, "fused": lbmd.KERNEL_FUSED, "twopass": lbmd.KERNEL_TWOPASS,
              "push": lbmd.KERNEL_PUSH}[args.kernel]
    r = run_workload(args.workload, stream, kernel, args.tiling, args.precision, args.autotune,
                     args.autotune_cache, args.graph, args.warmup, args.steps)
    if r is None:
        sys.exit(1)
    ms, N, npart, w, prec_name, s_bytes, label = r["ms"], r["N"], r["npart"], r["w"], r["prec"], r["s_bytes"], \
        r["label"]
    sim_org, tuned, kname = r["org"], r["tuned"], r["kname"]
    mlups = N * args.steps / (ms * 1e-3) / 1e6
    # the step: the populations every organisation must move (76 per site);
    # the kernel: its own algorithmic bytes
    alg_bytes = 76 * s_bytes * N
    kbytes = kernel_bytes_per_site(kname, prec_name)
    kavg_s = r["kernel_ms"] * 1e-3
    achieved = kbytes * N / kavg_s / 1e9
    traffic = measured_traffic(kname, label)
    ceil_gbs = r["ceiling_gbs"]
    line = {
        "metric": "MLUPS (2-component D3Q19 Shan-Chen + coupled particles, one full step)",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16dev": "f16 storage, f32 math",
                  "bf16dev": "bf16 storage, f32 math"}[prec_name],
        "data": "synthetic",
        "config": {"workload": label, "lattice": list(w["shape"]), "particles": npart,
                   "storage": prec_name,
                   "forcing": w["forcing"], "kT": w["kT"],
                   "kernel": {lbmd.KERNEL_FUSED: "fused", lbmd.KERNEL_TWOPASS: "twopass",
                              lbmd.KERNEL_PUSH: "push"}[sim_org],
                   "graph": bool(args.graph), "autotuned_tiling": None if tuned is None else list(tuned[:3]),
                   "particle_updates_per_s": round(npart * args.steps / (ms * 1e-3), 1)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": kname,
                     "kernel_ms_avg": round(kavg_s * 1e3, 5), "bytes_per_site": kbytes,
                     "step_achieved": round(alg_bytes / (ms / args.steps * 1e-3) / 1e9, 1),
                     "step_frac": round(alg_bytes / (ms / args.steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "step_bytes_per_site": 76 * s_bytes,
                     "pattern_ceiling": round(ceil_gbs, 1), "frac_of_pattern_ceiling": round(achieved / ceil_gbs, 4)},
    }
    for extra in args.also:
        # further workloads, timed the same way (own warm-up and window below
        # their recorded onset), reported as keys of the same line
        wx = workloads.WORKLOADS[extra]
        onx = wx.get("onset")
        kx = 70 if onx is None else min(70, onx - 5 - args.warmup)
        rx = run_workload(extra, stream, lbmd.KERNEL_AUTO, None, None, args.autotune, args.autotune_cache,
                          args.graph, args.warmup, kx)
        if rx is None:
            line[extra] = {"failed": True}
            continue
        bx = 76 * rx["s_bytes"] * rx["N"]
        kbx = kernel_bytes_per_site(rx["kname"], rx["prec"]) * rx["N"]
        line[extra] = {"MLUPS": round(rx["N"] * kx / (rx["ms"] * 1e-3) / 1e6, 2), "steps": kx,
                       "ms_per_step": round(rx["ms"] / kx, 5), "lattice": list(rx["w"]["shape"]),
                       "particles": rx["npart"], "kT": rx["w"]["kT"], "kernel": rx["kname"],
                       "kernel_ms_avg": round(rx["kernel_ms"], 5),
                       "kernel_frac": round(kbx / (rx["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "step_frac": round(bx / (rx["ms"] / kx * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "autotuned_tiling": None if rx["tuned"] is None else list(rx["tuned"][:3]),
                       "particle_updates_per_s": round(rx["npart"] * kx / (rx["ms"] * 1e-3), 1)}
    if jobs is not None:
        line["served"] = serving(args.serve_jobs, args.serve_rate, 5, args.serve_slots, args.serve_mem_gib,
                                 args.serve_one_by_one, jobs, args.serve_one_batch)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
