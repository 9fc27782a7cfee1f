"""Multi-lattice batches and the serving loop.

The batch kernels run the same per-site arithmetic as the fused single-job
kernels, so without particles a job's populations in the mix equal its
populations alone bit for bit (the fused kernel's results do not depend on
the tiling); with particles the float additions of the spread happen in
another order, and the comparison is at the FP32 one-step tolerance times
the step count."""
import numpy as np
import pytest

from paper_1306_0788_amd import lbmd, serve, workloads

pytestmark = pytest.mark.gpu


def job(shape, G, seed, npart=0, kT=0.0):
    rho = workloads.initial_densities(shape, seed, amp=0.03).reshape(2, -1)
    x = workloads.free_particles(npart, shape, seed) if npart else np.zeros((0, 3))
    return dict(shape=shape, G=G, rho=rho, x=x, kappa=(-0.2, 0.1), gamma=0.8, mass=20.0, kT=kT, seed=seed)


def sim_of(j, kernel=lbmd.KERNEL_FUSED):
    s = lbmd.Sim(j["shape"], precision=lbmd.FP32, kernel=kernel, G=((0, j["G"]), (j["G"], 0)), gamma=j["gamma"],
                 kappa=j["kappa"], mass=j["mass"], kT=j["kT"], seed=j["seed"], rho_init=j["rho"])
    if len(j["x"]):
        s.set_particles(j["x"])
    return s


def alone(j, steps):
    s = sim_of(j)
    s.step(steps)
    assert s.sync() == lbmd.OK, s.last_error()
    return s


def run_batch(jobs, steps, noise=False, chunk=7):
    b = lbmd.Batch(max_jobs=8, noise=noise)
    sims = [sim_of(j) for j in jobs]
    slots = [b.attach(s, n) for s, n in zip(sims, steps)]
    while True:
        b.step(chunk)
        st, state = b.poll()
        if all(state[k] in (lbmd.DONE, lbmd.FAILED) for k in slots):
            break
    for k in slots:
        b.detach(k)
    b.close()
    return sims, [state[k] for k in slots], [st[k] for k in slots]


@pytest.mark.parametrize("kT", [0.0, 1e-4])
def test_batch_equals_alone_without_particles(kT):
    jobs = [job((20, 24, 16), 1.5, 3, kT=kT), job((33, 17, 12), 1.7, 4, kT=kT), job((40, 40, 40), 1.6, 5, kT=kT)]
    steps = [12, 30, 21]
    print("batch vs alone, kT=%g" % kT, flush=True)
    sims, state, st = run_batch(jobs, steps, noise=kT > 0)
    for j, n, s, stt, k in zip(jobs, steps, sims, state, st):
        assert stt == lbmd.DONE and k == n
        assert s.step_index == n
        ref = alone(j, n)
        assert np.array_equal(s.populations(), ref.populations()), j["shape"]


def test_batch_jobs_match_the_oracle():
    """Three jobs of different sizes with particles, started between the
    coexistence densities of their own G (the served jobs' recipe), advanced
    together through lbmd_batch_* and compared element by element with the
    oracle: FP32 tolerance 1e-5 per step on the populations, and the
    particles' positions, velocities and forces."""
    import oracle
    from parity_cases import min_image_err, rel_err

    def droplet_job(L, G, R, npart, seed):
        a, b = workloads.coexistence(G)
        z, y, x = np.meshgrid(np.arange(L[2]), np.arange(L[1]), np.arange(L[0]), indexing="ij")
        d = np.sqrt((x - L[0] / 2) ** 2 + (y - L[1] / 2) ** 2 + (z - L[2] / 2) ** 2)
        s_ = 0.5 * (1 - np.tanh((d - R) / 2.0))
        rho = np.stack([b + (a - b) * s_, b + (a - b) * (1 - s_)]).reshape(2, -1)
        return dict(shape=L, G=G, rho=rho, x=workloads.free_particles(npart, L, seed), kappa=(-0.05, 0.0),
                    gamma=1.0, mass=100.0, kT=0.0, seed=seed)

    jobs = [droplet_job((20, 18, 16), 1.7, 4.0, 30, 1), droplet_job((33, 29, 23), 1.9, 6.0, 120, 2),
            droplet_job((12, 40, 9), 1.6, 3.5, 15, 3)]
    steps = [9, 14, 6]
    print("batch jobs vs oracle", flush=True)
    sims, state, st = run_batch(jobs, steps, chunk=4)
    for j, n, sim, stt in zip(jobs, steps, sims, state):
        assert stt == lbmd.DONE and sim.step_index == n
        P = oracle.make_params(j["shape"], G=((0, j["G"]), (j["G"], 0)), gamma=j["gamma"], kappa=(j["kappa"],),
                               mass=(j["mass"],))
        o = oracle.Sim(P, j["rho"], j["x"])
        assert o.step(n) == oracle.OK
        e = rel_err(sim.populations(), o.f)
        print("shape %s, %d steps: populations rel err %.2e" % (j["shape"], n, e), flush=True)
        assert e <= 1e-5 * n
        x, v, F, Fc = sim.particles()
        assert min_image_err(x, o.x, j["shape"]) <= 1e-5 * n
        assert np.abs(v - o.v).max() <= 1e-5 * n * max(np.abs(o.v).max(), 1e-3)
        assert np.abs(F - o.F).max() <= 1e-5 * n * max(np.abs(o.F).max(), 1e-6)


def test_batch_with_particles_matches_alone():
    jobs = [job((24, 20, 16), 1.4, 6, npart=40), job((48, 32, 20), 1.6, 7, npart=300), job((16, 16, 16), 1.3, 8)]
    steps = [10, 14, 9]
    print("batch with particles", flush=True)
    sims, state, st = run_batch(jobs, steps, chunk=4)
    for j, n, s in zip(jobs, steps, sims):
        ref = alone(j, n)
        a, r = s.populations(), ref.populations()
        e = np.max(np.abs(a - r) / np.abs(r))
        print("shape %s: max rel diff %.2e" % (j["shape"], e), flush=True)
        assert e <= 1e-5 * n
        if len(j["x"]):
            xa, va, Fa, _ = s.particles()
            xr, vr, Fr, _ = ref.particles()
            assert np.abs(va - vr).max() <= 1e-5 * n * max(np.abs(vr).max(), 1e-3)


def test_failed_job_leaves_the_others_unchanged():
    bad = job((24, 24, 24), 4.0, 9)  # far above the spinodal: a density reaches zero early
    good = [job((30, 22, 18), 1.5, 10), job((20, 20, 20), 1.6, 11)]
    print("failing job in the mix", flush=True)
    sims, state, st = run_batch([good[0], bad, good[1]], [40, 40, 25])
    assert state[1] == lbmd.FAILED and st[1] < 40
    assert sims[1].sync() == lbmd.EUNSTABLE
    assert state[0] == lbmd.DONE and state[2] == lbmd.DONE
    for j, n, s in ((good[0], 40, sims[0]), (good[1], 25, sims[2])):
        assert np.array_equal(s.populations(), alone(j, n).populations())


def test_late_join_and_leave():
    a, c = job((26, 18, 14), 1.5, 12), job((34, 20, 16), 1.4, 13)
    b = lbmd.Batch(max_jobs=4)
    sa, sc = sim_of(a), sim_of(c)
    ka = b.attach(sa, 20)
    b.step(6)
    kc = b.attach(sc, 11)
    b.step(30)
    st, state = b.poll()
    assert state[ka] == lbmd.DONE and state[kc] == lbmd.DONE and st[ka] == 20 and st[kc] == 11
    b.detach(ka)
    b.detach(kc)
    b.close()
    assert np.array_equal(sa.populations(), alone(a, 20).populations())
    assert np.array_equal(sc.populations(), alone(c, 11).populations())
    # a detached handle resumes on the single-job path
    sa.step(3)
    ref = alone(a, 23)
    assert np.array_equal(sa.populations(), ref.populations())


def test_attached_handle_is_locked_and_conditions_checked():
    b = lbmd.Batch(max_jobs=2)
    s = sim_of(job((16, 16, 16), 1.4, 14))
    k = b.attach(s, 5)
    with pytest.raises(lbmd.LbmdError):
        s.step(1)
    with pytest.raises(lbmd.LbmdError):
        b.attach(s, 5)
    b.detach(k)
    s64 = lbmd.Sim((8, 8, 8), precision=lbmd.FP64)
    with pytest.raises(lbmd.LbmdError):
        b.attach(s64, 5)
    b.close()


def test_serving_loop_completes_every_job():
    jobs = []
    for i, L in enumerate((20, 28, 36, 24, 32, 16)):
        j = job((L, L, L), 1.5, 20 + i, npart=30 + 10 * i)
        j["steps"] = 40 + 5 * i
        jobs.append(j)
    arrivals = np.array([0.0, 0.01, 0.02, 0.05, 0.06, 0.2])
    print("serving loop", flush=True)
    rec = serve.serve_batched(jobs, arrivals, max_jobs=3, mem_budget=1 << 30, chunk=8)
    for j, r in zip(jobs, rec):
        assert not r["failed"] and r["steps"] == j["steps"] and r["done"] >= r["arrival"]
    s = serve.summarize(jobs, rec)
    assert s["completed"] == len(jobs) and s["p99_s"] >= s["p50_s"] > 0


def test_size_class_serving_completes_every_job():
    jobs = []
    for i, L in enumerate((20, 40, 36, 24, 32, 16, 44)):
        j = job((L, L, L), 1.5, 30 + i, npart=30 + 10 * i)
        j["steps"] = 40 + 5 * i
        jobs.append(j)
    arrivals = np.array([0.0, 0.01, 0.02, 0.05, 0.06, 0.2, 0.21])
    print("size-class serving loop", flush=True)
    rec = serve.serve_batched_classes(jobs, arrivals, bounds=(28 ** 3,), max_jobs=4, mem_budget=1 << 30, chunk=8)
    for j, r in zip(jobs, rec):
        assert not r["failed"] and r["steps"] == j["steps"] and r["done"] >= r["admitted"] >= r["arrival"]
    s = serve.summarize(jobs, rec)
    assert s["completed"] == len(jobs) and s["p99_s"] >= s["p50_s"] > 0
