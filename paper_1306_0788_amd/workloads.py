"""Seeded synthetic inputs and the named workloads.

This module holds no arithmetic of the method: it only draws initial
densities, particle positions, chains and bonds, and records the parameter
sets of the workloads.  Both the GPU path and the oracle receive the same
arrays from here.

Recipe (the paper's simulations are its own synthetic set-ups; there is no
dataset):
  * densities: rho_A, rho_B = 1 + 0.01 * (2U - 1), independent per site and
    component, U uniform from numpy's Philox bit generator with the
    workload's seed -- a slightly perturbed 50/50 mixture, the starting point
    of spinodal decomposition;
  * free particles: uniform in the box, rejected while closer than `min_dist`
    to an earlier one (periodic minimum image);
  * chains: random walks of fixed bond length 0.97 started at uniform points,
    each new bead rejected while closer than `min_dist` to a bead already
    placed that is not its bonded predecessor; a chain that gets stuck is
    removed and restarted elsewhere;
  * emulsion jobs (serving): cubic box L = round(exp(U[ln 32, ln 128])),
    non-overlapping A droplets (periodic distance > r1 + r2 + 2) with radius
    U[4, 12] until the droplet volume reaches a fraction U[0.1, 0.3];
    G_AB = U[1.6, 2.2]; rho_A = b + (a - b) s, rho_B = b + (a - b)(1 - s)
    between the bulk coexistence densities a > b of that G_AB (total
    density 2; `coexistence`) with the smooth indicator
    s = (1 - tanh((d - R)/2))/2 of the nearest droplet;
    log-uniform 100..10,000 particles uniform in the box, kappa_A = -0.05
    (drawn to the A droplets), gamma = 1, m = 100; 500 steps; arrivals a
    Poisson stream of 20 jobs/s.
"""
import math

import numpy as np

WCA_CUT = 2.0 ** (1.0 / 6.0)

# Parameter sets.  "shape" = (nx, ny, nz); G is the 2x2 coupling matrix.
# "onset" is the first step at which a density reaches zero when the set-up
# starts from its seeded uniform mixture (G_AB = 1.8 is 1.8 times the spinodal
# coupling of the rho = 1 mixture with the paper's forcing; with the velocity
# shift the spinodal is at G rho = (tau - 1/2)/tau, so G_AB = 1.6 is 3.2 times
# it; the decomposition overshoots the coexistence densities and drains the
# minority component), as measured for these seeds; None where the run length
# stays below it.
WORKLOADS = {
    # 32^3 FP64, velocity-shift forcing, 64 free particles, friction only.
    "c1": dict(shape=(32, 32, 32), precision="fp64", forcing="shift", tau=(1.0, 1.0),
               G=((0.0, 1.6), (1.6, 0.0)), gamma=0.5, kT=0.0, seed=1,
               kappa=((0.0, 0.0),), mass=(1.0,), charge=(0.0,),
               particles=dict(kind="free", n=64, min_dist=0.0), wca=None, fene=None, dh=None,
               steps=100, onset=35),
    # 128^3 FP32 spinodal decomposition with 20,000 solvated WCA particles.
    "c2": dict(shape=(128, 128, 128), precision="fp32", forcing="paper", tau=(1.0, 1.0),
               G=((0.0, 1.8), (1.8, 0.0)), gamma=1.0, kT=0.0, seed=2,
               kappa=((0.05, 0.0),), mass=(100.0,), charge=(0.0,),
               particles=dict(kind="free", n=20000, min_dist=WCA_CUT), wca=(1.0, 1.0), fene=None,
               dh=None, steps=2000, onset=117),
    # 256^3 FP32 polyelectrolyte-like mixture: 2,000 chains x 100 beads,
    # FENE + WCA + screened Debye-Hueckel, fluctuating fluid.
    "c3": dict(shape=(256, 256, 256), precision="fp32", forcing="paper", tau=(1.0, 1.0),
               G=((0.0, 1.8), (1.8, 0.0)), gamma=1.0, kT=1e-4, seed=3,
               kappa=((0.1, 0.0),), mass=(2000.0,), charge=(1.0,),
               particles=dict(kind="chains", nchains=2000, nbeads=100, bond=0.97, min_dist=WCA_CUT),
               wca=(1.0, 1.0), fene=(30.0, 1.5), dh=(1.0, 3.0, 1.0), steps=1000, onset=87),
    # The 128^3 spinodal set-up at 256^3 (same particle number density:
    # 160,000 particles), plain FP32 storage.
    "c2_256": dict(shape=(256, 256, 256), precision="fp32", forcing="paper", tau=(1.0, 1.0),
                   G=((0.0, 1.8), (1.8, 0.0)), gamma=1.0, kT=0.0, seed=6,
                   kappa=((0.05, 0.0),), mass=(100.0,), charge=(0.0,),
                   particles=dict(kind="free", n=160000, min_dist=WCA_CUT), wca=(1.0, 1.0),
                   fene=None, dh=None, steps=200, onset=117),
    # The same at G_AB = 1.4 (still phase separating, no density reaches
    # zero within 1,000 steps): the long comparison of the storage forms.
    "c2_256_g14": dict(shape=(256, 256, 256), precision="fp32", forcing="paper", tau=(1.0, 1.0),
                       G=((0.0, 1.4), (1.4, 0.0)), gamma=1.0, kT=0.0, seed=6,
                       kappa=((0.05, 0.0),), mass=(100.0,), charge=(0.0,),
                       particles=dict(kind="free", n=160000, min_dist=WCA_CUT), wca=(1.0, 1.0),
                       fene=None, dh=None, steps=1000, onset=None),
}


def rng(seed):
    return np.random.Generator(np.random.Philox(seed))


def initial_densities(shape, seed, amp=0.01, mean=1.0):
    """[2][nz][ny][nx] float64: mean + amp*(2U-1) per site and component."""
    nx, ny, nz = shape
    g = rng(seed)
    return mean + amp * (2.0 * g.random((2, nz, ny, nx)) - 1.0)


def _too_close_grid(points, box, min_dist):
    """Cell hash for rejection sampling; returns (insert, check, remove)."""
    cell = max(min_dist, 1e-9)
    ncell = [max(1, int(math.floor(b / cell))) for b in box]
    grid = {}

    def key(p):
        return tuple(int(math.floor(p[a] / box[a] * ncell[a])) % ncell[a] for a in range(3))

    def insert(i, p):
        grid.setdefault(key(p), []).append(i)

    def remove(i, p):
        grid[key(p)].remove(i)

    def check(p, ignore=()):
        if min_dist <= 0.0:
            return False
        k = key(p)
        rng_ = [range(-1, 2) if ncell[a] >= 3 else range(0, ncell[a]) for a in range(3)]
        for dx in rng_[0]:
            for dy in rng_[1]:
                for dz in rng_[2]:
                    kk = ((k[0] + dx) % ncell[0], (k[1] + dy) % ncell[1], (k[2] + dz) % ncell[2])
                    for j in grid.get(kk, ()):
                        if j in ignore:
                            continue
                        d = points[j] - p
                        d -= np.asarray(box) * np.floor(d / np.asarray(box) + 0.5)
                        if d @ d < min_dist * min_dist:
                            return True
        return False

    return insert, check, remove


def free_particles(n, shape, seed, min_dist=0.0, max_tries=1000):
    """n positions uniform in the periodic box [0,nx)x[0,ny)x[0,nz)."""
    g = rng(seed + 1000003)
    box = np.asarray(shape, dtype=np.float64)
    if min_dist <= 0.0:
        return g.random((n, 3)) * box
    pts = np.zeros((n, 3))
    insert, check, _ = _too_close_grid(pts, box, min_dist)
    for i in range(n):
        for _ in range(max_tries):
            p = g.random(3) * box
            if not check(p):
                break
        else:
            raise RuntimeError("could not place particle %d" % i)
        pts[i] = p
        insert(i, p)
    return pts


def chains(nchains, nbeads, shape, seed, bond=0.97, min_dist=WCA_CUT, max_tries=200, max_restarts=100):
    """Random-walk chains.  Returns positions [nchains*nbeads][3] (wrapped into
    the box) and bonds [nchains*(nbeads-1)][2] (int32).  A chain whose next
    bead cannot be placed is removed and started again elsewhere, so no two
    non-bonded beads end up closer than min_dist."""
    g = rng(seed + 2000003)
    box = np.asarray(shape, dtype=np.float64)
    n = nchains * nbeads
    pts = np.zeros((n, 3))
    insert, check, remove = _too_close_grid(pts, box, min_dist)
    bonds = []
    for c in range(nchains):
        base = c * nbeads
        for _ in range(max_restarts):
            placed = 0
            p = None
            for _ in range(max_tries):
                p = g.random(3) * box
                if not check(p):
                    break
            else:
                continue
            pts[base] = p
            insert(base, p)
            placed = 1
            for b in range(1, nbeads):
                prev = pts[base + b - 1]
                for _ in range(max_tries):
                    d = g.normal(size=3)
                    d *= bond / np.linalg.norm(d)
                    p = np.mod(prev + d, box)
                    if not check(p, ignore=(base + b - 1,)):
                        break
                else:
                    break
                pts[base + b] = p
                insert(base + b, p)
                placed += 1
            if placed == nbeads:
                break
            for b in range(placed):
                remove(base + b, pts[base + b])
        else:
            raise RuntimeError("could not place chain %d" % c)
        bonds.extend((base + b - 1, base + b) for b in range(1, nbeads))
    return pts, np.asarray(bonds, dtype=np.int32).reshape(-1, 2)


def particles_for(w, shape=None):
    """Particles of workload dict `w` (optionally re-scaled to another box at
    the same number density).  Returns (x, bonds or None)."""
    shape = tuple(shape or w["shape"])
    spec = w["particles"]
    scale = np.prod(shape) / np.prod(w["shape"])
    if spec["kind"] == "free":
        n = int(round(spec["n"] * scale))
        return free_particles(n, shape, w["seed"], spec["min_dist"]), None
    nch = max(1, int(round(spec["nchains"] * scale)))
    return chains(nch, spec["nbeads"], shape, w["seed"], spec["bond"], spec["min_dist"])


def coexistence(G, total=2.0):
    """Bulk coexistence densities (a, b), a > b, a + b = total, of a symmetric
    two-component mixture with coupling G between the components: the
    non-trivial root of equal chemical potentials of the bulk free energy
    (Sec. 2, Eq. fbulk), ln(a / b) = G (a - b), by Newton's method.  Used
    only to lay out initial densities; the time step never calls it."""
    if G * total <= 2.0:
        return total / 2, total / 2  # below the spinodal: the mixture is stable
    a = 0.999 * total
    for _ in range(200):
        F = math.log(a / (total - a)) - G * (2.0 * a - total)
        dF = 1.0 / a + 1.0 / (total - a) - 2.0 * G
        a = min(max(a - F / dF, total / 2 + 1e-12), total * (1 - 1e-15))
    return a, total - a


def emulsion_job(seed, index):
    """Parameters and inputs of serving job `index` of stream `seed`:
    dict(shape, G, rho [2][N], x [n][3], kappa, gamma, mass, steps)."""
    g = rng(seed * 1000003 + index)
    L = int(round(math.exp(g.uniform(math.log(32.0), math.log(128.0)))))
    target = g.uniform(0.1, 0.3) * L ** 3
    cs = np.zeros((0, 3))
    rs = np.zeros(0)
    vol = 0.0
    for _ in range(10000):
        if vol >= target:
            break
        R = g.uniform(4.0, 12.0)
        c = g.random(3) * L
        d = cs - c
        d -= L * np.round(d / L)
        if np.all(np.sqrt((d * d).sum(axis=1)) >= rs + R + 2.0):
            cs = np.vstack([cs, c])
            rs = np.append(rs, R)
            vol += 4.0 / 3.0 * math.pi * R ** 3
    centres, radii = list(cs), list(rs)
    s = np.zeros((L, L, L))
    for c, R in zip(centres, radii):
        # the indicator is below 1e-5 beyond R + 12: work on the wrapped box
        h = int(math.ceil(R + 12.0))
        idx, off = [], []
        for a in range(3):
            i0 = int(math.floor(c[a])) - h
            raw = np.arange(i0, i0 + 2 * h + 2)
            if len(raw) > L:
                raw = np.arange(L)
            idx.append(np.mod(raw, L))
            d = raw - c[a]
            off.append(d - L * np.round(d / L))
        dz, dy, dx = np.meshgrid(off[2], off[1], off[0], indexing="ij")
        ind = 0.5 * (1.0 - np.tanh((np.sqrt(dx * dx + dy * dy + dz * dz) - R) / 2.0))
        sub = np.ix_(idx[2], idx[1], idx[0])
        s[sub] = np.maximum(s[sub], ind)
    n = int(round(math.exp(g.uniform(math.log(100.0), math.log(10000.0)))))
    G = float(g.uniform(1.6, 2.2))
    a, b = coexistence(G)
    rho = np.stack([b + (a - b) * s, b + (a - b) * (1.0 - s)]).reshape(2, -1)
    return dict(shape=(L, L, L), G=G, rho=rho, x=g.random((n, 3)) * L,
                kappa=(-0.05, 0.0), gamma=1.0, mass=100.0, steps=500, droplets=len(radii))


def poisson_arrivals(n, rate, seed):
    """Arrival times (s) of n jobs of a Poisson stream of the given rate."""
    return np.cumsum(rng(seed + 7).exponential(1.0 / rate, n))
