"""ctypes binding of the lbmd C ABI (include/lbmd.h).

Argument marshalling only: every step of the method runs in liblbmd.so on
the GPU.  Loading fails loudly if the library has not been built
(``python -m paper_1306_0788_amd.build``).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "liblbmd.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5
FP64, FP32, FP16DEV, BF16DEV = 0, 1, 2, 3
FORCE_PAPER, FORCE_SHIFT = 0, 1
KERNEL_FUSED, KERNEL_TWOPASS, KERNEL_AUTO, KERNEL_PUSH = 0, 1, 2, 3
RHO, U, POP = 1, 2, 4
PAIR_WCA, PAIR_DH, BOND_FENE = 0, 1, 2
MAX_TYPES = 8

EXPORTS = ["lbmd_create", "lbmd_destroy", "lbmd_set_particles", "lbmd_set_particle_types",
           "lbmd_set_pair_potential", "lbmd_set_bonds", "lbmd_step", "lbmd_sync", "lbmd_get_fields",
           "lbmd_get_particles", "lbmd_set_populations", "lbmd_reductions", "lbmd_get_step",
           "lbmd_last_error", "lbmd_set_tiling", "lbmd_kernel_timing", "lbmd_organisation", "lbmd_set_graph",
           "lbmd_autotune", "lbmd_batch_create", "lbmd_batch_destroy", "lbmd_batch_attach", "lbmd_batch_detach",
           "lbmd_batch_step", "lbmd_batch_poll", "lbmd_batch_last_error", "lbmd_set_solvation_lambda",
           "lbmd_set_mrt", "lbmd_stream_ceiling", "lbmd_get_state", "lbmd_set_state",
           "lbmd_get_fields_noalloc"]


class LbmdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lbmd error %d: %s" % (code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("forcing", ctypes.c_int32), ("kernel", ctypes.c_int32),
        ("tau", ctypes.c_double * 2), ("G", (ctypes.c_double * 2) * 2),
        ("gamma", ctypes.c_double), ("kappa", ctypes.c_double * 2), ("mass", ctypes.c_double),
        ("kT", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("check_every", ctypes.c_int32), ("reserved", ctypes.c_int32), ("rho0", ctypes.c_double),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)


def load():
    """Load liblbmd.so; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError("liblbmd.so is not built: run `python -m paper_1306_0788_amd.build` "
                           "(there is no fallback path)")
    # torch ships its own HIP runtime under the same soname as the system one
    # liblbmd.so links (libamdhip64.so.7); whichever is loaded first serves
    # the whole process, and torch fails on a runtime other than its own.
    # Loading torch first makes both use torch's.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIBPATH)
    H = ctypes.c_void_p
    L.lbmd_create.argtypes = [ctypes.POINTER(Params), _D, ctypes.c_void_p, ctypes.POINTER(H)]
    L.lbmd_destroy.argtypes = [H]
    L.lbmd_set_particles.argtypes = [H, ctypes.c_int64, _D, _D, _I32]
    L.lbmd_set_particle_types.argtypes = [H, ctypes.c_int32, _D, _D, _D]
    L.lbmd_set_pair_potential.argtypes = [H, ctypes.c_int32, _D]
    L.lbmd_set_solvation_lambda.argtypes = [H, ctypes.c_int32, _D]
    L.lbmd_set_mrt.argtypes = [H, ctypes.c_int32] + [ctypes.c_double] * 4
    L.lbmd_set_bonds.argtypes = [H, ctypes.c_int64, _I32]
    L.lbmd_step.argtypes = [H, ctypes.c_int64]
    L.lbmd_sync.argtypes = [H]
    L.lbmd_get_fields.argtypes = [H, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int32]
    L.lbmd_get_particles.argtypes = [H, _D, _D, _D, _D]
    L.lbmd_set_populations.argtypes = [H, _D]
    L.lbmd_reductions.argtypes = [H, _D, ctypes.POINTER(ctypes.c_int64)]
    L.lbmd_get_step.argtypes = [H]
    L.lbmd_get_step.restype = ctypes.c_int64
    L.lbmd_last_error.argtypes = [H]
    L.lbmd_last_error.restype = ctypes.c_char_p
    L.lbmd_set_tiling.argtypes = [H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.lbmd_kernel_timing.argtypes = [H, ctypes.c_int32, _D, ctypes.POINTER(ctypes.c_int64)]
    L.lbmd_organisation.argtypes = [H]
    L.lbmd_stream_ceiling.argtypes = [H, ctypes.c_int32, _D]
    L.lbmd_set_graph.argtypes = [H, ctypes.c_int32]
    L.lbmd_autotune.argtypes = [H, ctypes.c_int32, ctypes.c_char_p, _I32, _D]
    L.lbmd_get_fields_noalloc.argtypes = [H, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int32]
    L.lbmd_get_state.argtypes = [H, ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]
    L.lbmd_set_state.argtypes = [H, ctypes.c_void_p, ctypes.c_size_t]
    L.lbmd_batch_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(H)]
    L.lbmd_batch_destroy.argtypes = [H]
    L.lbmd_batch_attach.argtypes = [H, H, ctypes.c_int64, _I32]
    L.lbmd_batch_detach.argtypes = [H, ctypes.c_int32]
    L.lbmd_batch_step.argtypes = [H, ctypes.c_int64]
    L.lbmd_batch_poll.argtypes = [H, ctypes.POINTER(ctypes.c_int64), _I32]
    L.lbmd_batch_last_error.argtypes = [H]
    L.lbmd_batch_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("lbmd_get_step", "lbmd_last_error", "lbmd_batch_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Sim:
    """One simulation handle.  Parameters follow lbmd_params."""

    def __init__(self, shape, precision=FP32, forcing=FORCE_PAPER, kernel=KERNEL_AUTO, tau=(1.0, 1.0),
                 G=((0.0, 1.6), (1.6, 0.0)), gamma=0.0, kappa=(0.0, 0.0), mass=1.0, kT=0.0, seed=0,
                 check_every=0, rho_init=None, stream=None, rho0=1.0):
        L = load()
        p = Params()
        p.nx, p.ny, p.nz = (int(s) for s in shape)
        p.precision, p.forcing, p.kernel = precision, forcing, kernel
        p.tau[0], p.tau[1] = tau
        for a in range(2):
            for b in range(2):
                p.G[a][b] = G[a][b]
        p.gamma = gamma
        p.kappa[0], p.kappa[1] = kappa
        p.mass, p.kT, p.seed, p.check_every = mass, kT, seed, check_every
        p.rho0 = rho0
        self.shape = tuple(int(s) for s in shape)
        self.N = int(np.prod(self.shape))
        self.params = p
        rho = None if rho_init is None else _f64(rho_init, (2, self.N))
        self._h = ctypes.c_void_p()
        rc = L.lbmd_create(ctypes.byref(p), _dp(rho), ctypes.c_void_p(stream or 0), ctypes.byref(self._h))
        if rc != OK:
            raise LbmdError(rc, "lbmd_create failed")
        self.np = 0

    def _check(self, rc):
        if rc != OK:
            raise LbmdError(rc, load().lbmd_last_error(self._h).decode())
        return rc

    def close(self):
        if self._h:
            load().lbmd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_particles(self, pos, vel=None, type_=None):
        pos = _f64(pos).reshape(-1, 3)
        n = pos.shape[0]
        vel = None if vel is None else _f64(vel, (n, 3))
        t = None if type_ is None else np.ascontiguousarray(type_, np.int32)
        self._check(load().lbmd_set_particles(self._h, n, _dp(pos), _dp(vel),
                                              None if t is None else t.ctypes.data_as(_I32)))
        self.np = n

    def set_particle_types(self, kappa, mass, charge=None):
        kappa = _f64(kappa).reshape(-1, 2)
        mass = _f64(mass)
        charge = None if charge is None else _f64(charge)
        self._check(load().lbmd_set_particle_types(self._h, kappa.shape[0], _dp(kappa), _dp(mass), _dp(charge)))

    def set_mrt(self, lambdas=None):
        """lambdas = (bulk, shear, momentum, kinetic) eigenvalues, or None for BGK."""
        if lambdas is None:
            self._check(load().lbmd_set_mrt(self._h, 0, 0.0, 0.0, 0.0, 0.0))
        else:
            self._check(load().lbmd_set_mrt(self._h, 1, *[float(v) for v in lambdas]))

    def set_solvation_lambda(self, lambdas):
        """lambdas: per-type (lambda_A, lambda_B) of the fluid solvation force."""
        lam = _f64(lambdas, (len(lambdas), 2)) if len(lambdas) else None
        self._check(load().lbmd_set_solvation_lambda(self._h, len(lambdas), _dp(lam)))

    def set_pair_potential(self, kind, params):
        q = None if params is None else _f64(params)
        self._check(load().lbmd_set_pair_potential(self._h, kind, _dp(q)))

    def set_bonds(self, pairs):
        b = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
        self._check(load().lbmd_set_bonds(self._h, b.shape[0], b.ctypes.data_as(_I32)))

    def set_tiling(self, tile_y, tile_z, hold=1, xcd=0, nt=1):
        flags = (1 if hold else 0) | (2 if xcd else 0) | (4 if nt else 0)
        self._check(load().lbmd_set_tiling(self._h, tile_y, tile_z, flags))

    def step(self, n=1):
        return self._check(load().lbmd_step(self._h, n))

    def step_rc(self, n=1):
        return load().lbmd_step(self._h, n)

    def sync(self):
        return load().lbmd_sync(self._h)

    def get_fields(self, mask):
        n = 0
        if mask & RHO:
            n += 2 * self.N
        if mask & U:
            n += 3 * self.N
        if mask & POP:
            n += 38 * self.N
        out = np.empty(n)
        self._check(load().lbmd_get_fields(self._h, mask, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def get_fields_device(self, mask, out_ptr):
        """Write fields into device memory at out_ptr (e.g. a torch tensor's data_ptr())."""
        self._check(load().lbmd_get_fields(self._h, mask, ctypes.c_void_p(out_ptr), 1))

    def get_fields_noalloc(self, mask, out_ptr=None):
        """lbmd_get_fields_noalloc: into a new host array, or into device
        memory at out_ptr."""
        if out_ptr is not None:
            self._check(load().lbmd_get_fields_noalloc(self._h, mask, ctypes.c_void_p(out_ptr), 1))
            return None
        n = (2 * self.N if mask & RHO else 0) + (3 * self.N if mask & U else 0) + (38 * self.N if mask & POP else 0)
        out = np.empty(n)
        self._check(load().lbmd_get_fields_noalloc(self._h, mask, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def rho(self):
        return self.get_fields(RHO).reshape(2, self.N)

    def velocity(self):
        return self.get_fields(U).reshape(3, self.N)

    def populations(self):
        return self.get_fields(POP).reshape(2, 19, self.N)

    def set_populations(self, pop):
        pop = _f64(pop, (2, 19, self.N))
        self._check(load().lbmd_set_populations(self._h, _dp(pop)))

    def particles(self):
        n = self.np
        x, v, F, Fc = (np.empty((n, 3)) for _ in range(4))
        self._check(load().lbmd_get_particles(self._h, _dp(x), _dp(v), _dp(F), _dp(Fc)))
        return x, v, F, Fc

    def get_state(self):
        """The dynamic state (populations in stored form, particles, step
        index) as an opaque uint8 array (lbmd_get_state)."""
        n = ctypes.c_size_t(0)
        self._check(load().lbmd_get_state(self._h, None, ctypes.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        rc = load().lbmd_get_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n))
        if rc not in (OK, EUNSTABLE):
            self._check(rc)
        return buf[:n.value]

    def set_state(self, buf):
        """Replace the dynamic state with one from get_state (lbmd_set_state)."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(load().lbmd_set_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))
        self.np = int(np.frombuffer(buf[32:40].tobytes(), dtype=np.int64)[0])  # particle count in the blob header

    def reductions(self):
        out = np.empty(8)
        st = ctypes.c_int64()
        self._check(load().lbmd_reductions(self._h, _dp(out), ctypes.byref(st)))
        return out, st.value

    def status(self):
        return load().lbmd_sync(self._h)

    def last_error(self):
        return load().lbmd_last_error(self._h).decode()

    def kernel_timing(self, enable):
        """(total ms, launches) of the collide-stream kernel since timing was last enabled."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(load().lbmd_kernel_timing(self._h, int(enable), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def stream_ceiling(self, reps=10):
        """Average ms of one pass that moves the collide-stream kernel's bytes
        (38 pulled loads and 38 stores per site) with no arithmetic."""
        ms = ctypes.c_double()
        self._check(load().lbmd_stream_ceiling(self._h, int(reps), ctypes.byref(ms)))
        return ms.value

    def set_graph(self, enable=True):
        """Advance steps two at a time by replaying captured HIP graphs."""
        self._check(load().lbmd_set_graph(self._h, int(enable)))

    def autotune(self, reps=3, cache_path=None):
        """Time every candidate tiling of the fluid passes on the current state
        (not advanced) and keep the fastest.  Returns (tile_y, tile_z, flags, ms)."""
        ch = np.zeros(3, dtype=np.int32)
        ms = ctypes.c_double()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(load().lbmd_autotune(self._h, reps, path, ch.ctypes.data_as(_I32), ctypes.byref(ms)))
        return int(ch[0]), int(ch[1]), int(ch[2]), ms.value

    def organisation(self):
        """KERNEL_FUSED or KERNEL_TWOPASS: the organisation of the next step."""
        return load().lbmd_organisation(self._h)

    @property
    def step_index(self):
        return load().lbmd_get_step(self._h)


EMPTY, RUNNING, DONE, FAILED = 0, 1, 2, 3


class Batch:
    """A multi-lattice batch: attached Sim handles advance together
    (lbmd_batch_* in include/lbmd.h)."""

    def __init__(self, max_jobs=32, noise=False, stream=None):
        L = load()
        self._h = ctypes.c_void_p()
        rc = L.lbmd_batch_create(max_jobs, int(bool(noise)), ctypes.c_void_p(stream or 0), ctypes.byref(self._h))
        if rc != OK:
            raise LbmdError(rc, "lbmd_batch_create failed")
        self.max_jobs = max_jobs
        self.jobs = {}

    def _check(self, rc):
        if rc != OK:
            raise LbmdError(rc, load().lbmd_batch_last_error(self._h).decode())
        return rc

    def attach(self, sim, nsteps):
        slot = ctypes.c_int32()
        self._check(load().lbmd_batch_attach(self._h, sim._h, nsteps, ctypes.byref(slot)))
        self.jobs[slot.value] = sim
        return slot.value

    def detach(self, slot):
        self._check(load().lbmd_batch_detach(self._h, slot))
        return self.jobs.pop(slot)

    def step(self, n=1):
        self._check(load().lbmd_batch_step(self._h, n))

    def poll(self):
        """(steps[max_jobs], state[max_jobs]) with state EMPTY/RUNNING/DONE/FAILED."""
        steps = np.empty(self.max_jobs, dtype=np.int64)
        state = np.empty(self.max_jobs, dtype=np.int32)
        self._check(load().lbmd_batch_poll(self._h, steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           state.ctypes.data_as(_I32)))
        return steps, state

    def close(self):
        if self._h:
            load().lbmd_batch_destroy(self._h)
            self._h = ctypes.c_void_p()
            self.jobs = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
