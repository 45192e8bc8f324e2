"""ctypes binding of the C interface in include/lbm_abi.h (same names).

Argument marshalling only: every step of the method runs in the HIP library.
If the library is missing this module raises at load time; there is no
fallback path.
"""
import ctypes
import math
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsc_lbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ENONFINITE, LBM_ESTATE, LBM_EIO = \
    0, -1, -2, -3, -4, -5, -6
LBM_WNOTCONV = 1
LBM_BC_PERIODIC, LBM_BC_WALLS, LBM_BC_RESERVOIR = 0, 1, 2
LBM_NODE_FLUID, LBM_NODE_SOLID, LBM_NODE_RES_IN, LBM_NODE_RES_OUT = 0, 1, 2, 3
LBM_PT_CONVERGED, LBM_PT_NOT_CONVERGED, LBM_PT_NONFINITE, LBM_PT_NOT_RUN = 0, 1, 2, 3
LBM_WPARTIAL = 2
LBM_SCHED_NODE_LIST = -1

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_llp = ctypes.POINTER(ctypes.c_longlong)


class lbm_sphere(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double * 3), ("r", ctypes.c_double)]


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("bc", ctypes.c_int * 3),
        ("n_spheres", ctypes.c_int), ("spheres", ctypes.POINTER(lbm_sphere)),
        ("prism", ctypes.c_int), ("prism_ids", ctypes.c_int * 3),
        ("tau", ctypes.c_double * 2), ("G", ctypes.c_double), ("G_ads", ctypes.c_double * 2),
        ("rho_major", ctypes.c_double), ("rho_minor", ctypes.c_double),
        ("rho_in_nw", ctypes.c_double), ("rho_out_w", ctypes.c_double),
        ("rho_init", _dp), ("z_front", ctypes.c_int), ("probe", ctypes.c_int * 3),
        ("stream", ctypes.c_void_p),
    ]


class lbm_conv(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("check_every", ctypes.c_int),
                ("max_steps", ctypes.c_longlong), ("bisect_rel", ctypes.c_double)]


class lbm_drain_result(ctypes.Structure):
    _fields_ = [("pce", ctypes.c_double), ("pce_lo", ctypes.c_double),
                ("pce_hi", ctypes.c_double), ("invaded_at", ctypes.c_int),
                ("n_bisect", ctypes.c_int), ("total_steps", ctypes.c_longlong),
                ("S", _dp), ("steps", _llp), ("status", _ip), ("failed", ctypes.c_int)]


class lbm_batch_info(ctypes.Structure):
    _fields_ = [("tx", ctypes.c_int), ("ty", ctypes.c_int), ("lz", ctypes.c_int),
                ("n_tiles", ctypes.c_int), ("replays", ctypes.c_longlong),
                ("lattice_steps", ctypes.c_longlong), ("node_updates", ctypes.c_longlong),
                ("fluid_updates", ctypes.c_longlong), ("wall_ms", ctypes.c_double)]


# exported name -> (restype, argtypes)
SIGNATURES = {
    "lbm_throat_init": (ctypes.c_int, [ctypes.POINTER(lbm_params), ctypes.POINTER(ctypes.c_void_p)]),
    "lbm_throat_free": (None, [ctypes.c_void_p]),
    "lbm_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_longlong]),
    "lbm_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "lbm_set_rho_in": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "lbm_rho_in_for_pc": (ctypes.c_double, [ctypes.c_void_p, ctypes.c_double]),
    "lbm_nodes": (ctypes.c_longlong, [ctypes.c_void_p]),
    "lbm_get_types": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_ubyte)]),
    "lbm_get_populations": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "lbm_get_density": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "lbm_get_density_noalloc": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "lbm_reduce": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp]),
    "lbm_probe_invaded": (ctypes.c_int, [ctypes.c_void_p, _ip]),
    "lbm_drain_throat": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_int,
                                        ctypes.POINTER(lbm_conv),
                                        ctypes.POINTER(lbm_drain_result)]),
    "lbm_drain_batch": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(lbm_params), _dp, ctypes.c_int,
                                       ctypes.POINTER(lbm_conv), ctypes.POINTER(lbm_drain_result),
                                       ctypes.POINTER(lbm_batch_info)]),
    "lbm_drain_begin": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_int,
                                       ctypes.POINTER(lbm_conv)]),
    "lbm_drain_advance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_longlong, _ip]),
    "lbm_drain_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                     ctypes.POINTER(lbm_drain_result), _ip]),
    "lbm_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "lbm_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "lbm_time_steps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_longlong, _dp]),
    "lbm_set_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "lbm_get_schedule": (ctypes.c_int, [ctypes.c_void_p, _ip, _ip, _ip]),
    "lbm_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _ip, _ip, _ip]),
    "lbm_place": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp, _dp]),
    "lbm_bw_probe": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int, _dp]),
    "lbm_step_timer": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _llp]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_set_memory_budget": (ctypes.c_int, [ctypes.c_size_t]),
}

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class LBMError(RuntimeError):
    def __init__(self, code, what):
        msg = lib().lbm_last_error().decode(errors="replace")
        super().__init__(f"{what} failed with status {code}: {msg}")
        self.code = code


def _check(rc, what):
    if rc < 0:
        raise LBMError(rc, what)
    return rc


def _dptr(a):
    return a.ctypes.data_as(_dp)


def make_params(prob, stream=None):
    """lbm_params from a problem description (attributes of synth.Problem).
    Returns (params, keepalive) -- keep the second value alive while the
    params are in use."""
    sph = np.ascontiguousarray(np.asarray(prob.spheres, dtype=np.float64).reshape(-1, 4))
    n = sph.shape[0]
    arr = (lbm_sphere * max(n, 1))()
    for i in range(n):
        arr[i].c[0], arr[i].c[1], arr[i].c[2] = sph[i, 0], sph[i, 1], sph[i, 2]
        arr[i].r = sph[i, 3]
    P = lbm_params()
    P.nx, P.ny, P.nz = prob.nx, prob.ny, prob.nz
    P.bc[:] = list(prob.bc)
    P.n_spheres = n
    P.spheres = ctypes.cast(arr, ctypes.POINTER(lbm_sphere))
    P.prism = 1 if prob.prism_ids is not None else 0
    if prob.prism_ids is not None:
        P.prism_ids[:] = list(prob.prism_ids)
    P.tau[:] = list(prob.tau)
    P.G = prob.G
    P.G_ads[:] = list(prob.G_ads)
    P.rho_major, P.rho_minor = prob.rho_major, prob.rho_minor
    P.rho_in_nw, P.rho_out_w = prob.rho_in_nw, prob.rho_out_w
    rho0 = None
    if prob.rho_init is not None:
        rho0 = np.ascontiguousarray(prob.rho_init, dtype=np.float64)
        P.rho_init = _dptr(rho0)
    P.z_front = prob.z_front
    P.probe[:] = list(prob.probe) if prob.probe is not None else [-1, -1, -1]
    P.stream = stream
    return P, (arr, rho0)


class Throat:
    """One subdomain on the GPU (handle of lbm_throat_init)."""

    def __init__(self, prob, stream=None):
        self.prob = prob
        self.shape = (prob.nz, prob.ny, prob.nx)
        self.N = prob.nx * prob.ny * prob.nz
        P, keep = make_params(prob, stream)
        h = ctypes.c_void_p()
        _check(lib().lbm_throat_init(ctypes.byref(P), ctypes.byref(h)), "lbm_throat_init")
        self.h = h
        del keep

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.lbm_throat_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def step(self, n):
        _check(lib().lbm_step(self.h, int(n)), "lbm_step")

    def sync(self):
        _check(lib().lbm_sync(self.h), "lbm_sync")

    def set_rho_in(self, r):
        _check(lib().lbm_set_rho_in(self.h, float(r)), "lbm_set_rho_in")

    def rho_in_for_pc(self, pc):
        return lib().lbm_rho_in_for_pc(self.h, float(pc))

    def types(self):
        t = np.zeros(self.N, dtype=np.uint8)
        _check(lib().lbm_get_types(self.h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))),
               "lbm_get_types")
        return t.reshape(self.shape)

    def f(self):
        a = np.zeros(38 * self.N)
        _check(lib().lbm_get_populations(self.h, _dptr(a)), "lbm_get_populations")
        return a.reshape((2, 19) + self.shape)

    def density(self):
        a = np.zeros(2 * self.N)
        _check(lib().lbm_get_density(self.h, _dptr(a)), "lbm_get_density")
        return a.reshape((2,) + self.shape)

    def density_noalloc(self):
        """Densities through the allocation-free read-back (fixed staging array)."""
        a = np.zeros(2 * self.N)
        _check(lib().lbm_get_density_noalloc(self.h, _dptr(a)), "lbm_get_density_noalloc")
        return a.reshape((2,) + self.shape)

    def reduce(self):
        m = np.zeros(2)
        s = np.zeros(1)
        _check(lib().lbm_reduce(self.h, _dptr(m), _dptr(s)), "lbm_reduce")
        return m, float(s[0])

    def probe_invaded(self):
        v = ctypes.c_int(0)
        _check(lib().lbm_probe_invaded(self.h, ctypes.byref(v)), "lbm_probe_invaded")
        return bool(v.value)

    def drain(self, pc, tol=1e-6, check_every=100, max_steps=100000, bisect_rel=0.005):
        pc = np.ascontiguousarray(pc, dtype=np.float64)
        n = pc.size
        S = np.zeros(n)
        steps = np.zeros(n, dtype=np.int64)
        status = np.zeros(n, dtype=np.int32)
        c = lbm_conv(float(tol), int(check_every), int(max_steps), float(bisect_rel))
        r = lbm_drain_result()
        r.S = _dptr(S)
        r.steps = steps.ctypes.data_as(_llp)
        r.status = status.ctypes.data_as(_ip)
        rc = _check(lib().lbm_drain_throat(self.h, _dptr(pc), n, ctypes.byref(c), ctypes.byref(r)),
                    "lbm_drain_throat")
        return dict(S=S, steps=steps, status=status, pce=r.pce, pce_lo=r.pce_lo,
                    pce_hi=r.pce_hi, invaded_at=r.invaded_at, n_bisect=r.n_bisect,
                    total_steps=r.total_steps, warning=rc)

    def drain_begin(self, pc, tol=1e-6, check_every=100, max_steps=100000, bisect_rel=0.005):
        """Start the resumable drainage ramp (lbm_drain_begin)."""
        pc = np.ascontiguousarray(pc, dtype=np.float64)
        self._n_pc = pc.size
        c = lbm_conv(float(tol), int(check_every), int(max_steps), float(bisect_rel))
        _check(lib().lbm_drain_begin(self.h, _dptr(pc), pc.size, ctypes.byref(c)),
               "lbm_drain_begin")

    def drain_advance(self, max_steps):
        """Run the ramp for at most max_steps lattice steps; True once it has ended."""
        d = ctypes.c_int(0)
        _check(lib().lbm_drain_advance(self.h, int(max_steps), ctypes.byref(d)),
               "lbm_drain_advance")
        return bool(d.value)

    def drain_get(self, n_pc=None):
        """Results of the resumable ramp so far (dict as drain(), plus done)."""
        n = int(n_pc if n_pc is not None else self._n_pc)
        S = np.zeros(n)
        steps = np.zeros(n, dtype=np.int64)
        status = np.zeros(n, dtype=np.int32)
        r = lbm_drain_result()
        r.S = _dptr(S)
        r.steps = steps.ctypes.data_as(_llp)
        r.status = status.ctypes.data_as(_ip)
        d = ctypes.c_int(0)
        rc = _check(lib().lbm_drain_get(self.h, n, ctypes.byref(r), ctypes.byref(d)),
                    "lbm_drain_get")
        return dict(S=S, steps=steps, status=status, pce=r.pce, pce_lo=r.pce_lo,
                    pce_hi=r.pce_hi, invaded_at=r.invaded_at, n_bisect=r.n_bisect,
                    total_steps=r.total_steps, failed=bool(r.failed), warning=rc,
                    done=bool(d.value))

    def save(self, path):
        _check(lib().lbm_save(self.h, os.fsencode(path)), "lbm_save")

    def load(self, path, n_pc=None):
        _check(lib().lbm_load(self.h, os.fsencode(path)), "lbm_load")
        if n_pc is not None:
            self._n_pc = int(n_pc)

    def time_steps(self, n):
        ms = ctypes.c_double(0.0)
        _check(lib().lbm_time_steps(self.h, int(n), ctypes.byref(ms)), "lbm_time_steps")
        return ms.value

    def step_timer(self, enable=-1):
        """(ms, launches) of event-timed step launches inside drain(); enable
        1/0 resets and switches timing, -1 only reads."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_longlong(0)
        _check(lib().lbm_step_timer(self.h, int(enable), ctypes.byref(ms), ctypes.byref(n)),
               "lbm_step_timer")
        return ms.value, n.value

    def set_schedule(self, tx=0, ty=0, lz=0):
        _check(lib().lbm_set_schedule(self.h, int(tx), int(ty), int(lz)), "lbm_set_schedule")

    def autotune(self, trial_steps=20):
        """Pick the fastest launch shape for this subdomain (state unchanged)."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().lbm_autotune(self.h, int(trial_steps), ctypes.byref(a), ctypes.byref(b),
                                  ctypes.byref(c)), "lbm_autotune")
        return a.value, b.value, c.value

    def place(self, tries=2, trial_steps=4):
        """Try `tries` more placements of the population buffers and keep the
        fastest (lbm_place; state unchanged); returns (ms per step of the
        original pair, of the kept one)."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib().lbm_place(self.h, int(tries), int(trial_steps), ctypes.byref(a),
                               ctypes.byref(b)), "lbm_place")
        return a.value, b.value

    def schedule(self):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().lbm_get_schedule(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "lbm_get_schedule")
        return a.value, b.value, c.value


def drain_batch(probs, pcs, tol=1e-6, check_every=100, max_steps=100000, bisect_rel=0.005):
    """Batched drainage of many subdomains (lbm_drain_batch).  probs: list of
    problem descriptions; pcs: array [n][n_pc].  Returns (list of result
    dicts like Throat.drain, info dict)."""
    n = len(probs)
    pcs = np.ascontiguousarray(pcs, dtype=np.float64).reshape(n, -1)
    n_pc = pcs.shape[1]
    P = (lbm_params * n)()
    keep = []
    for i, pr in enumerate(probs):
        P[i], k = make_params(pr)
        keep.append(k)
    S = np.zeros((n, n_pc))
    steps = np.zeros((n, n_pc), dtype=np.int64)
    status = np.zeros((n, n_pc), dtype=np.int32)
    R = (lbm_drain_result * n)()
    for i in range(n):
        R[i].S = S[i].ctypes.data_as(_dp)
        R[i].steps = steps[i].ctypes.data_as(_llp)
        R[i].status = status[i].ctypes.data_as(_ip)
    c = lbm_conv(float(tol), int(check_every), int(max_steps), float(bisect_rel))
    info = lbm_batch_info()
    rc = _check(lib().lbm_drain_batch(n, P, _dptr(pcs), n_pc, ctypes.byref(c), R,
                                      ctypes.byref(info)), "lbm_drain_batch")
    out = [dict(S=S[i], steps=steps[i], status=status[i], pce=R[i].pce, pce_lo=R[i].pce_lo,
                pce_hi=R[i].pce_hi, invaded_at=R[i].invaded_at, n_bisect=R[i].n_bisect,
                total_steps=R[i].total_steps, failed=bool(R[i].failed)) for i in range(n)]
    inf = dict(tx=info.tx, ty=info.ty, lz=info.lz, n_tiles=info.n_tiles, replays=info.replays,
               lattice_steps=info.lattice_steps, node_updates=info.node_updates,
               fluid_updates=info.fluid_updates, wall_ms=info.wall_ms, warning=rc)
    del keep
    return out, inf


def set_memory_budget(nbytes):
    """Refuse allocating calls that would need more than nbytes of device
    memory (0: no budget)."""
    _check(lib().lbm_set_memory_budget(int(nbytes)), "lbm_set_memory_budget")


def bw_probe(nbytes=4 << 30, reps=20):
    """Achievable copy bandwidth in GB/s (read + write)."""
    v = ctypes.c_double(0.0)
    _check(lib().lbm_bw_probe(int(nbytes), int(reps), ctypes.byref(v)), "lbm_bw_probe")
    return v.value


def nan_safe(x):
    return None if x is None or (isinstance(x, float) and math.isnan(x)) else x
