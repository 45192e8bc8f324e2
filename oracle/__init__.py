"""FP64 CPU oracle of the two-component Shan-Chen LBM and its drainage ramp.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library; the ctypes wrapper below only marshals arguments to the
plain C implementation in sc_oracle.c.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libsc_oracle.so")
_lib = None

FLUID, SOLID, RES_IN, RES_OUT = 0, 1, 2, 3
CONVERGED, NOT_CONVERGED = 0, 1


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int), ("bc_z", ctypes.c_int),
        ("n_spheres", ctypes.c_int), ("spheres", ctypes.POINTER(ctypes.c_double)),
        ("prism", ctypes.c_int), ("prism_ids", ctypes.c_int * 3),
        ("tau", ctypes.c_double * 2), ("G", ctypes.c_double), ("G_ads", ctypes.c_double * 2),
        ("rho_major", ctypes.c_double), ("rho_minor", ctypes.c_double),
        ("rho_in_nw", ctypes.c_double), ("rho_out_w", ctypes.c_double),
        ("rho_init", ctypes.POINTER(ctypes.c_double)), ("z_front", ctypes.c_int),
        ("probe", ctypes.c_int * 3),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, dp, ip, llp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), \
            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_longlong)
        L.orc_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(vp)]
        L.orc_free.argtypes = [vp]
        L.orc_free.restype = None
        L.orc_clone.argtypes = [vp, ctypes.POINTER(vp)]
        L.orc_copy_state.argtypes = [vp, vp]
        L.orc_step.argtypes = [vp, ctypes.c_longlong]
        L.orc_set_rho_in.argtypes = [vp, ctypes.c_double]
        L.orc_rho_in_for_pc.argtypes = [vp, ctypes.c_double]
        L.orc_rho_in_for_pc.restype = ctypes.c_double
        L.orc_nodes.argtypes = [vp]
        L.orc_nodes.restype = ctypes.c_longlong
        L.orc_get_types.argtypes = [vp, ctypes.POINTER(ctypes.c_ubyte)]
        for name in ("orc_get_f", "orc_set_f", "orc_get_density", "orc_get_force",
                     "orc_get_velocity", "orc_get_pressure"):
            getattr(L, name).argtypes = [vp, dp]
        L.orc_reduce.argtypes = [vp, dp, dp, dp]
        L.orc_probe_invaded.argtypes = [vp]
        L.orc_drain.argtypes = [vp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                ctypes.c_longlong, ctypes.c_double, dp, llp, ip, dp, ip]
        L.orc_lattice.argtypes = [ip, dp, ip]
        L.orc_lattice.restype = None
        L.orc_feq.argtypes = [ctypes.c_double, dp, dp]
        L.orc_feq.restype = None
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice():
    """(e [19][3] int, w [19] float, opp [19] int) as tabulated by the oracle."""
    e = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    o = np.zeros(19, dtype=np.int32)
    lib().orc_lattice(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dptr(w),
                      o.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return e, w, o


def feq(rho, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(19)
    lib().orc_feq(float(rho), _dptr(u), _dptr(out))
    return out


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


class Oracle:
    """One FP64 subdomain run built from a problem description (an object with
    the attributes of synth.Problem)."""

    def __init__(self, prob, _handle=None):
        self.prob = prob
        self.shape = (prob.nz, prob.ny, prob.nx)
        self.N = prob.nx * prob.ny * prob.nz
        if _handle is not None:
            self.h = _handle
            return
        sph = np.ascontiguousarray(np.asarray(prob.spheres, dtype=np.float64).reshape(-1, 4))
        self._sph = sph
        rho0 = None if prob.rho_init is None else np.ascontiguousarray(prob.rho_init, np.float64)
        self._rho0 = rho0
        P = _Params()
        P.nx, P.ny, P.nz = prob.nx, prob.ny, prob.nz
        P.bc_x, P.bc_y, P.bc_z = prob.bc
        P.n_spheres = sph.shape[0]
        P.spheres = _dptr(sph) if sph.shape[0] else None
        P.prism = 1 if prob.prism_ids is not None else 0
        if prob.prism_ids is not None:
            P.prism_ids[:] = list(prob.prism_ids)
        P.tau[:] = list(prob.tau)
        P.G = prob.G
        P.G_ads[:] = list(prob.G_ads)
        P.rho_major, P.rho_minor = prob.rho_major, prob.rho_minor
        P.rho_in_nw, P.rho_out_w = prob.rho_in_nw, prob.rho_out_w
        P.rho_init = _dptr(rho0) if rho0 is not None else None
        P.z_front = prob.z_front
        P.probe[:] = list(prob.probe) if prob.probe is not None else [-1, -1, -1]
        h = ctypes.c_void_p()
        _check(lib().orc_create(ctypes.byref(P), ctypes.byref(h)), "orc_create")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.orc_free(h)
            self.h = None

    def clone(self):
        h = ctypes.c_void_p()
        _check(lib().orc_clone(self.h, ctypes.byref(h)), "orc_clone")
        return Oracle(self.prob, _handle=h)

    def step(self, n):
        _check(lib().orc_step(self.h, int(n)), "orc_step")

    def set_rho_in(self, r):
        _check(lib().orc_set_rho_in(self.h, float(r)), "orc_set_rho_in")

    def rho_in_for_pc(self, pc):
        return lib().orc_rho_in_for_pc(self.h, float(pc))

    def types(self):
        t = np.zeros(self.N, dtype=np.uint8)
        _check(lib().orc_get_types(self.h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))),
               "orc_get_types")
        return t.reshape(self.shape)

    def _get(self, fn, ncomp):
        a = np.zeros(ncomp * self.N)
        _check(getattr(lib(), fn)(self.h, _dptr(a)), fn)
        return a

    def f(self):
        """Pre-collision populations [2][19][nz][ny][nx]."""
        return self._get("orc_get_f", 38).reshape((2, 19) + self.shape)

    def set_f(self, f):
        a = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        _check(lib().orc_set_f(self.h, _dptr(a)), "orc_set_f")

    def density(self):
        return self._get("orc_get_density", 2).reshape((2,) + self.shape)

    def force(self):
        return self._get("orc_get_force", 6).reshape((2, 3) + self.shape)

    def velocity(self):
        return self._get("orc_get_velocity", 3).reshape((3,) + self.shape)

    def pressure(self):
        return self._get("orc_get_pressure", 1).reshape(self.shape)

    def reduce(self):
        """(masses [2], wetting saturation, total momentum [3]) over fluid nodes."""
        m = np.zeros(2)
        s = np.zeros(1)
        p = np.zeros(3)
        _check(lib().orc_reduce(self.h, _dptr(m), _dptr(s), _dptr(p)), "orc_reduce")
        return m, float(s[0]), p

    def probe_invaded(self):
        r = lib().orc_probe_invaded(self.h)
        if r < 0:
            raise OracleError("no probe node")
        return bool(r)

    def drain(self, pc, tol=1e-6, check_every=100, max_steps=100000, bisect_rel=0.005):
        pc = np.ascontiguousarray(pc, dtype=np.float64)
        n = pc.size
        S = np.zeros(n)
        steps = np.zeros(n, dtype=np.int64)
        status = np.zeros(n, dtype=np.int32)
        pce = np.zeros(3)
        inv = ctypes.c_int(-1)
        rc = lib().orc_drain(self.h, _dptr(pc), n, float(tol), int(check_every), int(max_steps),
                             float(bisect_rel), _dptr(S),
                             steps.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                             status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dptr(pce),
                             ctypes.byref(inv))
        _check(rc, "orc_drain")
        return dict(S=S, steps=steps, status=status, pce_lo=pce[0], pce=pce[1], pce_hi=pce[2],
                    invaded_at=inv.value)
