"""ctypes binding of include/lbm_surrogate.h (same names).

Argument marshalling only: descriptors, training, inference and the LBM
fallback all run in the HIP library; there is no other path.
"""
import ctypes

import numpy as np

from . import lbm

NFEAT, NOUT, NCURVE, NPARAM = 80, 17, 16, 156689
MAX_BATCH, MAX_MEMBERS = 4096, 16

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int)


class lbm_sg_train_cfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_double),
                ("lr_min_frac", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("seed", ctypes.c_ulonglong), ("bootstrap", ctypes.c_int)]


class lbm_sg_info(ctypes.Structure):
    _fields_ = [("n_fallback", ctypes.c_int), ("describe_ms", ctypes.c_double),
                ("predict_ms", ctypes.c_double), ("lbm_ms", ctypes.c_double),
                ("lbm", lbm.lbm_batch_info)]


SIGNATURES = {
    "lbm_surrogate_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_ulonglong, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_void_p)]),
    "lbm_surrogate_free": (None, [ctypes.c_void_p]),
    "lbm_surrogate_members": (ctypes.c_int, [ctypes.c_void_p]),
    "lbm_surrogate_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _fp]),
    "lbm_surrogate_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _fp]),
    "lbm_surrogate_set_stats": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp, _dp]),
    "lbm_surrogate_get_stats": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp, _dp]),
    "lbm_surrogate_describe": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(lbm.lbm_params), _dp,
                                              _dp]),
    "lbm_surrogate_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _fp]),
    "lbm_surrogate_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _fp, _dp]),
    "lbm_surrogate_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _dp,
                                           ctypes.POINTER(lbm_sg_train_cfg), _ip, _dp]),
    "lbm_surrogate_predict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]),
    "lbm_surrogate_pce": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                         ctypes.POINTER(lbm.lbm_params), _dp, ctypes.c_int,
                                         ctypes.POINTER(lbm.lbm_conv), ctypes.c_double,
                                         ctypes.c_int, _dp, _dp, _dp, _ip,
                                         ctypes.POINTER(lbm_sg_info)]),
}

_ready = False


def lib():
    global _ready
    L = lbm.lib()
    if not _ready:
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _ready = True
    return L


def _d(a):
    return a.ctypes.data_as(_dp)


def _f(a):
    return a.ctypes.data_as(_fp)


def _c64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _params_array(probs, stream=None):
    P = (lbm.lbm_params * len(probs))()
    keep = []
    for i, pr in enumerate(probs):
        P[i], k = lbm.make_params(pr, stream)
        keep.append(k)
    return P, keep


def describe(probs, with_scale=False):
    """Descriptors [n][80] of four-sphere throat problems (on the GPU), and
    with with_scale=True also the targets' scale [n]: the MS-P corner-meniscus
    radius at entry in lattice units (NaN where there is none)."""
    n = len(probs)
    out = np.zeros((n, NFEAT))
    r_msp = np.zeros(n)
    if n > 0:
        P, keep = _params_array(probs)
        lbm._check(lib().lbm_surrogate_describe(n, P, _d(out), _d(r_msp)),
                   "lbm_surrogate_describe")
        del keep
    return (out, r_msp) if with_scale else out


class Surrogate:
    """Ensemble handle (lbm_surrogate_create)."""

    def __init__(self, members=5, seed=0, stream=None):
        h = ctypes.c_void_p()
        lbm._check(lib().lbm_surrogate_create(int(members), int(seed), stream, ctypes.byref(h)),
                   "lbm_surrogate_create")
        self.h = h
        self.members = int(members)

    def close(self):
        if self.h:
            lib().lbm_surrogate_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, member, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == NPARAM
        lbm._check(lib().lbm_surrogate_set_params(self.h, int(member), _f(w)),
                   "lbm_surrogate_set_params")

    def get_params(self, member):
        w = np.zeros(NPARAM, dtype=np.float32)
        lbm._check(lib().lbm_surrogate_get_params(self.h, int(member), _f(w)),
                   "lbm_surrogate_get_params")
        return w

    def set_stats(self, xmu, xsd, tmu, tsd):
        a = [_c64(v) for v in (xmu, xsd, tmu, tsd)]
        lbm._check(lib().lbm_surrogate_set_stats(self.h, *[_d(v) for v in a]),
                   "lbm_surrogate_set_stats")

    def get_stats(self):
        a = [np.zeros(NFEAT), np.zeros(NFEAT), np.zeros(NOUT), np.zeros(NOUT)]
        lbm._check(lib().lbm_surrogate_get_stats(self.h, *[_d(v) for v in a]),
                   "lbm_surrogate_get_stats")
        return tuple(a)

    def forward(self, xs):
        xs = _c64(xs).reshape(-1, NFEAT)
        y = np.zeros((self.members, xs.shape[0], NOUT), dtype=np.float32)
        lbm._check(lib().lbm_surrogate_forward(self.h, xs.shape[0], _d(xs), _f(y)),
                   "lbm_surrogate_forward")
        return y

    def grad(self, xs, ts):
        xs = _c64(xs).reshape(-1, NFEAT)
        ts = _c64(ts).reshape(-1, NOUT)
        g = np.zeros((self.members, NPARAM), dtype=np.float32)
        loss = np.zeros(self.members)
        lbm._check(lib().lbm_surrogate_grad(self.h, xs.shape[0], _d(xs), _d(ts), _f(g), _d(loss)),
                   "lbm_surrogate_grad")
        return g, loss

    def train(self, feat, target, epochs, batch=128, lr=1e-3, lr_min_frac=0.0, beta1=0.9,
              beta2=0.999, eps=1e-8, seed=0, bootstrap=True, order=None):
        feat = _c64(feat).reshape(-1, NFEAT)
        target = _c64(target).reshape(-1, NOUT)
        n = feat.shape[0]
        cfg = lbm_sg_train_cfg(int(epochs), int(batch), float(lr), float(lr_min_frac),
                               float(beta1), float(beta2), float(eps), int(seed),
                               1 if bootstrap else 0)
        op = None
        if order is not None:
            order = np.ascontiguousarray(order, dtype=np.int32)
            assert order.shape == (epochs, self.members, n)
            op = order.ctypes.data_as(_ip)
        hist = np.zeros(int(epochs))
        lbm._check(lib().lbm_surrogate_train(self.h, n, _d(feat), _d(target), ctypes.byref(cfg),
                                             op, _d(hist)), "lbm_surrogate_train")
        return hist

    def predict(self, feat):
        feat = _c64(feat).reshape(-1, NFEAT)
        n = feat.shape[0]
        mean = np.zeros((n, NOUT))
        std = np.zeros((n, NOUT))
        lbm._check(lib().lbm_surrogate_predict(self.h, n, _d(feat), _d(mean), _d(std)),
                   "lbm_surrogate_predict")
        return mean, std

    def pce(self, probs, pcs, threshold=0.02, run_fallback=True, tol=1e-6, check_every=100,
            max_steps=100000, bisect_rel=0.005):
        """Entry pressures of throat problems; returns (dict of arrays, info dict)."""
        n = len(probs)
        pcs = _c64(pcs).reshape(n, -1)
        P, keep = _params_array(probs)
        c = lbm.lbm_conv(float(tol), int(check_every), int(max_steps), float(bisect_rel))
        pce = np.zeros(n)
        curve = np.zeros((n, NCURVE))
        pstd = np.zeros(n)
        used = np.zeros(n, dtype=np.int32)
        info = lbm_sg_info()
        rc = lbm._check(lib().lbm_surrogate_pce(self.h, n, P, _d(pcs), pcs.shape[1],
                                                ctypes.byref(c), float(threshold),
                                                1 if run_fallback else 0, _d(pce), _d(curve),
                                                _d(pstd), used.ctypes.data_as(_ip),
                                                ctypes.byref(info)), "lbm_surrogate_pce")
        del keep
        inf = dict(n_fallback=info.n_fallback, describe_ms=info.describe_ms,
                   predict_ms=info.predict_ms, lbm_ms=info.lbm_ms, lbm_wall_ms=info.lbm.wall_ms,
                   lbm_fluid_updates=info.lbm.fluid_updates, warning=rc)
        return dict(pce=pce, curve=curve, pce_std=pstd, used_fallback=used.astype(bool)), inf


def training_set(probs, drains):
    """Descriptors and targets of drained throats (lbm_drain_batch results):
    features [m][80] from the GPU descriptor, targets [m][17] = (p_c^e times
    the MS-P radius, the 16 ramp saturations), and the mask of the throats
    kept (those whose ramp found the entry pressure and that have an MS-P
    radius)."""
    F, r_msp = describe(probs, with_scale=True)
    pce = np.array([d["pce"] for d in drains], dtype=np.float64)
    S = np.stack([np.asarray(d["S"], dtype=np.float64) for d in drains])
    if S.shape[1] != NCURVE:
        raise ValueError(f"the surrogate's curve has {NCURVE} points, the drains {S.shape[1]}")
    ok = np.isfinite(pce) & (r_msp > 0)
    T = np.column_stack([pce * r_msp, S])
    return F[ok], T[ok], ok
