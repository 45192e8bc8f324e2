"""Host-side checks of the HIP library that need no GPU: it loads, exports
every entry point that the headers under include/ declare, and the Python
bindings name the same set."""
import ctypes
import os
import re

from paper_1906_04722_amd import lbm, network, surrogate

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src))
    return names


def test_header_declares_the_boundary_calls():
    names = declared_entry_points()
    for must in ("lbm_throat_init", "lbm_step", "lbm_drain_throat", "lbm_throat_free",
                 "lbm_get_populations", "lbm_reduce", "lbm_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(lbm.LIB_PATH)
    missing = [n for n in sorted(declared_entry_points()) if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    bound = [set(lbm.SIGNATURES), set(surrogate.SIGNATURES), set(network.SIGNATURES)]
    assert declared_entry_points() == set().union(*bound)
    assert sum(len(b) for b in bound) == len(set().union(*bound))


def test_surrogate_arguments_rejected_without_gpu_work():
    L = surrogate.lib()
    h = ctypes.c_void_p()
    assert L.lbm_surrogate_create(0, 1, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    assert L.lbm_surrogate_create(17, 1, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    assert b"members" in L.lbm_last_error()
    assert L.lbm_surrogate_predict(None, 1, None, None, None) == lbm.LBM_EINVAL
    assert L.lbm_surrogate_members(None) == 0
    L.lbm_surrogate_free(None)
    # a throat sphere of zero radius is refused before any device work (the
    # MS-P scale of the targets needs positive radii)
    import numpy as np
    import synth
    pr = synth.c1_problem()
    pr.spheres = np.array(pr.spheres, dtype=np.float64)
    pr.spheres[pr.prism_ids[0], 3] = 0.0
    P, keep = surrogate._params_array([pr])
    feat = np.zeros((1, surrogate.NFEAT))
    r = np.zeros(1)
    assert L.lbm_surrogate_describe(1, P, surrogate._d(feat), surrogate._d(r)) == lbm.LBM_EINVAL
    assert b"radius" in L.lbm_last_error()
    del keep


def test_invalid_arguments_rejected_without_gpu_work():
    """Validation runs before any device call: bad sizes and relaxation
    times are refused with LBM_EINVAL and a message."""
    L = lbm.lib()
    import synth
    p = synth.c1_problem()
    P, keep = lbm.make_params(p)
    P.tau[0] = 0.5
    h = ctypes.c_void_p()
    rc = L.lbm_throat_init(ctypes.byref(P), ctypes.byref(h))
    assert rc == lbm.LBM_EINVAL
    assert b"tau" in L.lbm_last_error()
    P.tau[0] = 1.0
    P.nx = 2
    assert L.lbm_throat_init(ctypes.byref(P), ctypes.byref(h)) == lbm.LBM_EINVAL
    # the three-plane pull offsets of the brick storage are 32-bit: at most
    # 9,418,786 nodes per z-plane once nx and ny are padded to multiples of 8
    # and 4 (here 4000 x 3000 x 3 nodes; 3065 x 3073 pads to 3072 x 3076)
    P.nx, P.ny, P.nz = 3065, 3073, 3
    assert L.lbm_throat_init(ctypes.byref(P), ctypes.byref(h)) == lbm.LBM_EINVAL
    assert b"plane" in L.lbm_last_error()
    P.nx, P.ny, P.nz = 4000, 3000, 3
    assert L.lbm_throat_init(ctypes.byref(P), ctypes.byref(h)) == lbm.LBM_EINVAL
    assert b"plane" in L.lbm_last_error()
    P.nx, P.ny, P.nz = 40, 40, 40
    P.bc[0] = lbm.LBM_BC_RESERVOIR
    assert L.lbm_throat_init(ctypes.byref(P), ctypes.byref(h)) == lbm.LBM_EINVAL
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    a, b = ctypes.c_double(-1.0), ctypes.c_double(-1.0)
    assert L.lbm_place(None, 2, 4, ctypes.byref(a), ctypes.byref(b)) == lbm.LBM_EINVAL
    assert (a.value, b.value) == (-1.0, -1.0)
    L.lbm_throat_free(None)
    del keep


def _batch_args(probs, pcs, conv=(1e-6, 100, 1000, 0.005)):
    import numpy as np
    n = len(probs)
    P = (lbm.lbm_params * n)()
    keep = []
    for i, pr in enumerate(probs):
        P[i], k = lbm.make_params(pr)
        keep.append(k)
    pcs = np.ascontiguousarray(pcs, dtype=np.float64)
    n_pc = pcs.shape[1]
    S = np.full((n, n_pc), -7.0)
    steps = np.full((n, n_pc), -7, dtype=np.int64)
    status = np.full((n, n_pc), -7, dtype=np.int32)
    R = (lbm.lbm_drain_result * n)()
    for i in range(n):
        R[i].pce = R[i].pce_lo = R[i].pce_hi = -7.0
        R[i].S = S[i].ctypes.data_as(lbm._dp)
        R[i].steps = steps[i].ctypes.data_as(lbm._llp)
        R[i].status = status[i].ctypes.data_as(lbm._ip)
    c = lbm.lbm_conv(*conv)
    return P, pcs, c, R, (S, steps, status), keep


def test_drain_batch_arguments_refused_with_outputs_untouched():
    """lbm_drain_batch validates everything before any device call: a
    non-increasing or non-positive ramp, an odd check interval and a missing
    probe are refused with LBM_EINVAL, and no output is written."""
    import numpy as np
    import synth
    L = lbm.lib()
    probs = [synth.small_throat_problem(seed=3), synth.small_throat_problem(seed=4)]
    good = np.array([[0.002, 0.01], [0.002, 0.01]])
    cases = [
        (good * np.array([[1.0, -1.0], [1.0, 1.0]]), (1e-6, 100, 1000, 0.005), b"increasing"),
        (good * np.array([[0.0, 1.0], [1.0, 1.0]]), (1e-6, 100, 1000, 0.005), b"positive"),
        (good[:, ::-1].copy(), (1e-6, 100, 1000, 0.005), b"increasing"),
        (good, (1e-6, 99, 1000, 0.005), b"check_every"),
        (good, (0.0, 100, 1000, 0.005), b"tol"),
        (good, (1e-6, 100, 10, 0.005), b"max_steps"),
    ]
    for pcs, conv, msg in cases:
        P, pcs_a, c, R, outs, keep = _batch_args(probs, pcs, conv)
        rc = L.lbm_drain_batch(2, P, lbm._dptr(pcs_a), pcs_a.shape[1], ctypes.byref(c), R, None)
        assert rc == lbm.LBM_EINVAL, (pcs, conv)
        assert msg in L.lbm_last_error(), L.lbm_last_error()
        for a in outs:
            assert np.all(a == -7)
        assert all(R[i].pce == -7.0 and R[i].pce_lo == -7.0 for i in range(2))
    # a subdomain without a probe node cannot be classified
    probs[1].probe = None
    P, pcs_a, c, R, outs, keep = _batch_args(probs, good)
    assert L.lbm_drain_batch(2, P, lbm._dptr(pcs_a), 2, ctypes.byref(c), R, None) == lbm.LBM_EINVAL
    assert b"probe" in L.lbm_last_error()


def test_memory_budget_refuses_before_any_allocation():
    """With a device-memory budget set, a subdomain or a batch that needs more
    is refused with LBM_ENOMEM before any device call (this host has no GPU:
    any device call would fail with LBM_EHIP instead), and the handle stays
    unset; budget 0 lifts the limit again."""
    import numpy as np
    import synth
    L = lbm.lib()
    p = synth.c1_problem()
    P, keep = lbm.make_params(p)
    h = ctypes.c_void_p(12345)
    try:
        assert L.lbm_set_memory_budget(1 << 20) == lbm.LBM_OK   # 1 MiB: below a 40^3 box
        assert L.lbm_throat_init(ctypes.byref(P), ctypes.byref(h)) == lbm.LBM_ENOMEM
        assert b"budget" in L.lbm_last_error()
        assert h.value == 12345
        probs = [synth.small_throat_problem(seed=3), synth.small_throat_problem(seed=4)]
        Pb, pcs_a, c, R, outs, keepb = _batch_args(probs, np.array([[0.002, 0.01]] * 2))
        rc = L.lbm_drain_batch(2, Pb, lbm._dptr(pcs_a), 2, ctypes.byref(c), R, None)
        assert rc == lbm.LBM_ENOMEM
        assert b"budget" in L.lbm_last_error()
        for a in outs:
            assert np.all(a == -7)
    finally:
        L.lbm_set_memory_budget(0)
    del keep


def test_checkpoint_and_resumable_ramp_refuse_bad_arguments():
    """lbm_save / lbm_load / lbm_drain_advance / lbm_drain_get refuse a NULL
    handle or path before any device call."""
    L = lbm.lib()
    assert L.lbm_save(None, b"/tmp/x.lbm") == lbm.LBM_EINVAL
    assert L.lbm_load(None, b"/tmp/x.lbm") == lbm.LBM_EINVAL
    assert L.lbm_drain_advance(None, 100, None) == lbm.LBM_EINVAL
    r = lbm.lbm_drain_result()
    assert L.lbm_drain_get(None, 1, ctypes.byref(r), None) == lbm.LBM_EINVAL
    assert L.lbm_drain_begin(None, None, 1, None) == lbm.LBM_EINVAL
