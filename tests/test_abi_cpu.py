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
    L.lbm_throat_free(None)
    del keep
