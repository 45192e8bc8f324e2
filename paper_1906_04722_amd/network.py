"""ctypes binding of include/lbm_network.h (same name): argument marshalling
only; the drainage runs in the native library."""
import ctypes

import numpy as np

from . import lbm

INLET, OUTLET = -1, -2
WETTING, INVADED, TRAPPED = 0, 1, 2

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)

SIGNATURES = {
    "lbm_network_drain": (ctypes.c_int, [ctypes.c_int, _dp, ctypes.c_int, _ip, _dp, ctypes.c_int,
                                         _dp, _dp, _ip, _ip]),
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


def drain(pore_vol, throats, pce, pressures):
    """Quasi-static drainage of a pore network (lbm_network_drain).  Returns
    (wetting saturation per pressure, pressure index of each pore's invasion
    or -1, final state per pore)."""
    vol = np.ascontiguousarray(pore_vol, dtype=np.float64)
    th = np.ascontiguousarray(np.asarray(throats).reshape(-1, 2), dtype=np.int32)
    pc = np.ascontiguousarray(pce, dtype=np.float64)
    p = np.ascontiguousarray(pressures, dtype=np.float64)
    sw = np.zeros(len(p))
    inv = np.zeros(len(vol), dtype=np.int32)
    st = np.zeros(len(vol), dtype=np.int32)
    lbm._check(lib().lbm_network_drain(len(vol), vol.ctypes.data_as(_dp), len(th),
                                       th.ctypes.data_as(_ip), pc.ctypes.data_as(_dp), len(p),
                                       p.ctypes.data_as(_dp), sw.ctypes.data_as(_dp),
                                       inv.ctypes.data_as(_ip), st.ctypes.data_as(_ip)),
               "lbm_network_drain")
    return sw, inv, st
