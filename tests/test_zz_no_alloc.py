"""The allocation-free density read-back (lbm_get_density_noalloc) against
lbm_get_density, called through the C interface: two calls in a row, the
second on a smaller box, each bit-identical to the allocating read-back (the
same kernel writes every value, the staging buffer alone differs); a box
beyond the fixed staging array is refused with the output untouched."""
import ctypes

import numpy as np
import pytest

import synth
from synth import BC_PERIODIC, Problem

lbm = pytest.importorskip("paper_1906_04722_amd.lbm")

pytestmark = pytest.mark.gpu


def _density_noalloc(t):
    out = np.full(2 * t.N, -7.0)
    rc = lbm.lib().lbm_get_density_noalloc(t.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return rc, out.reshape((2,) + t.shape)


def test_noalloc_density_matches_allocating_readback_twice():
    big = synth.c1_problem(seed=1)                    # 40^3 throat
    small = synth.small_throat_problem(n=24, seed=7)  # 24^3 throat, fewer nodes
    for prob, steps in ((big, 30), (small, 20)):
        t = lbm.Throat(prob)
        t.step(steps)
        ref = t.density()
        rc, got = _density_noalloc(t)
        print(f"box {prob.nx}x{prob.ny}x{prob.nz}, {steps} steps: rc {rc}", flush=True)
        assert rc == lbm.LBM_OK, lbm.lib().lbm_last_error()
        assert np.array_equal(got, ref)
        t.close()


def test_noalloc_density_refuses_a_box_beyond_the_staging_array():
    n = 130  # 130^3 = 2,197,000 nodes > 2^21
    b = 0.0609883
    p = Problem(nx=n, ny=n, nz=n, bc=(BC_PERIODIC,) * 3,
                rho_init=synth.flat_interface_density(n, n, n, n // 2, 2.0, b), rho_minor=b,
                G_ads=(0.0, 0.0))
    t = lbm.Throat(p)
    rc, got = _density_noalloc(t)
    assert rc == lbm.LBM_EINVAL
    assert np.all(got == -7.0)
    assert b"staging" in lbm.lib().lbm_last_error()
    t.close()
