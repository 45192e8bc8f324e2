"""The paper's example throat, three equal touching spheres in their prism
(Sec. 2.2.2): the figure's values are not given, so its entry pressure is
held to the band the geometry fixes (below the incircle estimate of a
perfectly wetting throat and within a few tens of percent of it), and the
ramp to the ordering invasion must show."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_three_sphere_entry_pressure_in_band():
    from paper_1906_04722_amd import estimators as est
    from paper_1906_04722_amd import lbm
    R = 16.0
    p = synth.three_sphere_throat(R)
    g = lbm.Throat(p)
    r_in = est.incircle_radius(R)
    pcs = synth.pc_ramp(synth.GAMMA_LAPLACE, r_in, 20, lo=0.3, hi=1.2)
    out = g.drain(pcs, tol=1e-6, check_every=100, max_steps=40000, bisect_rel=0.005)
    g.close()
    star = est.pc_star(out["pce"], R, synth.GAMMA_LAPLACE)
    inc = 4.0 * R / r_in
    msp = 2.0 * R / est.msp_radius(R)
    print("p_e* =", star, "incircle", inc, "MS-P", msp, "S", out["S"])
    assert 0.6 * inc < star < inc
    # the bracket is tight and lies inside the ramp
    assert (out["pce_hi"] - out["pce_lo"]) / out["pce_hi"] <= 0.005
    i = out["invaded_at"]
    assert 0 < i < len(pcs) and pcs[i - 1] <= out["pce_lo"] <= out["pce_hi"] <= pcs[i]
    # saturation only falls along the ramp, and invasion is one jump
    S = out["S"]
    assert np.all(np.diff(S) <= 1e-4)
    jumps = -np.diff(S)
    assert jumps.argmax() == i - 1 and jumps.max() > 0.2
    assert np.sort(jumps)[-2] < 0.05
