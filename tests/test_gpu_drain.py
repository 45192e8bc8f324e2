"""Drainage ramp (a pressure-controlled sequence of steady states with
bisection of the entry pressure) on the GPU against the FP64 oracle, and the
ramp's invariants at the full 96^3 size.

Bars (spec tolerances): saturation within 1e-3 at every ramp point,
p_c^e midpoints within 1 %, the same first invaded point."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

CONV = dict(tol=1e-5, check_every=100, max_steps=6000, bisect_rel=0.02)


def _small_c2():
    p = synth.c2_problem(n=40, mean_r=32.0 * 40 / 96)
    r_ins, _ = synth.throat_incircle(p.spheres)
    return p, synth.pc_ramp(synth.GAMMA_LAPLACE, r_ins, 5, 0.1, 0.7)


def test_drain_parity_small_throat():
    from paper_1906_04722_amd import lbm
    p, pcs = _small_c2()
    go = lbm.Throat(p).drain(pcs, **CONV)
    oo = oracle.Oracle(p).drain(pcs, **CONV)
    print("GPU", go["S"], go["pce"], go["invaded_at"], "oracle", oo["S"], oo["pce"],
          oo["invaded_at"])
    assert go["invaded_at"] == oo["invaded_at"] >= 0
    assert np.array_equal(go["steps"], oo["steps"])
    assert np.abs(go["S"] - oo["S"]).max() <= 1e-3
    assert abs(go["pce"] - oo["pce"]) <= 0.01 * oo["pce"]


def test_full_size_ramp_invariants():
    """96^3 throat: saturation never rises along a drainage ramp, invasion
    happens once and stays, and the bisected entry pressure lies inside the
    first invaded ramp interval."""
    from paper_1906_04722_amd import lbm
    p = synth.c2_problem()
    r_ins, _ = synth.throat_incircle(p.spheres)
    pcs = synth.pc_ramp(synth.GAMMA_LAPLACE, r_ins, 8, 0.1, 0.8)
    g = lbm.Throat(p)
    out = g.drain(pcs, tol=1e-6, check_every=100, max_steps=8000, bisect_rel=0.01)
    S = out["S"]
    print("S", S, "pce", out["pce"], out["pce_lo"], out["pce_hi"], "at", out["invaded_at"])
    assert np.all(np.diff(S) <= 2e-3)
    i = out["invaded_at"]
    assert i >= 1
    lo = pcs[i - 1]
    assert lo <= out["pce_lo"] < out["pce_hi"] <= pcs[i]
    assert (out["pce_hi"] - out["pce_lo"]) / out["pce_hi"] <= 0.01
    assert g.probe_invaded()
