"""Failure handling of the batched drainage: a subdomain whose state becomes
non-finite (here a cohesion strength G = 3, far past the model's stable
range, so that its densities overflow within the first check interval) stops
with its failure flagged, while the subdomains beside it in the same launches
finish and equal their single drains bit for bit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

CONV = dict(tol=1e-5, check_every=50, max_steps=1000, bisect_rel=0.05)


def test_one_non_finite_subdomain_is_flagged_and_the_others_finish():
    from paper_1906_04722_amd import lbm
    good = [synth.small_throat_problem(n=24, seed=3), synth.small_throat_problem(n=28, seed=5)]
    bad = synth.small_throat_problem(n=24, seed=4)
    bad.G = 3.0
    probs = [good[0], bad, good[1]]
    pcs = np.array([[0.002, 0.006, 0.012]] * 3)
    print("batch of 3 subdomains, the middle one with G = 3", flush=True)
    outs, info = lbm.drain_batch(probs, pcs, **CONV)
    print("warning", info["warning"], "results", outs, flush=True)
    assert info["warning"] == lbm.LBM_WPARTIAL
    f = outs[1]
    assert f["failed"]
    assert np.all(f["status"] == lbm.LBM_PT_NONFINITE)
    assert np.isnan(f["pce"]) and np.isnan(f["pce_lo"]) and np.isnan(f["pce_hi"])
    for p, pc, b in ((good[0], pcs[0], outs[0]), (good[1], pcs[2], outs[2])):
        assert not b["failed"]
        s = lbm.Throat(p).drain(pc, **CONV)
        assert np.all(b["status"] != lbm.LBM_PT_NOT_RUN)
        assert np.array_equal(s["S"], b["S"])
        assert np.array_equal(s["steps"], b["steps"])
        assert np.array_equal(s["status"], b["status"])
        assert s["invaded_at"] == b["invaded_at"] and s["total_steps"] == b["total_steps"]
        assert np.array_equal([s["pce"], s["pce_lo"], s["pce_hi"]],
                              [b["pce"], b["pce_lo"], b["pce_hi"]], equal_nan=True)


def test_single_drain_of_a_non_finite_throat_is_an_error():
    from paper_1906_04722_amd import lbm
    bad = synth.small_throat_problem(n=24, seed=4)
    bad.G = 3.0
    t = lbm.Throat(bad)
    with pytest.raises(lbm.LBMError) as e:
        t.drain(np.array([0.002, 0.006]), **CONV)
    assert e.value.code == lbm.LBM_ENONFINITE
