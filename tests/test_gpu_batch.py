"""Batched drainage (one fused-step launch over the tiles of all throats,
device-side ramp and bisection, graph replays) against the single-throat
drainage of each throat: the same kernels and reduction order, so every
result is bit-identical."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

CONV = dict(tol=1e-5, check_every=100, max_steps=3000, bisect_rel=0.02)


def _throats():
    probs, pcs = [], []
    for n, seed in ((32, 11), (40, 12), (36, 13), (28, 14)):
        p = synth.c2_problem(n=n, mean_r=32.0 * n / 96, seed=seed)
        r_ins, _ = synth.throat_incircle(p.spheres)
        probs.append(p)
        pcs.append(synth.pc_ramp(synth.GAMMA_LAPLACE, r_ins, 5, 0.1, 0.9))
    return probs, np.array(pcs)


def test_batch_equals_single_throat_drains():
    from paper_1906_04722_amd import lbm
    probs, pcs = _throats()
    outs, info = lbm.drain_batch(probs, pcs, **CONV)
    print("batch info", info)
    assert info["n_tiles"] > 0 and info["replays"] > 0
    for p, pc, b in zip(probs, pcs, outs):
        s = lbm.Throat(p).drain(pc, **CONV)
        print("single", s["S"], s["pce"], s["invaded_at"], "batch", b["S"], b["pce"],
              b["invaded_at"])
        assert np.array_equal(s["S"], b["S"])
        assert np.array_equal(s["steps"], b["steps"])
        assert np.array_equal(s["status"], b["status"])
        assert s["invaded_at"] == b["invaded_at"]
        assert s["n_bisect"] == b["n_bisect"]
        assert s["total_steps"] == b["total_steps"]
        if s["invaded_at"] >= 0:
            assert s["pce"] == b["pce"] and s["pce_lo"] == b["pce_lo"] and s["pce_hi"] == b["pce_hi"]
        else:
            assert np.isnan(b["pce"])


def test_batch_rejects_bad_arguments():
    from paper_1906_04722_amd import lbm
    probs, pcs = _throats()
    with pytest.raises(lbm.LBMError):
        lbm.drain_batch(probs[:2], pcs[:2, ::-1], **CONV)  # decreasing ramp
    with pytest.raises(lbm.LBMError):
        lbm.drain_batch(probs[:2], pcs[:2], tol=1e-5, check_every=99, max_steps=3000,
                        bisect_rel=0.02)  # odd chunk
