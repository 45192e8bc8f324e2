"""What the trained surrogate gains over the method without it.

Throats of one seeded packing are drained by the batched LBM and the ensemble
is trained on them on the GPU; on throats of another packing its entry
pressures are compared with the plain LBM's.  The network must beat the
no-network estimate (the training mean of p_c^e times the MS-P radius, over
the throat's MS-P radius: the Mayer-Stowe-Princen estimate calibrated on the
training throats, itself within about 10 % at these resolutions), and
answering from it must cost a small fraction of the LBM time it replaces."""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

CONV = dict(tol=1e-6, check_every=100, max_steps=800, bisect_rel=0.01)


def _throats(seed, n):
    probs, rins, _ = synth.packing_throats(n_throats=n, n_spheres=300, seed=seed, res=10.0,
                                           side_range=(24, 48), amp=0)
    return probs, np.array([synth.pc_ramp(synth.GAMMA_LAPLACE, r, 16) for r in rins])


def test_network_beats_no_network_estimate():
    from paper_1906_04722_amd import lbm, surrogate
    tr, tr_pc = _throats(21, 256)
    te, te_pc = _throats(22, 96)
    drains, _ = lbm.drain_batch(tr, tr_pc, **CONV)
    F, T, kept = surrogate.training_set(tr, drains)
    assert kept.mean() > 0.5
    m = surrogate.Surrogate(members=5, seed=3)
    hist = m.train(F, T, epochs=150, batch=64, lr=1e-3, seed=4)
    assert hist[-1] < 0.1 * hist[0]
    t0 = time.perf_counter()
    ref, _ = lbm.drain_batch(te, te_pc, **CONV)
    t_lbm = time.perf_counter() - t0
    pref = np.array([r["pce"] for r in ref])
    t0 = time.perf_counter()
    out, info = m.pce(te, te_pc, threshold=1e9, run_fallback=False)
    t_net = time.perf_counter() - t0
    _, r_msp = surrogate.describe(te, with_scale=True)
    ok = np.isfinite(pref) & np.isfinite(r_msp)
    err = np.abs(out["pce"][ok] - pref[ok]) / pref[ok]
    base = np.abs(T[:, 0].mean() / r_msp[ok] - pref[ok]) / pref[ok]
    print("network median err", np.median(err), "no-network", np.median(base),
          "time net", t_net, "lbm", t_lbm)
    assert np.median(err) < np.median(base)
    assert info["n_fallback"] == 0
    assert t_net < 0.1 * t_lbm
