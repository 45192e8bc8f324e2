"""Hybrid assembly on the GPU: the throats of a small packing's pore network
drained by the batched LBM, their entry pressures assembled by the native
network drainage, checked against the reference rules on the same entry
pressures."""
import numpy as np
import pytest

import synth
from oracle import network as ref
from synth import network as net_geo

pytestmark = pytest.mark.gpu


def test_network_of_lbm_throats():
    from paper_1906_04722_amd import lbm, network
    x, r, L, _, _ = synth.dense_packing(12, seed=7)
    nw = net_geo.pore_network(x, r, L)
    probs, r_lu, scale, r_unit = net_geo.throat_problems(nw, res=8.0, side_range=(20, 40))
    idx = [i for i, p in enumerate(probs) if p is not None]
    pcs = np.array([synth.pc_ramp(synth.GAMMA_LAPLACE, r_lu[i], 16) for i in idx])
    drains, _ = lbm.drain_batch([probs[i] for i in idx], pcs, tol=1e-5, check_every=100,
                                max_steps=600, bisect_rel=0.02)
    pce = np.full(len(probs), np.inf)
    got = 0
    for i, d in zip(idx, drains):
        if np.isfinite(d["pce"]):
            pce[i] = d["pce"] * scale[i] / synth.GAMMA_LAPLACE
            got += 1
            assert d["pce_lo"] < d["pce_hi"] and d["pce_lo"] > 0
    assert got > len(idx) // 2
    p = np.linspace(0.5 * pce[np.isfinite(pce)].min(), pce[np.isfinite(pce)].max(), 10)
    sw, inv, st = network.drain(nw["pore_vol"], nw["throats"], pce, p)
    sw_r, inv_r, st_r = ref.drain(list(nw["pore_vol"]), nw["throats"].tolist(), list(pce), list(p))
    print("S_w", np.round(sw, 3), "trapped", (st == network.TRAPPED).sum())
    assert np.array_equal(sw, np.array(sw_r))
    assert np.array_equal(inv, inv_r) and np.array_equal(st, st_r)
    assert sw[0] > sw[-1] and np.all(np.diff(sw) <= 0)
