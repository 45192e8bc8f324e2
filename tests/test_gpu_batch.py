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


def test_batch_with_z_periodic_subdomains_equals_single_drains():
    """z-periodic subdomains carry ghost planes that a kernel after each step
    refreshes, inside the batch's graph and outside it for a single drain:
    two periodic droplet boxes batched with a prism throat give the single
    drains' results bit for bit."""
    from paper_1906_04722_amd import lbm
    from synth import BC_PERIODIC, Problem
    probs, pcs = _throats()
    boxes = []
    # wetting droplets in the non-wetting bulk, away from the sphere; the
    # probe at a droplet's centre stays wetting, so every ramp point runs to
    # its cap and no bisection starts
    for seed, c in ((5, (16.0, 9.0, 10.0)), (6, (20.0, 10.0, 12.0))):
        rho0 = synth.droplet_density(33, 18, 20, c, 5.0, 2.0, 0.0609883, seed=seed, amp=1e-3)
        boxes.append(Problem(nx=33, ny=18, nz=20, bc=(BC_PERIODIC,) * 3, tau=(0.9, 1.1),
                             spheres=np.array([[3.0, 3.0, 3.0, 2.5]]), rho_init=rho0,
                             probe=tuple(int(v) for v in c)))
    mix = [boxes[0], probs[0], boxes[1]]
    n_pc = pcs.shape[1]
    ramp = np.vstack([np.linspace(0.002, 0.01, n_pc), pcs[0], np.linspace(0.002, 0.01, n_pc)])
    conv = dict(tol=1e-7, check_every=100, max_steps=600, bisect_rel=0.02)
    outs, _ = lbm.drain_batch(mix, ramp, **conv)
    for p, pc, b in zip(mix, ramp, outs):
        s = lbm.Throat(p).drain(pc, **conv)
        assert np.array_equal(s["S"], b["S"])
        assert np.array_equal(s["steps"], b["steps"])
        assert s["total_steps"] == b["total_steps"]


def test_invaded_at_the_first_point_ends_with_a_bracket():
    """A throat whose probe holds the non-wetting phase from the start is
    invaded at every pressure: the bracket starts at 0 and halving never
    reaches the relative width, so bisection stops at its run limit (40) with
    a warning, the same in the single drain and in a batch."""
    from paper_1906_04722_amd import lbm
    p = synth.small_throat_problem(n=24)
    p.rho_init = synth.layered_density(24, 24, 24, 20, p.rho_major, p.rho_minor, 3, 1e-3)
    r_ins, _ = synth.throat_incircle(p.spheres)
    pc = synth.pc_ramp(synth.GAMMA_LAPLACE, r_ins, 4, 0.2, 0.8)
    conv = dict(tol=1e-5, check_every=50, max_steps=100, bisect_rel=0.02)
    s = lbm.Throat(p).drain(pc, **conv)
    assert s["invaded_at"] == 0 and s["n_bisect"] == 40
    assert s["pce_lo"] == 0.0 and 0.0 < s["pce_hi"] <= pc[0] * 2.0 ** -40
    assert s["warning"] == lbm.LBM_WNOTCONV
    (b,), _ = lbm.drain_batch([p], pc[None, :], **conv)
    assert b["n_bisect"] == 40 and b["pce_hi"] == s["pce_hi"]
    assert np.array_equal(b["S"], s["S"]) and b["total_steps"] == s["total_steps"]


def test_batch_without_graph_equals_graph_replay(monkeypatch):
    """LBM_BATCH_NO_GRAPH=1 launches each chunk's kernels one by one instead
    of replaying the captured graph: the same kernels in the same order, so
    the results are bit-identical."""
    from paper_1906_04722_amd import lbm
    probs, pcs = _throats()
    probs, pcs = probs[:2], pcs[:2]
    a, ia = lbm.drain_batch(probs, pcs, **CONV)
    monkeypatch.setenv("LBM_BATCH_NO_GRAPH", "1")
    b, ib = lbm.drain_batch(probs, pcs, **CONV)
    assert ia["replays"] == ib["replays"]
    for x, y in zip(a, b):
        for k in ("S", "steps", "status"):
            assert np.array_equal(x[k], y[k])
        assert np.array_equal([x["pce"], x["pce_lo"], x["pce_hi"]],
                              [y["pce"], y["pce_lo"], y["pce_hi"]], equal_nan=True)
