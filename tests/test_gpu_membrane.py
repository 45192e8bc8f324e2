"""The fully resolved drainage sample with its porous membrane on the GPU:
populations against the oracle on a small sample of the same construction,
and what the quasi-static ramp must show (the membrane holds the non-wetting
phase, the slab drains)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _small(res):
    x, r, L, _, _ = synth.dense_packing(10, seed=7)
    return synth.membrane_sample(x, r, L, res=res)


def test_membrane_sample_populations_match_oracle():
    """60 steps from a perturbed layered state (nw up to the slab's middle);
    each population's error against its natural scale w_k rho (1e-5)."""
    from paper_1906_04722_amd import lbm
    p, info = _small(6.0)
    zf = (info["slab"][0] + info["slab"][1]) // 2
    p.rho_init = synth.layered_density(p.nx, p.ny, p.nz, zf, p.rho_major, p.rho_minor, 5, 1e-3)
    o, g = oracle.Oracle(p), lbm.Throat(p)
    assert np.array_equal(g.types() == lbm.LBM_NODE_SOLID, o.types() == oracle.SOLID)
    o.step(60)
    g.step(60)
    live = o.types() != oracle.SOLID
    a, b = g.f()[:, :, live], o.f()[:, :, live]
    g.close()
    rho = b.sum(axis=1, keepdims=True)
    err = float(np.max(np.abs(a - b) / (W[None, :, None] * rho)))
    print("max scaled err", err)
    assert err <= 1e-5


def test_membrane_holds_and_slab_drains():
    from paper_1906_04722_amd import sample_drain
    from synth import membrane
    p, info = _small(8.0)
    P = np.array([1.0, 6.0, 12.0])               # capillary pressure x packing length / gamma
    pcs = P * synth.GAMMA_LAPLACE / info["scale"]
    x, r, L, _, _ = synth.dense_packing(10, seed=7)
    nw = synth.pore_network(x, r, L)
    pts = membrane.lattice_points(nw["pore_xyz"], info)
    out = sample_drain.drain_sample(p, pcs, info["slab"], info["membrane_z"], tol=1e-5,
                                    check_every=200, max_steps=8000, points=pts)
    S = np.array(out["S_slab"])
    print("S_slab", S, "sharp", out["S_slab_sharp"], "outlet",
          out["S_outlet"], "steps", out["steps"])
    # below the throats' entry pressures the slab stays saturated
    assert S[0] > 0.95
    # the membrane keeps the wetting layer behind it at every pressure
    assert min(out["S_outlet"]) > 0.97
    # the slab drains as the pressure rises
    assert S[-1] < S[0] - 0.25
    Sp = np.array(out["S_points"])
    assert Sp.shape == (3, len(nw["pore_vol"]))
    fin = np.isfinite(Sp)
    assert fin[0].mean() > 0.8
    # pores drain with the slab: more pore centroids are non-wetting at the top
    assert (Sp[-1][fin[-1]] < 0.5).mean() > (Sp[0][fin[0]] < 0.5).mean()
