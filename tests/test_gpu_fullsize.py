"""GPU against the FP64 oracle at full sizes and in the launch shapes that
the benchmark runs there.

* the 96^3 four-sphere throat, 200 steps, every population: on the node-list
  path (two passes over the non-solid nodes, the shape the autotuner picks on
  this mostly solid box) and on 32 x 4 tiles;
* a throat of the batched workload (packing seed 3, 32 lu per unit radius),
  200 steps, every population;
* the 512^3 packed sample: after 6 steps, the densities of 16^3 windows
  against the oracle run on a crop around each window.  Information moves at
  most two nodes per step (one streaming link plus the one-node density
  stencil of the force), so with a 12-node margin the crop's own walls cannot
  reach the window and the window's values are exact.

Bar: each population's error against its natural scale w_k rho_s within
1e-5 (plain relative error is meaningless where a sharp initial interface
drives single populations through zero); densities within 1e-6 relative."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _scaled_err(fg, fo, types):
    live = types != oracle.SOLID
    a, b = fg[:, :, live], fo[:, :, live]
    rho = b.sum(axis=1, keepdims=True)
    return float(np.max(np.abs(a - b) / (W[None, :, None] * rho)))


def _run_pair(p, sched, steps):
    from paper_1906_04722_amd import lbm
    g = lbm.Throat(p)
    g.set_schedule(*sched)
    o = oracle.Oracle(p)
    g.step(steps)
    o.step(steps)
    err = _scaled_err(g.f(), o.f(), o.types())
    g.close()
    return err


@pytest.mark.parametrize("sched", [(-1, 0, 0), (32, 4, 1)])
def test_c2_full_size(sched):
    err = _run_pair(synth.c2_problem(), sched, 200)
    print("96^3 throat, schedule", sched, "200 steps, max scaled error", err)
    assert err <= 1e-5


def test_batch_throat_full_resolution():
    probs, _, _ = synth.packing_throats(n_throats=1, seed=3)
    p = probs[0]
    print("throat box", p.nx, p.ny, p.nz)
    err = _run_pair(p, (64, 4, 8), 200)
    print("packing throat, 200 steps, max scaled error", err)
    assert err <= 1e-5


@pytest.mark.parametrize("sched", [(32, 8, 16), (64, 4, 32)])
def test_sample_512_windows(sched):
    from paper_1906_04722_amd import lbm
    p, _ = synth.packed_sample(512, 1000, seed=4)
    steps, margin, w = 6, 12, 16
    g = lbm.Throat(p)
    g.set_schedule(*sched)
    g.step(steps)
    rho = g.density()
    T = g.types()
    g.close()
    S = np.asarray(p.spheres, dtype=np.float64)
    rng = np.random.default_rng(1)
    n = w + 2 * margin
    origins = []
    while len(origins) < 3:
        # windows that hold a fair share of fluid (a sphere can fill 16^3)
        o = rng.integers(40, 512 - 40 - n, size=3)
        win = T[o[2] + margin:o[2] + margin + w, o[1] + margin:o[1] + margin + w,
                o[0] + margin:o[0] + margin + w]
        if (win == lbm.LBM_NODE_FLUID).mean() > 0.25:
            origins.append(o)
    for o in origins:
        Sc = S.copy()
        Sc[:, :3] -= o
        keep = np.all((Sc[:, :3] + Sc[:, 3:4] > -2) & (Sc[:, :3] - Sc[:, 3:4] < n + 1), axis=1)
        # the window lies far above the inlet layer: wetting fluid everywhere
        rho0 = synth.layered_density(n, n, n, -1, p.rho_major, p.rho_minor)
        c = synth.Problem(nx=n, ny=n, nz=n, bc=(synth.BC_WALLS,) * 3, spheres=Sc[keep],
                          rho_init=rho0, probe=None)
        oc = oracle.Oracle(c)
        oc.step(steps)
        ro = oc.density()[:, margin:margin + w, margin:margin + w, margin:margin + w]
        t = oc.types()[margin:margin + w, margin:margin + w, margin:margin + w]
        rg = rho[:, o[2] + margin:o[2] + margin + w, o[1] + margin:o[1] + margin + w,
                 o[0] + margin:o[0] + margin + w]
        fl = t == oracle.FLUID
        assert fl.any()
        err = float(np.max(np.abs(rg[:, fl] - ro[:, fl]) / ro[:, fl]))
        moved = float(np.max(np.abs(ro[:, fl] - rho0[:, :w, :w, :w][:, fl])))
        print("window at", o + margin, "max density error", err, "largest change", moved)
        assert moved > 1e-4   # the adhesion at the sphere surfaces has moved the fluid
        assert err <= 1e-6
