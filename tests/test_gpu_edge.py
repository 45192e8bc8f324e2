"""Degenerate and smallest inputs on the GPU: a box with no fluid node (no
tile and no list entry to launch), the smallest box the library accepts
(3 x 3 x 3, every tile ragged) against the oracle, and a probe placed on a
solid node."""
import numpy as np
import pytest

import oracle
import synth
from synth import BC_PERIODIC, BC_WALLS, Problem

pytestmark = pytest.mark.gpu

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def test_box_without_fluid_nodes():
    from paper_1906_04722_amd import lbm
    p = Problem(nx=8, ny=9, nz=10, bc=(BC_WALLS,) * 3, spheres=np.array([[4.0, 4.0, 5.0, 20.0]]))
    g = lbm.Throat(p)
    assert (g.types() == lbm.LBM_NODE_SOLID).all()
    for sched in ((32, 4, 1), (8, 8, 4), (lbm.LBM_SCHED_NODE_LIST, 0, 0)):
        g.set_schedule(*sched)
        g.step(5)
    g.sync()
    m, S = g.reduce()
    assert np.array_equal(m, [0.0, 0.0]) and S == 0.0
    assert not g.f().any() and not g.density().any()
    g.close()


def test_probe_on_a_solid_node_is_refused():
    from paper_1906_04722_amd import lbm
    p = synth.c1_problem()
    S = np.asarray(p.spheres)
    p.probe = tuple(int(round(v)) for v in S[0, :3])   # a sphere centre
    with pytest.raises(lbm.LBMError):
        lbm.Throat(p)


@pytest.mark.parametrize("sched", [(32, 4, 1), (8, 8, 2), (-1, 0, 0)])
def test_smallest_box_against_the_oracle(sched):
    """3 x 3 x 3 periodic nodes, one sphere node solid: 30 steps from a
    perturbed two-phase state, every population within 1e-5 of its scale."""
    from paper_1906_04722_amd import lbm
    rho0 = synth.layered_density(3, 3, 3, 0, 2.0, 0.0609883, 4, 1e-3)
    p = Problem(nx=3, ny=3, nz=3, bc=(BC_PERIODIC,) * 3, spheres=np.array([[0.0, 0.0, 0.0, 0.4]]),
                rho_init=rho0)
    o, g = oracle.Oracle(p), lbm.Throat(p)
    g.set_schedule(*sched)
    assert np.array_equal(g.types() == lbm.LBM_NODE_SOLID, o.types() == oracle.SOLID)
    o.step(30)
    g.step(30)
    live = o.types() != oracle.SOLID
    a, b = g.f()[:, :, live], o.f()[:, :, live]
    g.close()
    rho = b.sum(axis=1, keepdims=True)
    err = float(np.max(np.abs(a - b) / (W[None, :, None] * rho)))
    print("max scaled err", err)
    assert err <= 1e-5
