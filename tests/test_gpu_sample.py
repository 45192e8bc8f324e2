"""The fully resolved packed sample: many spheres binned by the voxelizer,
walls and baths, at small sizes against the oracle and at 512^3 through
sampled windows and properties that hold at any size."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _lbm():
    from paper_1906_04722_amd import lbm
    return lbm


@pytest.mark.parametrize("n,ns,nz", [(96, 60, None), (80, 40, 56), (33, 9, 47)])
def test_node_classes_many_spheres_bitwise(n, ns, nz):
    lbm = _lbm()
    p, _ = synth.packed_sample(n, ns, seed=4, nz=nz)
    assert len(p.spheres) > ns
    assert np.array_equal(oracle.Oracle(p).types(), lbm.Throat(p).types())


W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def test_small_sample_populations_match_oracle():
    """60 steps on a 40 x 40 x 44 packed sample; each population's error is
    measured against its natural scale w_k rho_s (1e-5)."""
    lbm = _lbm()
    p, _ = synth.packed_sample(40, 10, seed=7, nz=44)
    p.rho_init = synth.layered_density(40, 40, 44, 2, p.rho_major, p.rho_minor, 3, 1e-3)
    o, g = oracle.Oracle(p), lbm.Throat(p)
    o.step(60)
    g.step(60)
    live = o.types() != oracle.SOLID
    a, b = g.f()[:, :, live], o.f()[:, :, live]
    rho = b.sum(axis=1, keepdims=True)
    err = float(np.max(np.abs(a - b) / (W[None, :, None] * rho)))
    print("max scaled err", err)
    assert err <= 1e-5


@pytest.fixture(scope="module")
def sample512():
    p, summ = synth.packed_sample(512, 1000, seed=4)
    return p, summ


def test_512_node_classes_in_windows(sample512):
    """Windows of the 512^3 sample: the oracle classifies the same nodes from
    the shifted sphere list (walled window, no baths)."""
    lbm = _lbm()
    p, _ = sample512
    g = lbm.Throat(p)
    T = g.types()
    g.close()
    rng = np.random.default_rng(0)
    for _ in range(3):
        o = rng.integers(1, 512 - 48, size=3)
        S = np.asarray(p.spheres, dtype=np.float64).copy()
        S[:, :3] -= o
        keep = np.all((S[:, :3] + S[:, 3:4] > -1) & (S[:, :3] - S[:, 3:4] < 49), axis=1)
        w = synth.Problem(nx=48, ny=48, nz=48, bc=(synth.BC_WALLS,) * 3, spheres=S[keep],
                          probe=None)
        ref = oracle.Oracle(w).types() == oracle.SOLID
        got = T[o[2]:o[2] + 48, o[1]:o[1] + 48, o[0]:o[0] + 48] == lbm.LBM_NODE_SOLID
        assert np.array_equal(ref, got), o


def test_512_closed_sample_conserves_mass(sample512):
    """The same 512^3 geometry closed on all sides: each component's mass is
    conserved (FP32 storage with FP64 sums: drift well below 1e-6)."""
    lbm = _lbm()
    p, _ = sample512
    q = synth.Problem(nx=512, ny=512, nz=512, bc=(synth.BC_WALLS,) * 3, spheres=p.spheres,
                      z_front=256, probe=None)
    g = lbm.Throat(q)
    m0 = g.reduce()[0]
    g.step(20)
    m1 = g.reduce()[0]
    g.close()
    print("mass", m0, m1)
    assert np.all(np.isfinite(m1))
    assert np.all(np.abs(np.asarray(m1) - np.asarray(m0)) <= 1e-6 * np.asarray(m0))
