"""Host inputs of the batched workload: the seeded dense packing, its regular
(weighted Delaunay) triangulation (Sec. 2.2.1) and the throat subdomains cut
from its interior facets (Sec. 2.2.2).

The triangulation is pinned by properties it must have, each checked by brute
force rather than by the lifting construction it is built with: with equal
radii it is the Delaunay triangulation; every tetrahedron's orthosphere is
empty in the power distance; the tetrahedra tile the periodic cell."""
import itertools

import numpy as np
import pytest

import oracle
import synth
from synth import packing


@pytest.fixture(scope="module")
def pack():
    x, r, L, phi, worst = packing.dense_packing(200, seed=11)
    return x, r, L, phi, worst


def test_packing_density_and_overlap(pack):
    x, r, L, phi, worst = pack
    assert abs(phi - 0.62) < 1e-9
    # brute-force periodic overlap over every pair, normalised by the mean radius
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.round(d / L)
    dist = np.sqrt((d * d).sum(-1))
    ov = (r[:, None] + r[None, :] - dist)[np.triu_indices(len(x), 1)]
    assert ov.max() < 1e-4  # in units of the mean radius parameter (1.0)
    # lognormal radii: log-sd close to 0.2, arithmetic mean close to 1
    assert abs(np.log(r).std() - 0.2) < 0.03
    assert abs(r.mean() - 1.0) < 0.05


def test_equal_radii_reduce_to_delaunay():
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 6, size=(40, 3))
    r = np.full(40, 0.5)
    P, R, I, tets = packing.regular_triangulation(x, r, 6.0, margin=1.5)
    mine = {tuple(sorted(t)) for t in tets}
    ref = {tuple(sorted(t)) for t in Delaunay(P).simplices}
    assert mine == ref


def _orthocentre(V, w):
    # |c - v_i|^2 - w_i equal for all four vertices: linear in c
    A = 2.0 * (V[1:] - V[0])
    b = (V[1:] ** 2).sum(1) - (V[0] ** 2).sum() - (w[1:] - w[0])
    c = np.linalg.solve(A, b)
    return c, ((c - V[0]) ** 2).sum() - w[0]


def test_power_empty_orthospheres(pack):
    x, r, L, _, _ = pack
    P, R, I, tets = packing.regular_triangulation(x, r, L)
    w = R * R
    cen = P[tets].mean(1)
    inner = np.nonzero(np.all((cen >= 0) & (cen < L), axis=1))[0]
    rng = np.random.default_rng(0)
    for t in rng.choice(inner, 60, replace=False):
        c, pw = _orthocentre(P[tets[t]], w[tets[t]])
        others = np.setdiff1d(np.arange(len(P)), tets[t])
        pow_o = ((P[others] - c) ** 2).sum(1) - w[others]
        assert pow_o.min() >= pw - 1e-9 * (1 + abs(pw))


def test_tetrahedra_tile_the_cell(pack):
    x, r, L, _, _ = pack
    P, R, I, tets = packing.regular_triangulation(x, r, L)
    V = P[tets]
    vol = np.abs(np.einsum("ij,ij->i", V[:, 1] - V[:, 0],
                           np.cross(V[:, 2] - V[:, 0], V[:, 3] - V[:, 0]))) / 6.0
    cen = V.mean(1)
    inner = np.all((cen >= 0) & (cen < L), axis=1)
    assert abs(vol[inner].sum() / L ** 3 - 1.0) < 1e-9
    facets = packing.interior_facets(P, tets, L)
    assert len(facets) > 0
    for f, a, b in facets[:200]:
        assert a != b and a not in f and b not in f


def test_throat_boxes():
    probs, rins, summ = packing.packing_throats(n_throats=6, n_spheres=200, seed=11)
    assert len(probs) == 6 and abs(summ["porosity"] - 0.38) < 1e-9
    x, r, L, _, _ = packing.dense_packing(200, seed=11)
    for p, ri in zip(probs, rins):
        assert all(48 <= s <= 128 for s in (p.nx, p.ny, p.nz))
        assert ri > 0
        # the mapping is a rigid motion plus one scale: the ratio of every
        # centre distance to the sum of the two radii is preserved, and the
        # scaled radii are radii of the packing
        S = p.spheres
        for i, j in itertools.combinations(range(4), 2):
            q = np.linalg.norm(S[i, :3] - S[j, :3]) / (S[i, 3] + S[j, 3])
            assert q > 1.0 - 1e-4  # no overlap beyond the packing tolerance
        fits = [s for s in S[0, 3] / r
                if all(np.abs(S[k, 3] / s - r).min() < 1e-9 for k in range(4))]
        assert fits
        # the facet plane is z = const, the apex above it, inside the box
        assert np.ptp(S[:3, 2]) < 1e-9 and S[3, 2] > S[0, 2]
        assert np.all(S[:, :3] > -S[:, 3:4]) and S[:, 2].max() < p.nz
        # the pore-body probe is a fluid node of the oracle's voxelization
        t = oracle.Oracle(p).types().reshape(p.nz, p.ny, p.nx)
        px, py, pz = p.probe
        assert t[pz, py, px] == 0
        assert (t == 0).mean() > 0.05


def test_packing_of_a_given_cell_side():
    # the paper's sample sizes: 40 spheres of mean radius 1.26 in a 10-unit
    # cell; the solid fraction then follows from the drawn radii
    x, r, L, phi, worst = packing.dense_packing(40, mean_r=1.26, seed=7, side=10.0)
    assert L == 10.0
    assert abs(phi - (4.0 / 3.0) * np.pi * (r ** 3).sum() / 1000.0) < 1e-12
    assert worst < 1e-4
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.round(d / L)
    dist = np.sqrt((d ** 2).sum(-1)) + np.eye(len(r)) * 1e9
    assert ((r[:, None] + r[None, :] - dist) / r.mean()).max() < 1e-4
