"""Exact pins of the FP64 oracle: lattice identities, equilibrium moments,
conservation laws, symmetry and brute-force agreement with a hand-unrolled
4^3 step.  None of these recomputes the oracle's own formula: each checks a
property that the paper's equations (Eq. 1-5) or the lattice fix."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth import BC_PERIODIC, BC_RESERVOIR, BC_WALLS, Problem
from tests import unrolled4

CS2 = Fraction(1, 3)


def test_d3q19_identities_exact():
    """P1: the tabulated D3Q19 set has the moments that make Eq. 1 recover
    Navier-Stokes and Eq. 5's pressure: sum w = 1, sum w e = 0,
    sum w e_a e_b = c_s^2 delta_ab, fourth-order isotropy; opposite table."""
    e, w, opp = oracle.lattice()
    wf = [Fraction(x).limit_denominator(1000) for x in w]
    assert all(abs(float(a) - b) == 0 for a, b in zip(wf, w))
    assert len({tuple(v) for v in e}) == 19
    assert sum(wf) == 1
    for a in range(3):
        assert sum(wk * int(ek[a]) for wk, ek in zip(wf, e)) == 0
        for b in range(3):
            m2 = sum(wk * int(ek[a]) * int(ek[b]) for wk, ek in zip(wf, e))
            assert m2 == (CS2 if a == b else 0)
            for c in range(3):
                m3 = sum(wk * int(ek[a]) * int(ek[b]) * int(ek[c]) for wk, ek in zip(wf, e))
                assert m3 == 0
                for d in range(3):
                    m4 = sum(wk * int(ek[a]) * int(ek[b]) * int(ek[c]) * int(ek[d])
                             for wk, ek in zip(wf, e))
                    want = CS2 * CS2 * ((a == b) * (c == d) + (a == c) * (b == d)
                                        + (a == d) * (b == c))
                    assert m4 == want
    for k in range(19):
        assert (e[opp[k]] == -e[k]).all()
        assert opp[opp[k]] == k
    # D3Q19: the rest vector, 6 face and 12 edge vectors, no corners
    norms = sorted(int((v * v).sum()) for v in e)
    assert norms == [0] + [1] * 6 + [2] * 12


def test_equilibrium_moments():
    """P2: the equilibrium carries the density and momentum it was built from
    (Eq. 2-3 applied to f_eq), and its second moment is
    rho (c_s^2 I + u u)."""
    e, _, _ = oracle.lattice()
    rng = np.random.default_rng(0)
    for _ in range(20):
        rho = rng.uniform(0.3, 3.0)
        u = rng.uniform(-0.1, 0.1, 3)
        fe = oracle.feq(rho, u)
        assert abs(fe.sum() - rho) <= 1e-15 * rho * 4
        np.testing.assert_allclose(fe @ e, rho * u, rtol=0, atol=1e-15 * 8)
        Pi = np.einsum("k,ka,kb->ab", fe, e.astype(float), e.astype(float))
        np.testing.assert_allclose(Pi, rho * (np.eye(3) / 3.0 + np.outer(u, u)), atol=1e-14)


def _rand_f(prob, seed, amp=0.05):
    """Random near-equilibrium populations with random velocities."""
    rng = np.random.default_rng(seed)
    e, w, _ = oracle.lattice()
    shape = (prob.nz, prob.ny, prob.nx)
    f = np.zeros((2, 19) + shape)
    for c in range(2):
        rho = rng.uniform(0.6, 2.0, shape)
        u = rng.uniform(-0.05, 0.05, (3,) + shape)
        eu = np.einsum("ka,a...->k...", e.astype(float), u)
        uu = (u * u).sum(0)
        f[c] = w[:, None, None, None] * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu)
        f[c] *= 1 + amp * rng.uniform(-1, 1, f[c].shape)
    return f


def test_closed_box_mass_conservation():
    """P3: with walls on every face and no baths, Eq. 1 with bounce-back only
    moves populations around: each component's mass is conserved."""
    n = 20
    sph = np.array([[6.0, 7.0, 9.0, 4.5], [14.0, 12.0, 10.0, 3.7]])
    rho0 = synth.droplet_density(n, n, n, (10, 10, 10), 5.0, 2.0, 0.0609883, seed=3, amp=1e-3)
    p = Problem(nx=n, ny=n, nz=n, bc=(BC_WALLS, BC_WALLS, BC_WALLS), spheres=sph,
                tau=(1.0, 0.8), rho_init=rho0)
    o = oracle.Oracle(p)
    m0, _, _ = o.reduce()
    o.step(200)
    m1, _, _ = o.reduce()
    np.testing.assert_allclose(m1, m0, rtol=1e-12, atol=0)
    assert np.abs(m1 - m0).max() / m0.max() < 1e-12


def test_periodic_momentum_conservation_and_force_balance():
    """P4: with symmetric cross-component coupling (Eq. 4) on a periodic,
    solid-free lattice the cohesion forces cancel pairwise, so total force is
    zero and total momentum is constant."""
    n = 8
    p = Problem(nx=n, ny=n, nz=n, bc=(BC_PERIODIC,) * 3, tau=(1.0, 0.7))
    o = oracle.Oracle(p)
    o.set_f(_rand_f(p, 11))
    F = o.force()
    Ftot = F.sum(axis=(0, 2, 3, 4))
    scale = np.abs(F).sum()
    assert np.abs(Ftot).max() <= 1e-13 * scale
    _, _, P0 = o.reduce()
    o.step(50)
    _, _, P1 = o.reduce()
    m, _, _ = o.reduce()
    assert np.abs(P1 - P0).max() <= 1e-13 * m.sum()
    assert np.abs(P0).max() > 1e-3  # the test has momentum to conserve


def test_translation_invariance_bitwise():
    """P11: on a periodic lattice, shifting the initial state by one node in x
    shifts the result by one node, bit for bit."""
    n = 6
    p = Problem(nx=n, ny=n, nz=n, bc=(BC_PERIODIC,) * 3, G_ads=(0.0, 0.0))
    f = _rand_f(p, 5)
    a = oracle.Oracle(p)
    a.set_f(f)
    a.step(7)
    b = oracle.Oracle(p)
    b.set_f(np.roll(f, 1, axis=-1))
    b.step(7)
    assert np.array_equal(np.roll(a.f(), 1, axis=-1), b.f())


def test_mirror_invariance():
    """P11: mirroring x -> -x (with the matching relabel of directions) maps
    the evolution onto itself."""
    n = 6
    p = Problem(nx=n, ny=n, nz=n, bc=(BC_PERIODIC,) * 3)
    e, _, _ = oracle.lattice()
    mirror = [int(np.flatnonzero((e == e[k] * np.array([-1, 1, 1])).all(1))[0]) for k in range(19)]
    f = _rand_f(p, 6)

    def flip(g):
        return g[:, mirror][..., ::-1]

    a = oracle.Oracle(p)
    a.set_f(f)
    a.step(5)
    b = oracle.Oracle(p)
    b.set_f(np.ascontiguousarray(flip(f)))
    b.step(5)
    np.testing.assert_allclose(flip(a.f()), b.f(), rtol=1e-13, atol=1e-15)


def _unrolled_params(p):
    return dict(tau=p.tau, G=p.G, G_ads=p.G_ads, rho_major=p.rho_major, rho_minor=p.rho_minor,
                rho_in_nw=p.rho_in_nw, rho_out_w=p.rho_out_w)


@pytest.mark.parametrize("case", ["periodic", "one_solid", "walls_and_baths"])
def test_bruteforce_unrolled_4cube(case):
    """P8: ten steps of the oracle agree with the hand-unrolled 4^3 step."""
    n = 4
    if case == "periodic":
        p = Problem(nx=n, ny=n, nz=n, bc=(BC_PERIODIC,) * 3, tau=(1.0, 0.75))
        types = np.zeros((n, n, n), dtype=np.uint8)
    elif case == "one_solid":
        p = Problem(nx=n, ny=n, nz=n, bc=(BC_PERIODIC,) * 3, tau=(0.9, 1.3),
                    spheres=np.array([[1.0, 2.0, 1.0, 0.25]]))
        types = np.zeros((n, n, n), dtype=np.uint8)
        types[1, 2, 1] = 1
    else:
        p = Problem(nx=n, ny=n, nz=n, bc=(BC_WALLS, BC_PERIODIC, BC_RESERVOIR), tau=(1.0, 1.2),
                    spheres=np.array([[2.0, 1.0, 2.0, 0.25]]), rho_in_nw=2.07, rho_out_w=1.97)
        types = np.zeros((n, n, n), dtype=np.uint8)
        types[0] = 2
        types[n - 1] = 3
        types[2, 1, 2] = 1
    o = oracle.Oracle(p)
    assert np.array_equal(o.types(), types)
    f = _rand_f(p, 21)
    o.set_f(f)
    g = o.f()  # the oracle's state after imposing node classes
    periodic = tuple(b == BC_PERIODIC for b in p.bc)
    P = _unrolled_params(p)
    for _ in range(10):
        g = unrolled4.step(g, types, P, periodic)
    o.step(10)
    h = o.f()
    scale = np.abs(g).max()
    assert np.abs(h - g).max() <= 1e-14 * scale * 10


def _single_component_bgk(f, tau, nsteps, periodic_shape):
    """Textbook single-component D3Q19 BGK on a periodic lattice (no forces):
    the limit the two-component model must reduce to when G = 0."""
    e = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
                  [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    for _ in range(nsteps):
        rho = f.sum(0)
        u = np.einsum("ka,k...->a...", e.astype(float), f) / rho
        eu = np.einsum("ka,a...->k...", e.astype(float), u)
        uu = (u * u).sum(0)
        feq = w[:, None, None, None] * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu)
        post = f - (f - feq) / tau
        f = np.stack([np.roll(post[k], shift=(e[k][2], e[k][1], e[k][0]), axis=(0, 1, 2))
                      for k in range(19)])
    return f


def test_g0_reduces_to_single_component_bgk():
    """P9: with G = 0, no adhesion and equal tau, f_w + f_nw obeys the
    single-component BGK equation exactly (f_eq is linear in rho at fixed u and
    the common velocity is the barycentric one)."""
    n = 6
    p = Problem(nx=n, ny=n, nz=n, bc=(BC_PERIODIC,) * 3, tau=(0.8, 0.8), G=0.0,
                G_ads=(0.0, 0.0))
    o = oracle.Oracle(p)
    f = _rand_f(p, 9)
    o.set_f(f)
    o.step(12)
    got = o.f().sum(0)
    want = _single_component_bgk(f.sum(0), 0.8, 12, None)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-15)
