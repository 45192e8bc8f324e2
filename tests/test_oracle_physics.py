"""Physics pins of the FP64 oracle: closed forms and limits that the paper's
model (Eq. 1-5, velocity-shift forcing of the cited Shan-Chen model) must
reproduce.  Each test pins a different reading:

  flat interface    -> forcing scheme and physical-velocity definition
                       (zero velocity at steady state), Eq. 5 pressure balance,
                       and the coexistence densities of the discrete model
  Laplace law       -> cohesion force + equation of state together, on
                       cylinders (one curvature; gives the interfacial
                       tension used to scale the ramps) and on spherical
                       droplets (two curvatures)
  plane Poiseuille  -> bath boundaries and half-way bounce-back
  wetting           -> sign of the adhesion force (perfect wetting, Sec. 3.1.1)
  drainage ramp     -> monotone saturation, single invasion (Sec. 2.2.2)
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
import synth
from synth import BC_PERIODIC, BC_RESERVOIR, BC_WALLS, Problem

CS2 = 1.0 / 3.0


def coexistence_minor(rho_major, G, tau):
    """Minority density of the symmetric coexisting pair for velocity-shift
    forcing with equal relaxation times: integrating the steady, flux-free
    balance of each component across a flat interface gives
    (tau - 1/2) ln(rho_a/rho_b) = tau G (rho_a - rho_b)."""
    f = lambda b: (tau - 0.5) * math.log(rho_major / b) - tau * G * (rho_major - b)  # noqa
    # b = rho_major is the trivial root; bracket the other one below it
    return brentq(f, 1e-9, 0.9 * rho_major)


def _run_to_rest(o, chunk=2000, max_steps=100000, tol=1e-16):
    prev = o.f()
    n = 0
    d = np.inf
    while n < max_steps:
        o.step(chunk)
        n += chunk
        f = o.f()
        d = np.abs(f - prev).max() / chunk
        prev = f
        if d < tol:
            break
    return n, d


@pytest.mark.parametrize("gads", [(0.0, 0.0), (-0.4, 0.4)])
def test_flat_interface_between_walls_comes_to_rest(gads):
    """A flat w/nw interface between two walls relaxes to exact rest: at the
    steady state the physical velocity (sum_s j_s + sum_s F_s / 2) / rho of the
    velocity-shift forcing vanishes at every node to round-off (the discrete
    face fluxes are zero, so j + j* = 0 per component and sum j = -sum F / 2)."""
    nx = 24
    b = coexistence_minor(2.0, 0.9, 1.0)
    rho0 = synth.flat_interface_density(nx, 4, 4, nx // 2, 2.0, b)
    p = Problem(nx=nx, ny=4, nz=4, bc=(BC_WALLS, BC_PERIODIC, BC_PERIODIC), rho_init=rho0,
                rho_minor=b, G_ads=gads)
    o = oracle.Oracle(p)
    n, d = _run_to_rest(o)
    assert d < 1e-15, (n, d)
    u = o.velocity()
    assert np.abs(u).max() < 1e-12


@pytest.mark.parametrize("tau", [1.0, 1.2])
def test_flat_interface_coexistence_and_pressure(tau):
    """Two flat interfaces on a periodic lattice relax to a symmetric pair of
    bulk phases with equal bulk pressures given by Eq. 5.  At tau = 1 the
    post-collision populations are exact equilibria, and the zero-flux
    balance of each component integrates to the closed form
    (tau - 1/2) ln(rho_a/rho_b) = tau G (rho_a - rho_b), i.e.
    ln(rho_a/rho_b) = 2 G (rho_a - rho_b): twice the G of the continuum free
    energy behind Eq. 5 (velocity-shift forcing); the bulk pair must lie on it
    within the 1 % left by the diffuse interface.  At tau != 1 the
    non-equilibrium part of the post-collision populations adds terms and only
    the symmetry and the pressure balance are pinned."""
    nx = 48
    b = coexistence_minor(2.0, 0.9, tau)
    rho0 = synth.flat_interface_density(nx, 4, 4, nx // 2, 2.0, b)
    rho0 = np.roll(rho0, nx // 4, axis=3)  # w in the middle half, nw around it
    p = Problem(nx=nx, ny=4, nz=4, bc=(BC_PERIODIC,) * 3, rho_init=rho0, tau=(tau, tau),
                rho_minor=b, G_ads=(0.0, 0.0))
    o = oracle.Oracle(p)
    n, d = _run_to_rest(o)
    assert d < 1e-15, (n, d)
    assert np.abs(o.velocity()).max() < 1e-12
    r = o.density()[:, 0, 0, :]
    pr = o.pressure()[0, 0, :]
    iw, inw = nx // 2, 0          # bulk of the w slab, bulk of the nw slab
    wa, wb = r[0, iw], r[1, iw]
    na, nb = r[1, inw], r[0, inw]
    assert abs(wa - na) < 1e-10 and abs(wb - nb) < 1e-10
    lhs = (tau - 0.5) * math.log(wa / wb)
    rhs = tau * 0.9 * (wa - wb)
    print("tau", tau, "bulk pair", wa, wb, "closed-form residual", (lhs - rhs) / rhs)
    if tau == 1.0:
        assert abs(lhs - rhs) < 0.01 * rhs
    assert abs(pr[iw] - pr[inw]) < 1e-12
    assert abs(pr[iw] - (CS2 * (wa + wb) + CS2 * 0.9 * wa * wb)) < 1e-12


def test_laplace_law_cylinders():
    """Static w cylinders in nw (periodic, one-node-thin in z... three nodes):
    the pressure jump (Eq. 5 inside minus outside) is linear in 1/R
    (Laplace-Young for one curvature: dp = gamma / R)."""
    n = 64
    b = coexistence_minor(2.0, 0.9, 1.0)
    res = []
    for R in (10, 13, 16, 20):
        c = (n - 1) / 2.0
        yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        ins = (xx - c) ** 2 + (yy - c) ** 2 <= R * R
        rho0 = np.zeros((2, 3, n, n))
        rho0[0] = np.where(ins, 2.0, b)[None]
        rho0[1] = np.where(ins, b, 2.0)[None]
        p = Problem(nx=n, ny=n, nz=3, bc=(BC_PERIODIC,) * 3, rho_init=rho0, rho_minor=b,
                    G_ads=(0.0, 0.0))
        o = oracle.Oracle(p)
        o.step(6000)
        r = o.density()
        pr = o.pressure()
        phib = (2.0 - b) / (2.0 + b)
        phi = (r[0, 1] - r[1, 1]) / (r[0, 1] + r[1, 1])
        area = ((phi + phib) / (2 * phib)).sum()
        Re = math.sqrt(area / math.pi)
        ic = int(round(c))
        res.append((Re, pr[1, ic, ic] - pr[1, 0, 0]))
    Re = np.array([a for a, _ in res])
    dp = np.array([d for _, d in res])
    A = np.vstack([1 / Re, np.ones_like(Re)]).T
    (gamma, icpt), *_ = np.linalg.lstsq(A, dp, rcond=None)
    pred = A @ np.array([gamma, icpt])
    r2 = 1 - ((dp - pred) ** 2).sum() / ((dp - dp.mean()) ** 2).sum()
    per_r = dp * Re
    print("gamma", gamma, "intercept", icpt, "R2", r2, "gamma per radius", per_r)
    assert r2 >= 0.999
    assert abs(icpt) <= 0.05 * dp.min()
    assert np.all(np.abs(per_r - gamma) <= 0.05 * gamma)
    # the tension the ramps are scaled with
    assert abs(gamma - synth.GAMMA_LAPLACE) < 0.005


def test_laplace_law_droplets():
    """Static w droplets in nw on a periodic lattice at four radii: the Eq. 5
    pressure jump between the droplet's centre and the far field is linear in
    1/R with the coefficient 2 gamma of the Laplace law for a sphere (two
    principal curvatures), where R is the radius of a sphere holding the
    droplet's wetting mass at its bulk density contrast,
    R = (3 V_w / 4 pi)^(1/3), V_w = sum (rho_w - rho_w,out)/(rho_w,in -
    rho_w,out).

    Bars: R^2 >= 0.999 for dp = 2 gamma / R + b; |b| <= 8 % of the smallest
    jump; the per-radius tensions dp R / 2 within 5 % of their mean; gamma
    within 6 % of the tension measured on cylinders (one curvature).  At
    R = 10-16 lu the ~3 lu diffuse interface bends the line by a
    curvature correction of the Tolman kind: the per-radius tension falls
    from 0.193 to 0.189 as R grows, which tilts the straight-line fit to an
    intercept of about -6 % of the smallest jump (it shrinks as 1/R_min;
    radii of 14-26 lu give the same trend and do not reach a steady state in
    3000 steps)."""
    b = coexistence_minor(2.0, 0.9, 1.0)
    res = []
    for R in (10.0, 12.0, 14.0, 16.0):
        n = int(2 * R + 16)
        c = (n - 1) / 2.0
        rho0 = synth.droplet_density(n, n, n, (c, c, c), R, 2.0, b)
        p = Problem(nx=n, ny=n, nz=n, bc=(BC_PERIODIC,) * 3, rho_init=rho0, rho_minor=b,
                    G_ads=(0.0, 0.0))
        o = oracle.Oracle(p)
        o.step(2000)
        r = o.density()
        pr = o.pressure()
        h = n // 2
        core = (slice(h - 1, h + 1),) * 3
        w_in, w_out = r[0][core].mean(), r[0][0, 0, 0]
        Vw = ((r[0] - w_out) / (w_in - w_out)).sum()
        Rw = (3.0 * Vw / (4.0 * math.pi)) ** (1.0 / 3.0)
        dp = pr[core].mean() - pr[0, 0, 0]
        res.append((Rw, dp))
        print("R0", R, "box", n, "R_w", Rw, "dp", dp, "dp R / 2", dp * Rw / 2)
    Rw = np.array([a for a, _ in res])
    dp = np.array([d for _, d in res])
    A = np.vstack([2.0 / Rw, np.ones_like(Rw)]).T
    (gamma, icpt), *_ = np.linalg.lstsq(A, dp, rcond=None)
    pred = A @ np.array([gamma, icpt])
    r2 = 1 - ((dp - pred) ** 2).sum() / ((dp - dp.mean()) ** 2).sum()
    per_r = dp * Rw / 2
    print("gamma", gamma, "intercept / smallest dp", icpt / dp.min(), "R2", r2)
    assert np.all(np.diff(dp) < 0)
    assert r2 >= 0.999
    assert abs(icpt) <= 0.08 * dp.min()
    assert np.all(np.abs(per_r - per_r.mean()) <= 0.05 * per_r.mean())
    assert abs(gamma - synth.GAMMA_LAPLACE) <= 0.06 * synth.GAMMA_LAPLACE


def test_plane_poiseuille_between_baths():
    """With G = 0 and equal relaxation times the mixture is one ideal BGK fluid
    (total density, barycentric velocity).  A small total-density difference
    between the inlet and outlet baths drives it between two walls; the steady
    velocity profile is the plane-Poiseuille parabola with each wall half-way
    between the last fluid node and the solid one."""
    W, L = 16, 40
    m = 0.5
    rho0 = np.full((2, L, 4, W), m)
    p = Problem(nx=W, ny=4, nz=L, bc=(BC_WALLS, BC_PERIODIC, BC_RESERVOIR), rho_init=rho0,
                tau=(1.0, 1.0), G=0.0, G_ads=(0.0, 0.0), rho_major=m, rho_minor=m,
                rho_in_nw=m + 0.01, rho_out_w=m)
    o = oracle.Oracle(p)
    o.step(15000)
    u = o.velocity()
    uz = u[2, L // 2, 0, :]
    x = np.arange(W) + 0.5  # walls at x = 0 and x = W (half-way)
    shape = x * (W - x)
    amp = (uz * shape).sum() / (shape * shape).sum()
    fit = amp * shape
    err = np.abs(uz - fit).max() / np.abs(fit).max()
    print("max |u_z|", np.abs(uz).max(), "relative deviation from parabola", err)
    assert 1e-4 < np.abs(uz).max() < 0.05
    assert np.abs(u[0, L // 2]).max() < 1e-3 * np.abs(uz).max()  # away from the baths
    assert err < 0.02


def test_wetting_droplet_spreads():
    """A w droplet resting on a flat wall with adhesion (-0.4, +0.4) spreads:
    its contact footprint on the wall grows and its height drops (the w phase
    wets the solid, Sec. 3.1.1: perfect wetting of the solid by w)."""
    n = 32
    b = 0.0609883
    z, y, x = np.meshgrid(np.arange(6 + 14), np.arange(n), np.arange(n), indexing="ij")
    rho0 = np.zeros((2, 20, n, n))
    ball = (x - 15.5) ** 2 + (y - 15.5) ** 2 + (z - 0.0) ** 2 <= 8.0 ** 2
    rho0[0] = np.where(ball, 2.0, b)
    rho0[1] = np.where(ball, b, 2.0)
    p = Problem(nx=n, ny=n, nz=20, bc=(BC_PERIODIC, BC_PERIODIC, BC_WALLS), rho_init=rho0,
                rho_minor=b, G_ads=(-0.4, 0.4))
    o = oracle.Oracle(p)

    def footprint_and_height():
        r = o.density()
        w = r[0] > r[1]
        foot = int(w[0].sum())
        col = w[:, 16, 16]
        h = int(np.max(np.nonzero(col)[0])) if col.any() else 0
        return foot, h

    f0, h0 = footprint_and_height()
    o.step(3000)
    f1, h1 = footprint_and_height()
    print("footprint", f0, "->", f1, "height", h0, "->", h1)
    assert f1 > 1.3 * f0
    assert h1 < h0


def test_ramp_saturation_monotone_single_invasion():
    """Along a pressure-controlled drainage ramp the wetting saturation never
    increases and the pore-body probe is invaded once and stays invaded."""
    p = synth.c2_problem(n=32, mean_r=32.0 * 32 / 96)
    r_ins, _ = synth.throat_incircle(p.spheres)
    pcs = synth.pc_ramp(synth.GAMMA_LAPLACE, r_ins, 4, 0.1, 0.9)
    o = oracle.Oracle(p)
    S, inv = [], []
    for pc in pcs:
        o.set_rho_in(o.rho_in_for_pc(pc))
        o.step(2500)
        S.append(o.reduce()[1])
        inv.append(o.probe_invaded())
    print("S", S, "invaded", inv)
    assert np.all(np.diff(S) <= 1e-4)
    assert inv[-1]
    first = inv.index(True)
    assert all(inv[first:])
