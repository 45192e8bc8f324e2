"""Pins of the oracle's reductions, imposed pressure and drainage ramp, each
against something other than the oracle's own formula:

  saturation      -> fields whose wetting saturation is known exactly
                     (pure phases, a layered field, an equal mixture), with
                     bath and solid nodes left out of the mean
  imposed p_c     -> the Eq. 5 pressures of the two baths differ by the
                     requested capillary pressure; at a static meniscus the
                     bulk pressure of each phase equals its bath's
  drainage ramp   -> a brute-force quasi-static scan at fine pressure steps
                     locates the same invasion threshold as the ramp's
                     bisection (Sec. 2.2.2: the entry pressure is the largest
                     capillary pressure held before the non-wetting phase
                     passes the throat)
"""
import numpy as np
import pytest

import oracle
import synth
from synth import BC_PERIODIC, BC_RESERVOIR, BC_WALLS, Problem

CS2 = 1.0 / 3.0
RHO_M = 0.0609883


def _box_with_baths_and_sphere(rho_init):
    nz, ny, nx = rho_init.shape[1:]
    return Problem(nx=nx, ny=ny, nz=nz, bc=(BC_WALLS, BC_WALLS, BC_RESERVOIR),
                   spheres=np.array([[5.0, 4.0, 6.0, 2.6]]), rho_init=rho_init,
                   rho_minor=RHO_M, rho_in_nw=2.0, rho_out_w=2.0)


def _field(nx, ny, nz, w_mask, rho_w_in=2.0, rho_w_out=RHO_M):
    """rho_w = rho_w_in where w_mask, else rho_w_out; rho_nw the other way."""
    rho = np.empty((2, nz, ny, nx))
    rho[0] = np.where(w_mask, rho_w_in, rho_w_out)
    rho[1] = np.where(w_mask, rho_w_out, rho_w_in)
    return rho


def test_saturation_of_known_fields():
    """S_w is the mean over fluid nodes (bath and solid nodes excluded) of the
    linear map of phi = (rho_w - rho_nw)/(rho_w + rho_nw) that sends the
    wetting bulk (rho_major, rho_minor) to 1 and the non-wetting bulk to 0:
    a pure wetting field gives exactly 1, a pure non-wetting one 0, a field
    whose fluid nodes are wetting above a plane gives the fluid fraction
    above it, and an equal mixture (phi = 0) gives 1/2.  The masses are the
    plain sums of the densities over the fluid nodes."""
    nx, ny, nz = 11, 9, 14
    z = np.arange(nz)[:, None, None] * np.ones((nz, ny, nx))
    cases = []
    cases.append((_field(nx, ny, nz, np.ones((nz, ny, nx), bool)), lambda fl: 1.0))
    cases.append((_field(nx, ny, nz, np.zeros((nz, ny, nx), bool)), lambda fl: 0.0))
    above = z > 5
    cases.append((_field(nx, ny, nz, above), lambda fl: above[fl].mean()))
    cases.append((np.ones((2, nz, ny, nx)), lambda fl: 0.5))
    for rho0, expect in cases:
        o = oracle.Oracle(_box_with_baths_and_sphere(rho0))
        T = o.types()
        fl = T == oracle.FLUID
        assert (T == oracle.SOLID).any() and (T == oracle.RES_IN).any()
        m, S, _ = o.reduce()
        want = float(expect(fl))
        print("expected S", want, "oracle", S)
        assert abs(S - want) <= 1e-13
        for c in range(2):
            assert abs(m[c] - rho0[c][fl].sum()) <= 1e-13 * rho0[c][fl].sum()


@pytest.mark.parametrize("pc", [0.0, 0.004, 0.0123, 0.05])
def test_imposed_pc_is_the_eq5_bath_pressure_difference(pc):
    """Setting the inlet density for a capillary pressure p_c makes the Eq. 5
    pressure of the inlet bath exceed that of the outlet bath by p_c (the
    minority densities of both baths stay fixed)."""
    p = synth.small_throat_problem(n=16, seed=3)
    o = oracle.Oracle(p)
    o.set_rho_in(o.rho_in_for_pc(pc))
    T = o.types()
    P = o.pressure()
    pin, pout = P[T == oracle.RES_IN], P[T == oracle.RES_OUT]
    assert np.ptp(pin) == 0.0 and np.ptp(pout) == 0.0
    r = o.density()
    ri, ro = r[:, T == oracle.RES_IN][:, 0], r[:, T == oracle.RES_OUT][:, 0]
    assert ri[0] == pytest.approx(p.rho_minor, abs=1e-15)   # w minority at the inlet
    assert ro[1] == pytest.approx(p.rho_minor, abs=1e-15)   # nw minority at the outlet
    assert abs((pin[0] - pout[0]) - pc) <= 1e-14


def test_static_meniscus_bulk_pressures_equal_the_baths():
    """Below the entry pressure the meniscus stays in the throat and nothing
    flows: each bulk phase is at the pressure of the bath it touches, so the
    Eq. 5 pressures measured in the non-wetting bulk next to the inlet and in
    the wetting bulk next to the outlet differ by the imposed p_c (the
    diffuse interface's own pressure profile lies inside the throat)."""
    p = synth.constriction_problem()
    o = oracle.Oracle(p)
    pc = 0.3 * 2 * synth.GAMMA_LAPLACE / 6.0
    o.set_rho_in(o.rho_in_for_pc(pc))
    o.step(5000)
    P = o.pressure()
    T = o.types()
    u = o.velocity()
    # at rest away from the meniscus (the diffuse interface keeps its own
    # small stationary currents)
    for z in (1, -2):
        assert np.abs(u[:, z][:, T[z] == oracle.FLUID]).max() < 1e-3
    r = o.density()
    inlet_bulk = P[1][T[1] == oracle.FLUID]
    outlet_bulk = P[-2][T[-2] == oracle.FLUID]
    assert (r[1, 1] > r[0, 1])[T[1] == oracle.FLUID].all()      # nw next to the inlet
    assert (r[0, -2] > r[1, -2])[T[-2] == oracle.FLUID].all()   # w next to the outlet
    measured = inlet_bulk.mean() - outlet_bulk.mean()
    print("imposed p_c", pc, "bulk pressure difference", measured)
    assert abs(measured - pc) <= 0.03 * pc


# ---- the drainage ramp against a brute-force scan -------------------------

CONV = dict(tol=1e-5, check_every=100, max_steps=10000)


def _to_steady(o, tol, every, cap):
    """Plain run to steady state: check S_w every `every` steps, stop when it
    changed by less than tol or at the cap."""
    S_old = o.reduce()[1]
    n = 0
    while True:
        o.step(every)
        n += every
        S = o.reduce()[1]
        if abs(S - S_old) < tol or n >= cap:
            return S, n
        S_old = S


def test_drain_bracket_matches_a_fine_quasi_static_scan():
    """orc_drain on the slit throat: the ramp's first invaded point i has the
    bisected bracket inside (pc[i-1], pc[i]] and at most bisect_rel wide; the
    saturation never rises up to the invasion; the ramp points before invasion
    are the same steady states a plain quasi-static walk reaches; and a walk
    that continues from pc[i-1] in eight equal pressure steps is first
    invaded in the step interval that holds the bracket (the threshold does
    not depend on the path from below)."""
    p = synth.constriction_problem()
    p_hat = 2 * synth.GAMMA_LAPLACE / 6.0
    pcs = np.linspace(0.2, 1.4, 5) * p_hat
    rel = 0.02
    d = oracle.Oracle(p).drain(pcs, bisect_rel=rel, **CONV)
    i = d["invaded_at"]
    lo, hi = d["pce_lo"], d["pce_hi"]
    print("ramp S", d["S"], "invaded at", i, "bracket", lo, hi)
    assert i >= 1
    assert pcs[i - 1] <= lo < hi <= pcs[i]
    assert (hi - lo) / hi <= rel
    # quasi-static up to the first invasion; after breakthrough the
    # non-wetting phase flows on into the outlet bath and no static state
    # need exist (those points run to their cap)
    assert np.all(np.diff(d["S"][:i + 1]) <= 1e-6)

    # the quasi-static walk up to the last stable ramp point
    o = oracle.Oracle(p)
    for k in range(i):
        o.set_rho_in(o.rho_in_for_pc(pcs[k]))
        S, n = _to_steady(o, CONV["tol"], CONV["check_every"], CONV["max_steps"])
        assert S == d["S"][k] and n == d["steps"][k]
        assert not o.probe_invaded()
    stable = o.clone()
    # fine steps from pc[i-1] to pc[i]
    q = np.linspace(pcs[i - 1], pcs[i], 9)[1:]
    first = None
    for j, qq in enumerate(q):
        o.set_rho_in(o.rho_in_for_pc(qq))
        _to_steady(o, CONV["tol"], CONV["check_every"], CONV["max_steps"])
        if o.probe_invaded():
            first = j
            break
    assert first is not None
    q_lo = pcs[i - 1] if first == 0 else q[first - 1]
    q_hi = q[first]
    print("fine scan: first invaded between", q_lo, q_hi)
    assert lo < q_hi and hi > q_lo
    # the bracket's ends classify as reported when run from the last stable
    # ramp state
    for pr, want in ((lo, False), (hi, True)):
        t = stable.clone()
        t.set_rho_in(t.rho_in_for_pc(pr))
        _to_steady(t, CONV["tol"], CONV["check_every"], CONV["max_steps"])
        assert t.probe_invaded() == want, (pr, want)
