"""Quasi-static drainage of a fully resolved sample (Sec. 3): the full-LBM
experiment that the hybrid pore-network result is checked against.

Host orchestration over the C-ABI only: every lattice step, reduction and
density read-back runs in the HIP library (lbm_step, lbm_reduce,
lbm_get_density).  Per imposed capillary pressure the inlet density is set
from Eq. 5, the lattice is stepped in chunks until the whole-domain wetting
saturation changes by less than `tol` over a chunk (or `max_steps` is
reached), and the saturation is then measured over the packing slab alone,
so that the non-wetting buffer at the inlet and the wetting layer behind the
membrane do not dilute it.
"""
import time

import numpy as np

from . import lbm


def region_saturation(rho, types, z0, z1, rho_major, rho_minor, sharp=False):
    """Wetting saturation over the fluid nodes of planes z0..z1 from component
    densities rho [2][nz][ny][nx] (wetting first): the mean of
    (phi / phi_b + 1) / 2 with phi = (rho_w - rho_nw) / (rho_w + rho_nw) and
    phi_b its bulk value (the library's saturation map); with `sharp`, the
    fraction of nodes where the wetting component is the denser one (the
    diffuse interface then counts by the side of its midpoint)."""
    w, nw = rho[0, z0:z1 + 1], rho[1, z0:z1 + 1]
    live = types[z0:z1 + 1] == lbm.LBM_NODE_FLUID
    if sharp:
        return float(np.mean(w[live] > nw[live]))
    phib = (rho_major - rho_minor) / (rho_major + rho_minor)
    phi = (w[live] - nw[live]) / (w[live] + nw[live])
    return float(np.mean((phi / phib + 1.0) / 2.0))


def ball_nodes(points, radius, shape):
    """Flat indices of the nodes within `radius` of each lattice point
    (float coordinates [m][3], x y z), wrapped on x and y (periodic) and
    clipped on z: a list of index arrays."""
    nz, ny, nx = shape
    r = int(np.ceil(radius))
    d = np.arange(-r, r + 1)
    out = []
    for X, Y, Z in np.asarray(points, dtype=np.float64):
        cx, cy, cz = np.floor([X, Y, Z]).astype(int)
        gz, gy, gx = np.meshgrid(cz + d, cy + d, cx + d, indexing="ij")
        near = (gx - X) ** 2 + (gy - Y) ** 2 + (gz - Z) ** 2 <= radius * radius
        near &= (gz >= 0) & (gz < nz)
        out.append(((gz[near] * ny + np.mod(gy[near], ny)) * nx + np.mod(gx[near], nx)))
    return out


def drain_sample(prob, pressures, slab, membrane_z, tol=1e-5, check_every=200, max_steps=30000,
                 autotune=True, points=None, radius=2.0, log=None):
    """Ramp `pressures` (lattice units, increasing) on the sample `prob`.

    Returns dict(S_slab, S_slab_sharp, S_outlet (behind the membrane),
    steps, converged) per pressure, plus the launch schedule,
    the lattice steps and the wall time.  With `points` (lattice coordinates
    [m][3]), also S_points [n_p][m]: the saturation over the fluid nodes
    within `radius` of each point (NaN where there are none)."""
    g = lbm.Throat(prob)
    try:
        sched = g.autotune(5) if autotune else g.schedule()
        types = g.types()
        out = dict(S_slab=[], S_slab_sharp=[], S_outlet=[], steps=[], converged=[],
                   S_points=[])
        balls = None
        if points is not None:
            flat_t = types.reshape(-1)
            balls = [b[flat_t[b] == lbm.LBM_NODE_FLUID]
                     for b in ball_nodes(points, radius, types.shape)]
            phib = (prob.rho_major - prob.rho_minor) / (prob.rho_major + prob.rho_minor)
        total = 0
        t0 = time.perf_counter()
        for pc in pressures:
            g.set_rho_in(g.rho_in_for_pc(float(pc)))
            prev, n, ok = None, 0, False
            while n < max_steps:
                g.step(check_every)
                n += check_every
                _, S = g.reduce()
                if prev is not None and abs(S - prev) < tol:
                    ok = True
                    break
                prev = S
            total += n
            rho = g.density()
            a = (prob.rho_major, prob.rho_minor)
            out["S_slab"].append(region_saturation(rho, types, slab[0], slab[1], *a))
            out["S_slab_sharp"].append(
                region_saturation(rho, types, slab[0], slab[1], *a, sharp=True))
            out["S_outlet"].append(region_saturation(rho, types, membrane_z + 1, prob.nz - 2, *a))
            if balls is not None:
                w, nw = rho[0].reshape(-1), rho[1].reshape(-1)
                out["S_points"].append([
                    float(np.mean(((w[b] - nw[b]) / (w[b] + nw[b]) / phib + 1.0) / 2.0))
                    if b.size else float("nan") for b in balls])
            out["steps"].append(n)
            out["converged"].append(ok)
            if log:
                log(f"sample drain: pc {pc:.5f}: S_slab {out['S_slab'][-1]:.4f} after {n} steps")
        out["wall_s"] = time.perf_counter() - t0
        out["lattice_steps"] = total
        out["schedule"] = list(sched)
        return out
    finally:
        g.close()
