"""Pore network of a sphere packing (Sec. 2.2.1): the tetrahedra of the regular
triangulation are pore bodies, their shared facets pore throats.

Input generation only (geometry on the host): pores of the periodic cell, the
throats between them, and which throats open onto the two reservoirs of a
drainage experiment -- the non-wetting reservoir above the sample (z = L) and
the wetting reservoir below it (z = 0; the paper's porous membrane lets only
the wetting phase through).  The sample is periodic in x and y.
"""
import math

import numpy as np

from .packing import regular_triangulation

INLET, OUTLET = -1, -2


def _solid_angle(a, b, c):
    """Solid angle at the origin of the triangle (a, b, c) (Van Oosterom and
    Strackee, IEEE Trans. Biomed. Eng. 1983)."""
    la, lb, lc = np.linalg.norm(a), np.linalg.norm(b), np.linalg.norm(c)
    num = abs(np.dot(a, np.cross(b, c)))
    den = la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la
    return 2.0 * math.atan2(num, den)


def pore_void_volume(V, R):
    """Void volume of a tetrahedron with vertices V [4][3] at sphere centres of
    radii R [4]: its volume minus the four sphere sectors inside it (sphere
    overlaps inside the tetrahedron are neglected)."""
    vol = abs(np.dot(V[1] - V[0], np.cross(V[2] - V[0], V[3] - V[0]))) / 6.0
    solid = 0.0
    for i in range(4):
        o = [V[j] - V[i] for j in range(4) if j != i]
        solid += _solid_angle(*o) * R[i] ** 3 / 3.0
    return max(vol - solid, 0.0)


def pore_network(x, r, L):
    """Pores and throats of the periodic packing (centres x [n][3], radii r,
    cell side L).

    Returns a dict with
      pore_vol [m]          void volume of each pore (tetrahedra whose centroid
                            lies in the cell),
      pore_z [m]            centroid height,
      pore_xyz [m][3]       centroid of the tetrahedron's sphere centres,
      throats [k][2]        pore indices; INLET / OUTLET for a throat that opens
                            onto the reservoir above / below the sample,
      facets [k][3][4]      the three throat spheres (centre, radius) as placed
                            in the triangulation,
      apex [k][4]           the fourth sphere of the pore on the outlet side
                            (the lower one), the downstream pore of drainage.
    """
    P, R, I, tets = regular_triangulation(x, r, L)
    cen = P[tets].mean(axis=1)
    inside = np.all((cen >= 0) & (cen < L), axis=1)

    def key_of(t):
        # canonical identity of a tetrahedron up to periodic images in x, y:
        # its original sphere indices and its centroid wrapped into the cell
        c = cen[t].copy()
        c[:2] -= L * np.floor(c[:2] / L)
        return tuple(sorted(I[tets[t]])), tuple(np.round(c, 6))

    pore_of = {}
    pores = []
    for t in np.nonzero(inside)[0]:
        pore_of[key_of(t)] = len(pores)
        pores.append(t)
    pore_vol = np.array([pore_void_volume(P[tets[t]], R[tets[t]]) for t in pores])
    pore_xyz = np.array([cen[t] for t in pores]).reshape(-1, 3)
    pore_z = pore_xyz[:, 2].copy()

    def pore_index(t):
        c = cen[t]
        if c[2] >= L:
            return INLET
        if c[2] < 0:
            return OUTLET
        return pore_of.get(key_of(t))

    # facets of every in-cell tetrahedron; each shared facet once
    owners = {}
    for t in range(len(tets)):
        for k in range(4):
            f = tuple(sorted(np.delete(tets[t], k)))
            owners.setdefault(f, []).append((t, tets[t][k]))
    throats, facets, apex, seen = [], [], [], set()
    for f, own in owners.items():
        if len(own) != 2:
            continue
        (ta, va), (tb, vb) = own
        a, b = pore_index(ta), pore_index(tb)
        if a is None or b is None:
            continue
        if a < 0 and b < 0:
            continue
        if a < 0 or b < 0:
            # a reservoir throat is kept from the pore's side only
            if (a < 0 and not inside[tb]) or (b < 0 and not inside[ta]):
                continue
        elif not (inside[ta] or inside[tb]):
            continue
        ident = (min(a, b), max(a, b), tuple(sorted(I[list(f)])))
        if ident in seen:
            continue
        seen.add(ident)
        lower_is_a = cen[ta][2] <= cen[tb][2]
        throats.append((a, b))
        facets.append(np.column_stack([P[list(f)], R[list(f)]]))
        v = va if lower_is_a else vb
        apex.append(np.concatenate([P[v], [R[v]]]))
    return dict(pore_vol=pore_vol, pore_z=pore_z, pore_xyz=pore_xyz,
                throats=np.array(throats, dtype=np.int64),
                facets=np.array(facets), apex=np.array(apex))


def throat_problems(nw, res=12.0, side_range=(24, 64), amp=0.0, seed=7):
    """LBM subdomains of the network's throats: each facet with the apex of
    its downstream pore, mapped into a box as the packing throats are
    (synth.packing).  Returns (problems, incircle radii in lattice units,
    lattice units per packing length unit); a throat whose opening lies
    outside its triangle of centres gets None (no prism subdomain) and NaN
    for the other two values.  Also returns every throat's incircle radius in
    packing units (the opening's radius, for the incircle estimate)."""
    from .packing import _incircle_3d, _throat_problem
    probs, rins, scales, r_unit = [], [], [], []
    for k, (f, a) in enumerate(zip(nw["facets"], nw["apex"])):
        P = np.vstack([f[:, :3], a[:3]])
        R = np.concatenate([f[:, 3], [a[3]]])
        p, r_lu = _throat_problem(P, R, (0, 1, 2), 3, res, side_range, seed + k, amp)
        probs.append(p)
        rins.append(r_lu if p is not None else np.nan)
        scales.append(p.spheres[0, 3] / R[0] if p is not None else np.nan)
        r_unit.append(_incircle_3d(P, R, (0, 1, 2))[0])
    return probs, np.array(rins), np.array(scales), np.array(r_unit)
