"""Seeded dense random sphere packings and the pore throats cut from them.

Sec. 2.2.1: the pore space of a sphere packing is decomposed by a regular
triangulation whose vertices are the sphere centres; each tetrahedron is a
pore body and each of its facets a pore throat (Sec. 2.2.2: each throat is
solved on its own small subdomain, a prism over the three facet spheres).
The paper builds its packing with YADE (Sec. 3.1.1); here a seeded
overlap-removal relaxation stands in for it.

Everything here is input generation on the host (not timed): sphere
positions, the triangulation (the lower convex hull of the points lifted to
(x, |x|^2 - r^2), i.e. the weighted Delaunay triangulation), and the mapping
of one facet plus its downstream apex sphere into a throat box.
"""
import math

import numpy as np
from scipy.spatial import ConvexHull, cKDTree

from .fields import layered_density
from .rng import uniform01
from .spec import BC_RESERVOIR, BC_WALLS, Problem
from .throats import _normals, throat_incircle


def dense_packing(n=500, mean_r=1.0, sigma=0.2, solid_fraction=0.62, seed=3, tol=1e-4,
                  max_iter=20000, side=None):
    """n spheres with lognormal radii (arithmetic mean mean_r, log-sd sigma)
    relaxed to no overlap in a periodic cube whose side gives the requested
    solid fraction (or of the given side, the solid fraction then following
    from the radii).  Returns (centres [n][3], radii [n], box side, achieved
    solid fraction, largest remaining overlap / mean radius)."""
    z = _normals(seed, n)
    r = np.exp(math.log(mean_r) - 0.5 * sigma * sigma + sigma * z)
    vol = (4.0 / 3.0) * math.pi * (r ** 3).sum()
    L = float(side) if side is not None else (vol / solid_fraction) ** (1.0 / 3.0)
    x = uniform01(seed + 77, 3 * n).reshape(n, 3) * L
    rmax = r.max()
    worst = np.inf
    for _ in range(max_iter):
        x %= L
        tree = cKDTree(x, boxsize=L)
        pairs = tree.query_pairs(2.0 * rmax, output_type="ndarray")
        if len(pairs) == 0:
            worst = 0.0
            break
        i, j = pairs[:, 0], pairs[:, 1]
        d = x[j] - x[i]
        d -= L * np.round(d / L)
        dist = np.linalg.norm(d, axis=1)
        ov = r[i] + r[j] - dist
        m = ov > 0
        worst = ov[m].max() / mean_r if m.any() else 0.0
        if worst < tol:
            break
        i, j, d, dist, ov = i[m], j[m], d[m], dist[m], ov[m]
        u = d / np.maximum(dist, 1e-12)[:, None]
        # each sphere of an overlapping pair moves half the overlap apart,
        # weighted so the larger sphere moves less
        wi = r[j] ** 3 / (r[i] ** 3 + r[j] ** 3)
        wj = 1.0 - wi
        dx = np.zeros_like(x)
        np.add.at(dx, i, -(0.55 * ov * wi)[:, None] * u)
        np.add.at(dx, j, (0.55 * ov * wj)[:, None] * u)
        x += dx
    x %= L
    return x, r, L, vol / L ** 3, worst


def regular_triangulation(x, r, L, margin=None):
    """Tetrahedra of the regular (weighted Delaunay) triangulation of a
    periodic packing: periodic images within `margin` of the cell are added,
    the points are lifted to (x, |x|^2 - r^2) and the lower convex hull is
    taken.  Returns (points [m][3], radii [m], original index [m],
    tetrahedra [k][4] into the point list)."""
    if margin is None:
        margin = 4.0 * r.max()
    pts, rad, idx = [x], [r], [np.arange(len(x))]
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            for sz in (-1, 0, 1):
                if sx == sy == sz == 0:
                    continue
                y = x + L * np.array([sx, sy, sz])
                keep = np.all((y > -margin) & (y < L + margin), axis=1)
                pts.append(y[keep])
                rad.append(r[keep])
                idx.append(np.nonzero(keep)[0])
    P = np.concatenate(pts)
    R = np.concatenate(rad)
    I = np.concatenate(idx)
    lifted = np.column_stack([P, (P * P).sum(1) - R * R])
    hull = ConvexHull(lifted)
    lower = hull.equations[:, 3] < 0
    return P, R, I, hull.simplices[lower]


def interior_facets(P, tets, L):
    """Facets shared by two tetrahedra whose centroid lies in the periodic
    cell: (facet vertex triple, apex of one side, apex of the other side)."""
    owners = {}
    for t in tets:
        for k in range(4):
            f = tuple(sorted(np.delete(t, k)))
            owners.setdefault(f, []).append(t[k])
    out = []
    for f, ap in owners.items():
        if len(ap) != 2:
            continue
        c = P[list(f)].mean(0)
        if np.all((c >= 0) & (c < L)):
            out.append((f, ap[0], ap[1]))
    return out


def _throat_problem(P, R, facet, apex, res, side_range, seed, amp):
    """One facet and its downstream apex mapped into a throat box: facet
    plane normal to z near the inlet, apex above it, the triangle of facet
    centres centred in xy with its longest edge along x, `res` lattice units per unit length (reduced if
    the box would exceed the largest side).  Returns (problem or None when no
    pore-body probe exists, incircle radius in lattice units)."""
    tri = P[list(facet)]
    c0 = tri.mean(0)
    nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    nrm /= np.linalg.norm(nrm)
    if np.dot(P[apex] - c0, nrm) < 0:
        nrm = -nrm
    # x along the longest facet edge: the prism's bounding rectangle is then
    # about half the area of a square around the triangle
    ij = max(((0, 1), (1, 2), (2, 0)), key=lambda e: np.linalg.norm(tri[e[1]] - tri[e[0]]))
    e1 = tri[ij[1]] - tri[ij[0]]
    e1 -= np.dot(e1, nrm) * nrm
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(nrm, e1)
    frame = np.stack([e1, e2, nrm])
    loc = (np.vstack([tri, P[apex]]) - c0) @ frame.T  # facet spheres at z = 0
    rad = np.concatenate([R[list(facet)], [R[apex]]])
    h = loc[3, 2]
    lo_xy = loc[:3, :2].min(0)
    span = loc[:3, :2].max(0) - lo_xy
    lo, hi = side_range
    # the prism over the facet triangle plus a two-node border in x and y;
    # inlet bath, facet at 0.3 nz, apex centre below 0.9 nz
    ext = max(span.max(), h / 0.6)
    scale = res if ext * res + 6.0 <= hi else (hi - 6.0) / ext
    nx, ny = (int(min(hi, max(lo, math.ceil(s_ * scale) + 5))) for s_ in span)
    nz = int(min(hi, max(lo, math.ceil(h / 0.6 * scale) + 6)))
    sph = np.zeros((4, 4))
    sph[:, :3] = loc * scale
    sph[:, 3] = rad * scale
    zf = 0.3 * nz
    sph[:, 0] += (nx - 1) / 2.0 - (lo_xy[0] + 0.5 * span[0]) * scale
    sph[:, 1] += (ny - 1) / 2.0 - (lo_xy[1] + 0.5 * span[1]) * scale
    sph[:, 2] += zf
    # pore-body probe: on the axis of the throat opening (the incircle centre,
    # inside the prism), halfway up to the apex, nudged along z to the nearest
    # node outside every sphere
    r_in, (cx, cy) = throat_incircle(sph)
    z0 = zf + 0.5 * h * scale
    probe = None
    # an obtuse facet can put the opening outside the triangle of centres,
    # where the prism closure would cut through it: such facets get no probe
    # and are skipped
    tri2 = sph[:3, :2]

    def edge_dist(q):
        """Signed distances of the xy point q to the triangle's edge lines,
        positive inside for either orientation."""
        d = []
        for i in range(3):
            a, b = tri2[i], tri2[(i + 1) % 3]
            d.append(((b[0] - a[0]) * (q[1] - a[1]) - (b[1] - a[1]) * (q[0] - a[0]))
                     / np.linalg.norm(b - a))
        return np.array(d) if sum(d) > 0 else -np.array(d)

    inside = edge_dist(np.array([cx, cy])).min() > 1.0
    q_xy = np.floor(np.array([cx, cy]) + 0.5)
    inside = inside and edge_dist(q_xy).min() > 1.0
    for dz in [] if not inside else np.concatenate([[0.0], np.ravel(np.column_stack([np.arange(1, nz), -np.arange(1, nz)])) * 0.5]):
        q = np.array([q_xy[0], q_xy[1], math.floor(z0 + dz + 0.5)])
        if not (zf + 1 < q[2] < nz - 2):
            continue
        d2 = ((sph[:, :3] - q) ** 2).sum(1)
        if np.all(d2 > sph[:, 3] ** 2 + 1.0):
            probe = tuple(int(v) for v in q)
            break
    if probe is None:
        return None, r_in
    p = Problem(nx=nx, ny=ny, nz=nz, bc=(BC_WALLS, BC_WALLS, BC_RESERVOIR), spheres=sph,
                prism_ids=(0, 1, 2), rho_in_nw=2.0, rho_out_w=2.0, z_front=2, probe=probe)
    if amp:
        p.rho_init = layered_density(nx, ny, nz, p.z_front, p.rho_major, p.rho_minor, seed, amp)
    return p, r_in


def packing_throats(n_throats=512, n_spheres=600, seed=3, res=32.0, side_range=(48, 128),
                    min_incircle=0.05, amp=1e-3):
    """Throat problems cut from a seeded dense packing (radii lognormal, mean
    1.0, log-sd 0.2, solid fraction 0.62): `n_throats` interior facets drawn
    without replacement, each mapped into a box with sides in `side_range`.
    amp > 0 adds the seeded +-amp density perturbation to the layered initial
    state; amp = 0 leaves it unperturbed (no initial-density array).
    Returns (problems, incircle radii in lattice units, packing summary)."""
    x, r, L, phi, worst = dense_packing(n_spheres, seed=seed)
    P, R, I, tets = regular_triangulation(x, r, L)
    facets = interior_facets(P, tets, L)
    order = np.argsort(uniform01(seed + 5, len(facets)), kind="stable")
    probs, rins = [], []
    for k in order:
        f, a, b = facets[k]
        r_in, _ = _incircle_3d(P, R, f)
        if not (r_in > min_incircle):
            continue
        p, r_lu = _throat_problem(P, R, f, a, res, side_range, seed + 1000 + len(probs), amp)
        if p is None:
            continue
        probs.append(p)
        rins.append(r_lu)
        if len(probs) == n_throats:
            break
    summary = dict(n_spheres=n_spheres, box=L, solid_fraction=phi, porosity=1.0 - phi,
                   max_overlap=worst, tetrahedra=len(tets), interior_facets=len(facets))
    return probs, np.array(rins), summary


def _incircle_3d(P, R, facet):
    """Radius of the circle in the facet plane tangent to the three sphere
    sections through their centres."""
    tri = P[list(facet)]
    c0 = tri.mean(0)
    e1 = tri[1] - tri[0]
    e1 /= np.linalg.norm(e1)
    nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    nrm /= np.linalg.norm(nrm)
    e2 = np.cross(nrm, e1)
    loc = np.column_stack([(tri - c0) @ e1, (tri - c0) @ e2, np.zeros(3), R[list(facet)]])
    return throat_incircle(loc)


def packed_sample(n=512, n_spheres=1000, seed=4, nz=None, probe_depth=6):
    """A fully resolved sample: a seeded dense packing (radii lognormal, mean
    1, log-sd 0.2, solid fraction 0.62) scaled so its periodic cell fills an
    n x n x nz box (nz = n by default), its periodic images that reach into
    the box included, walls on the four sides and baths at z = 0 (non-wetting
    inlet) and z = nz - 1 (wetting outlet).  The invasion probe is a fluid
    node near the outlet.  Returns (problem, packing summary)."""
    nz = n if nz is None else nz
    x, r, L, phi, worst = dense_packing(n_spheres, seed=seed)
    box = np.array([n, n, nz], dtype=np.float64)
    scale = box / L
    # one isotropic scale keeps spheres round: the smallest axis ratio
    s = float(scale.min())
    pts, rad = [], []
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            for sz in (-1, 0, 1):
                c = (x + L * np.array([sx, sy, sz])) * s
                rr = r * s
                keep = np.all((c + rr[:, None] > -1.0) & (c - rr[:, None] < box + 1.0), axis=1)
                pts.append(c[keep])
                rad.append(rr[keep])
    C = np.concatenate(pts)
    R = np.concatenate(rad)
    sph = np.column_stack([C, R])
    probe = None
    cx, cy = (n - 1) // 2, (n - 1) // 2
    for d in range(0, n // 2):
        for q in ((cx + d, cy, nz - 1 - probe_depth), (cx, cy + d, nz - 1 - probe_depth),
                  (cx - d, cy, nz - 1 - probe_depth), (cx, cy - d, nz - 1 - probe_depth)):
            d2 = ((C - np.array(q, dtype=np.float64)) ** 2).sum(1)
            if np.all(d2 > R * R + 1.0):
                probe = tuple(int(v) for v in q)
                break
        if probe is not None:
            break
    p = Problem(nx=n, ny=n, nz=nz, bc=(BC_WALLS, BC_WALLS, BC_RESERVOIR), spheres=sph,
                prism_ids=None, rho_in_nw=2.0, rho_out_w=2.0, z_front=2, probe=probe)
    summary = dict(n_spheres=n_spheres, spheres_in_box=len(R), scale=s, solid_fraction=phi,
                   max_overlap=worst, mean_radius_lu=float(r.mean() * s))
    return p, summary
