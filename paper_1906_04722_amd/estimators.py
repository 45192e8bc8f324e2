"""Closed-form entry-pressure estimates of a throat of three equal spheres in
mutual contact (the paper's example throat, Sec. 2.2.2), for a perfectly
wetting solid.  Both are the cheap estimates the paper contrasts with its LBM
throats (Sec. 1, the incircle and the Mayer-Stowe-Princen methods); they serve
as references for the LBM's p_c^e, not as part of the hot path.

Cross-section: the plane of the sphere centres, where the pore is the
curvilinear triangle between three touching circles of radius R.

* Incircle: the largest circle in the pore, radius r_in = R (2/sqrt(3) - 1),
  and p_c = 2 gamma / r_in (a spherical meniscus through that circle).
* MS-P (Mayer & Stowe 1965; Princen 1969): the non-wetting phase enters a
  straight tube of this cross-section at p_c = gamma / r, where r is the
  radius of the wetting-phase menisci left in the three corners and
  satisfies the force balance p_c A_n = gamma (L_nw + L_ns cos(theta)) with
  theta = 0: A_n is the area the non-wetting phase takes, L_nw the length of
  the corner menisci and L_ns that of its contact with the solid.  A corner
  meniscus is the arc of the circle of radius r tangent to both circles of
  its corner; with alpha = arccos(R / (R + r)) the half-angle it subtends at
  a sphere centre and beta = pi - 2 alpha its angle at its own centre:
    corner area   = R sqrt((R + r)^2 - R^2) - R^2 alpha - r^2 beta / 2,
    A_n           = (sqrt(3) - pi / 2) R^2 - 3 corner area,
    L_nw + L_ns   = 3 r beta + 3 R (pi / 3 - 2 alpha).
"""
import math

from scipy.optimize import brentq


def incircle_radius(R):
    """Radius of the opening between three touching circles of radius R."""
    return R * (2.0 / math.sqrt(3.0) - 1.0)


def msp_parts(R, r):
    """(A_n, L_nw + L_ns) of the MS-P balance for corner menisci of radius r."""
    a = math.acos(R / (R + r))
    b = math.pi - 2.0 * a
    corner = R * math.sqrt((R + r) ** 2 - R * R) - R * R * a - 0.5 * r * r * b
    area = (math.sqrt(3.0) - 0.5 * math.pi) * R * R - 3.0 * corner
    length = 3.0 * r * b + 3.0 * R * (math.pi / 3.0 - 2.0 * a)
    return area, length


def msp_radius(R):
    """Corner-meniscus radius r at entry: the root of A_n = r (L_nw + L_ns)
    between 0 and the incircle radius (where the menisci close the pore)."""
    return brentq(lambda r: msp_parts(R, r)[0] - r * msp_parts(R, r)[1],
                  1e-6 * R, incircle_radius(R), xtol=1e-14 * R)


def opening_radius(circles):
    """Radius of the circle tangent from outside to three circles [(x, y, R)]
    in their gap (the throat opening; the incircle estimate's radius): the
    tangency conditions |c - C_i| = r + R_i subtracted pairwise make the
    centre linear in r, and the first condition leaves a quadratic whose
    smallest positive root is the gap circle.  NaN if there is none."""
    C = [(float(c[0]), float(c[1])) for c in circles]
    R = [float(c[2]) for c in circles]
    A, b, d = [], [], []
    for i in (1, 2):
        A.append((2.0 * (C[0][0] - C[i][0]), 2.0 * (C[0][1] - C[i][1])))
        b.append(R[i] ** 2 - R[0] ** 2 - (C[i][0] ** 2 + C[i][1] ** 2) + (C[0][0] ** 2 + C[0][1] ** 2))
        d.append(2.0 * (R[i] - R[0]))
    det = A[0][0] * A[1][1] - A[0][1] * A[1][0]
    if det == 0.0:
        return float("nan")
    u = ((A[1][1] * b[0] - A[0][1] * b[1]) / det, (A[0][0] * b[1] - A[1][0] * b[0]) / det)
    v = ((A[1][1] * d[0] - A[0][1] * d[1]) / det, (A[0][0] * d[1] - A[1][0] * d[0]) / det)
    w = (u[0] - C[0][0], u[1] - C[0][1])
    qa = v[0] ** 2 + v[1] ** 2 - 1.0
    qb = 2.0 * (w[0] * v[0] + w[1] * v[1] - R[0])
    qc = w[0] ** 2 + w[1] ** 2 - R[0] ** 2
    if abs(qa) < 1e-14:
        roots = [-qc / qb] if qb != 0.0 else []
    else:
        disc = qb * qb - 4.0 * qa * qc
        roots = [] if disc < 0 else [(-qb - math.sqrt(disc)) / (2.0 * qa),
                                     (-qb + math.sqrt(disc)) / (2.0 * qa)]
    pos = [r for r in roots if r > 0]
    return min(pos) if pos else float("nan")


def pc_star(pc, R, gamma):
    """The paper's normalised capillary pressure p_c* = 2 p_c R / gamma."""
    return 2.0 * pc * R / gamma


def v_star(volume, R):
    """The paper's normalised volume V* = V / (4/3 pi R^3)."""
    return volume / (4.0 / 3.0 * math.pi * R ** 3)


# ---- MS-P for any throat of three circles in a prism ------------------------
# The cross-section through the three sphere centres: the triangle of centres
# (the prism's walls run along its edges) minus the disks of radii R_i.  For
# corner menisci of radius r the wetting phase holds:
#   * where two disks overlap or touch, the corner between them, closed by the
#     arc of the circle of radius r tangent to both;
#   * where they leave a gap on their edge, the two 90-degree corners between
#     each disk and the wall, each closed by the arc of radius r tangent to the
#     disk and the wall; once those two arcs would meet, the whole gap, closed
#     by the arc tangent to both disks (the wall is then wetted over the gap).
# The non-wetting phase takes the rest, A_n, bounded by the arcs (L_nw), the
# disks' remaining arcs and the dry wall segments (L_ns); MS-P entry is the
# root of A_n = r (L_nw + L_ns), p_c = gamma / r.

def _half_lens(a, b, d):
    """Half the area of the intersection of disks of radii a, b at distance d."""
    if d >= a + b:
        return 0.0
    ca = max(-1.0, min(1.0, (d * d + a * a - b * b) / (2.0 * d * a)))
    cb = max(-1.0, min(1.0, (d * d + b * b - a * a) / (2.0 * d * b)))
    k = max(0.0, (-d + a + b) * (d + a - b) * (d - a + b) * (d + a + b))
    return 0.5 * (a * a * math.acos(ca) + b * b * math.acos(cb) - 0.5 * math.sqrt(k))


def _vertex_angle(p, q, s):
    u = (q[0] - p[0], q[1] - p[1])
    v = (s[0] - p[0], s[1] - p[1])
    c = (u[0] * v[0] + u[1] * v[1]) / (math.hypot(*u) * math.hypot(*v))
    return math.acos(max(-1.0, min(1.0, c)))


def pore_area(circles):
    """Area of the triangle of centres minus the disks (pairwise overlaps
    counted once; the three disks are assumed not to share a point inside)."""
    C = [(float(c[0]), float(c[1])) for c in circles]
    R = [float(c[2]) for c in circles]
    area = 0.5 * abs((C[1][0] - C[0][0]) * (C[2][1] - C[0][1]) -
                     (C[2][0] - C[0][0]) * (C[1][1] - C[0][1]))
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        area -= 0.5 * R[i] * R[i] * _vertex_angle(C[i], C[j], C[k])
        area += _half_lens(R[i], R[j], math.dist(C[i], C[j]))
    return area


def msp_general_parts(circles, r):
    """(A_n, L_nw + L_ns, valid) for corner menisci of radius r; valid is False
    when the menisci would overlap (r beyond the geometry's range)."""
    C = [(float(c[0]), float(c[1])) for c in circles]
    R = [float(c[2]) for c in circles]
    theta = [_vertex_angle(C[i], C[(i + 1) % 3], C[(i + 2) % 3]) for i in range(3)]
    used = [0.0, 0.0, 0.0]
    wet = 0.0
    length = 0.0
    for i in range(3):
        j = (i + 1) % 3
        d = math.dist(C[i], C[j])
        bridged = R[i] + R[j] >= d
        if not bridged:
            fi = math.sqrt((R[i] + r) ** 2 - r * r)
            fj = math.sqrt((R[j] + r) ** 2 - r * r)
            if fi + fj <= d:
                for f, q in ((fi, i), (fj, j)):
                    g = math.atan2(r, f)
                    wet += 0.5 * f * r - 0.5 * R[q] ** 2 * g - 0.5 * r * r * (0.5 * math.pi - g)
                    length += r * (0.5 * math.pi - g)
                    used[q] += g
                length += d - fi - fj
                continue
        a, b = R[i] + r, R[j] + r
        ai = math.acos(max(-1.0, min(1.0, (d * d + a * a - b * b) / (2.0 * d * a))))
        aj = math.acos(max(-1.0, min(1.0, (d * d + b * b - a * a) / (2.0 * d * b))))
        beta = math.pi - ai - aj
        wet += (0.5 * d * a * math.sin(ai) - 0.5 * R[i] ** 2 * ai - 0.5 * R[j] ** 2 * aj -
                0.5 * r * r * beta + _half_lens(R[i], R[j], d))
        length += r * beta
        used[i] += ai
        used[j] += aj
    valid = True
    for i in range(3):
        rest = theta[i] - used[i]
        valid &= rest >= 0.0
        length += R[i] * max(rest, 0.0)
    An = pore_area(circles) - wet
    return An, length, valid and An > 0.0


def msp_general_radius(circles):
    """MS-P corner-meniscus radius at entry for three circles [(x, y, R)] at
    the prism's corners (NaN where no root lies in the valid range)."""
    scale = max(float(c[2]) for c in circles)
    f = lambda r: msp_general_parts(circles, r)[0] - r * msp_general_parts(circles, r)[1]
    lo = 1e-6 * scale
    if f(lo) <= 0.0:
        return float("nan")
    r = lo
    while True:
        nxt = r * 1.15
        An, L, ok = msp_general_parts(circles, nxt)
        if not ok:
            return float("nan")
        if An - nxt * L < 0.0:
            return brentq(f, r, nxt, xtol=1e-13 * scale)
        r = nxt
        if r > 10.0 * scale:
            return float("nan")
