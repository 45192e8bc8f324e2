"""Entry-pressure estimates of the three-touching-sphere throat, pinned by
brute force: areas by sampling the cross-section on a fine grid, arc lengths
from explicitly constructed tangent points, and the incircle by the
tangency it must have."""
import math

import numpy as np
import pytest

from paper_1906_04722_amd import estimators as est

R = 1.0
C = np.array([[0.0, 0.0], [2.0 * R, 0.0], [R, math.sqrt(3.0) * R]])
G = C.mean(axis=0)


def test_incircle_is_tangent_to_the_three_circles():
    r = est.incircle_radius(R)
    assert np.allclose(np.hypot(*(C - G).T), R + r, rtol=0, atol=1e-15)


def _meniscus_centre(i, j, r):
    """Centre of the circle of radius r tangent to circles i and j, inside."""
    m = 0.5 * (C[i] + C[j])
    n = G - m
    n /= np.hypot(*n)
    return m + n * math.sqrt((R + r) ** 2 - R * R)


@pytest.mark.parametrize("r", [0.03, 0.0883, 0.13])
def test_msp_area_by_sampling(r):
    h = 1.5e-3
    xs = np.arange(0.0, 2.0 * R, h) + h / 2
    ys = np.arange(0.0, math.sqrt(3.0) * R, h) + h / 2
    X, Y = np.meshgrid(xs, ys)
    inside_tri = (Y <= math.sqrt(3.0) * X) & (Y <= math.sqrt(3.0) * (2.0 * R - X))
    pore = inside_tri.copy()
    for c in C:
        pore &= (X - c[0]) ** 2 + (Y - c[1]) ** 2 > R * R
    corner = np.zeros_like(pore)
    for i, j in ((0, 1), (1, 2), (2, 0)):
        m = _meniscus_centre(i, j, r)
        # the wetting corner: pore points on the contact side of the meniscus
        # circle, inside the triangle (c_i, c_j, meniscus centre)
        a, b, c = C[i], C[j], m
        d1 = (b[0] - a[0]) * (Y - a[1]) - (b[1] - a[1]) * (X - a[0])
        d2 = (c[0] - b[0]) * (Y - b[1]) - (c[1] - b[1]) * (X - b[0])
        d3 = (a[0] - c[0]) * (Y - c[1]) - (a[1] - c[1]) * (X - c[0])
        tri = ((d1 >= 0) & (d2 >= 0) & (d3 >= 0)) | ((d1 <= 0) & (d2 <= 0) & (d3 <= 0))
        corner |= pore & tri & ((X - m[0]) ** 2 + (Y - m[1]) ** 2 > r * r)
    An_sampled = (pore & ~corner).sum() * h * h
    An, _ = est.msp_parts(R, r)
    assert abs(An_sampled - An) < 2e-3 * (math.sqrt(3.0) - math.pi / 2)


@pytest.mark.parametrize("r", [0.03, 0.0883, 0.13])
def test_msp_lengths_from_tangent_points(r):
    total = 0.0
    tang = {}
    for i, j in ((0, 1), (1, 2), (2, 0)):
        m = _meniscus_centre(i, j, r)
        ti = C[i] + R * (m - C[i]) / np.hypot(*(m - C[i]))
        tj = C[j] + R * (m - C[j]) / np.hypot(*(m - C[j]))
        u, v = ti - m, tj - m
        total += r * math.acos(np.dot(u, v) / (r * r))          # meniscus arc
        tang.setdefault(i, []).append(ti)
        tang.setdefault(j, []).append(tj)
    for i, (p, q) in tang.items():                                # solid arcs
        u, v = p - C[i], q - C[i]
        total += R * math.acos(np.clip(np.dot(u, v) / (R * R), -1.0, 1.0))
    _, L = est.msp_parts(R, r)
    assert abs(total - L) < 1e-12


def test_msp_root_and_its_place_below_the_incircle():
    r = est.msp_radius(R)
    An, L = est.msp_parts(R, r)
    assert abs(An - r * L) < 1e-13
    # the corner menisci are open (0 < r < r_in) and the estimate lies below
    # the incircle one: p = gamma / r against 2 gamma / r_in
    r_in = est.incircle_radius(R)
    assert 0.0 < r < r_in
    ratio = (1.0 / r) / (2.0 / r_in)
    assert 0.8 < ratio < 0.95
    # scale invariance
    assert est.msp_radius(7.0) == pytest.approx(7.0 * r, rel=1e-12)
    # the paper's normalisation p* = 2 p R / gamma
    assert est.pc_star(1.0 / r, R, 1.0) == pytest.approx(2.0 / r)


def _opening(circles, r, h):
    """Sampled MS-P non-wetting region: the union of the disks of radius r
    that fit in the pore (triangle of centres minus the circles)."""
    from scipy.ndimage import distance_transform_edt as edt
    C = np.array([[c[0], c[1]] for c in circles])
    R = np.array([c[2] for c in circles])
    lo, hi = C.min(axis=0) - h, C.max(axis=0) + h
    xs = np.arange(lo[0], hi[0], h)
    ys = np.arange(lo[1], hi[1], h)
    X, Y = np.meshgrid(xs, ys)
    a, b, c = C
    d1 = (b[0] - a[0]) * (Y - a[1]) - (b[1] - a[1]) * (X - a[0])
    d2 = (c[0] - b[0]) * (Y - b[1]) - (c[1] - b[1]) * (X - b[0])
    d3 = (a[0] - c[0]) * (Y - c[1]) - (a[1] - c[1]) * (X - c[0])
    pore = ((d1 >= 0) & (d2 >= 0) & (d3 >= 0)) | ((d1 <= 0) & (d2 <= 0) & (d3 <= 0))
    for (x, y), rr in zip(C, R):
        pore &= (X - x) ** 2 + (Y - y) ** 2 > rr * rr
    centres = edt(pore) * h >= r
    return edt(~centres) * h <= r, pore


def _constructed_length(circles, r):
    """L_nw + L_ns from the boundary built point by point: meniscus centres,
    tangent points on the circles and feet on the walls, arc angles by
    atan2, dry wall segments as distances between feet."""
    C = np.array([[c[0], c[1]] for c in circles], dtype=float)
    R = np.array([c[2] for c in circles], dtype=float)
    G = C.mean(axis=0)
    ang = lambda u, v: abs(math.atan2(u[0] * v[1] - u[1] * v[0], u[0] * v[0] + u[1] * v[1]))
    touch = {0: [], 1: [], 2: []}          # tangent points per circle
    total = 0.0
    for i in range(3):
        j = (i + 1) % 3
        e = (C[j] - C[i]) / np.linalg.norm(C[j] - C[i])
        n = np.array([-e[1], e[0]])
        if np.dot(G - C[i], n) < 0:
            n = -n                          # toward the pore
        d = np.linalg.norm(C[j] - C[i])
        fi = math.sqrt((R[i] + r) ** 2 - r * r)
        fj = math.sqrt((R[j] + r) ** 2 - r * r)
        if R[i] + R[j] < d and fi + fj <= d:
            for q, f, sgn in ((i, fi, 1.0), (j, fj, -1.0)):
                foot = C[q] + sgn * f * e
                m = foot + r * n
                t = C[q] + R[q] * (m - C[q]) / np.linalg.norm(m - C[q])
                total += r * ang(t - m, foot - m)
                touch[q].append(t)
            total += d - fi - fj
        else:
            # the point at distances R_i + r and R_j + r, on the pore side
            a, b = R[i] + r, R[j] + r
            x = (d * d + a * a - b * b) / (2.0 * d)
            m = C[i] + x * e + math.sqrt(a * a - x * x) * n
            ti = C[i] + R[i] * (m - C[i]) / a
            tj = C[j] + R[j] * (m - C[j]) / b
            total += r * ang(ti - m, tj - m)
            touch[i].append(ti)
            touch[j].append(tj)
    for q in range(3):
        t1, t2 = touch[q]
        total += R[q] * ang(t1 - C[q], t2 - C[q])
    return total


GENERAL = [
    # a gap on two edges (wall corners), touching on none
    ([(0.0, 0.0, 1.0), (2.4, 0.0, 0.9), (1.1, 2.0, 1.2)], [0.05, 0.15]),
    # one overlapping pair, one gap
    ([(0.0, 0.0, 1.0), (2.1, 0.2, 1.3), (0.9, 2.2, 0.8)], [0.06, 0.16]),
]


@pytest.mark.parametrize("circles,rs", GENERAL)
def test_general_msp_parts_by_sampling(circles, rs):
    h = 1.2e-3
    for r in rs:
        An, L, ok = est.msp_general_parts(circles, r)
        assert ok
        opened, pore = _opening(circles, r, h)
        assert abs(pore.sum() * h * h - est.pore_area(circles)) < 3e-3 * est.pore_area(circles)
        assert abs(opened.sum() * h * h - An) < 6e-3 * An, (r, opened.sum() * h * h, An)
        assert abs(_constructed_length(circles, r) - L) < 1e-12 * L


def test_general_msp_reduces_to_the_equal_touching_case():
    C = [(0.0, 0.0, R), (2.0 * R, 0.0, R), (R, math.sqrt(3.0) * R, R)]
    assert est.msp_general_radius(C) == pytest.approx(est.msp_radius(R), rel=1e-12)


@pytest.mark.parametrize("circles,rs", GENERAL)
def test_general_msp_root(circles, rs):
    r = est.msp_general_radius(circles)
    An, L, ok = est.msp_general_parts(circles, r)
    assert ok and abs(An - r * L) < 1e-12


def test_opening_radius_is_the_gap_circle():
    """The closed-form opening radius (the incircle estimate's radius, a
    no-network baseline): the equal-touching case, and general triples
    against the oracle's root finder on the three tangency conditions."""
    import oracle.mlp as mlp
    equal = [(0.0, 0.0, 1.0), (2.0, 0.0, 1.0), (1.0, math.sqrt(3.0), 1.0)]
    assert est.opening_radius(equal) == pytest.approx(2.0 / math.sqrt(3.0) - 1.0, rel=1e-13)
    rng = np.random.default_rng(3)
    for _ in range(20):
        R = rng.uniform(0.8, 1.2, 3)
        ang = np.array([0.0, 2.0 * np.pi / 3, 4.0 * np.pi / 3]) + rng.uniform(-0.1, 0.1, 3)
        rad = rng.uniform(1.8, 2.4, 3) / math.sqrt(3.0)
        circles = [(rad[i] * math.cos(ang[i]), rad[i] * math.sin(ang[i]), R[i]) for i in range(3)]
        spheres = [(c[0], c[1], 0.0, c[2]) for c in circles]
        r_ref = mlp.opening_radius(spheres)
        r = est.opening_radius(circles)
        assert abs(r - r_ref) <= 1e-9 * r_ref, (circles, r, r_ref)
