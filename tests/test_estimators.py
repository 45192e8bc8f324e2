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
