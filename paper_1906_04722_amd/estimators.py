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


def pc_star(pc, R, gamma):
    """The paper's normalised capillary pressure p_c* = 2 p_c R / gamma."""
    return 2.0 * pc * R / gamma


def v_star(volume, R):
    """The paper's normalised volume V* = V / (4/3 pi R^3)."""
    return volume / (4.0 / 3.0 * math.pi * R ** 3)
