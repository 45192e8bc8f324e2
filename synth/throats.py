"""Pore-throat geometries: a tetrahedron of four spheres whose lower face is
the throat (three spheres whose centres span the prism cross-section) and
whose apex sphere closes the pore body above it (Sec. 2.2.1: each tetrahedron
of the regular triangulation is a pore body, each facet a throat)."""
import math

import numpy as np

from .fields import layered_density
from .rng import uniform01
from .spec import BC_PERIODIC, BC_RESERVOIR, BC_WALLS, Problem


def tetra_throat(centroid, edge, radii, jitter=None):
    """Spheres at the vertices of a regular tetrahedron with one face normal
    to z, below the centroid (the throat, facing the inlet at z = 0), and
    the apex above.  Face vertices sit at azimuths 90, 210 and 330 degrees.
    Returns an array [4][cx, cy, cz, r]; rows 0-2 are the throat spheres."""
    cx, cy, cz = centroid
    h = edge * math.sqrt(2.0 / 3.0)          # height of the tetrahedron
    rc = edge / math.sqrt(3.0)               # circumradius of a face
    zf = cz - h / 4.0                        # the centroid is h/4 above a face
    sph = np.zeros((4, 4))
    for i, az in enumerate((90.0, 210.0, 330.0)):
        a = math.radians(az)
        sph[i, :3] = (cx + rc * math.cos(a), cy + rc * math.sin(a), zf)
    sph[3, :3] = (cx, cy, cz + 0.75 * h)
    sph[:, 3] = radii
    if jitter is not None:
        sph[:, :3] += jitter
    return sph


def _probe_near(p):
    return tuple(int(math.floor(v + 0.5)) for v in p)


def c1_problem(seed=1, amp=1e-3, rho_in=2.05):
    """40^3 throat: four spheres of radius 14 on a regular tetrahedron of edge
    30 centred in the box, prism closure over the three lower spheres, baths at
    z = 0 (non-wetting) and z = 39 (wetting), tau = 1, G = 0.9, adhesion
    -0.4 / +0.4, majority density 2.0, +-1e-3 uniform density perturbation."""
    n = 40
    c = ((n - 1) / 2.0,) * 3
    sph = tetra_throat(c, 30.0, 14.0)
    p = Problem(nx=n, ny=n, nz=n, bc=(BC_WALLS, BC_WALLS, BC_RESERVOIR), spheres=sph,
                prism_ids=(0, 1, 2), rho_in_nw=rho_in, rho_out_w=2.0, z_front=2,
                probe=_probe_near(c))
    p.rho_init = layered_density(n, n, n, p.z_front, p.rho_major, p.rho_minor, seed, amp)
    return p


def _normals(seed, n):
    # Box-Muller transform of SplitMix64 uniforms (pairs of draws)
    u = uniform01(seed, 2 * n)
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def c2_problem(seed=2, n=96, mean_r=32.0, sigma=0.15, amp=1e-3):
    """n^3 throat: four spheres with lognormal radii (arithmetic mean mean_r,
    log-sd sigma) on the 40^3 layout scaled by mean_r/14 (edge 30*mean_r/14),
    each centre jittered by U[-2, 2) lu per axis."""
    c = ((n - 1) / 2.0,) * 3
    z = _normals(seed, 4)
    radii = np.exp(math.log(mean_r) - 0.5 * sigma * sigma + sigma * z)
    jit = 4.0 * uniform01(seed + 1000, 12).reshape(4, 3) - 2.0
    sph = tetra_throat(c, 30.0 * mean_r / 14.0, radii, jitter=jit)
    cen = sph[:, :3].mean(axis=0)
    p = Problem(nx=n, ny=n, nz=n, bc=(BC_WALLS, BC_WALLS, BC_RESERVOIR), spheres=sph,
                prism_ids=(0, 1, 2), rho_in_nw=2.0, rho_out_w=2.0, z_front=2,
                probe=_probe_near(cen))
    p.rho_init = layered_density(n, n, n, p.z_front, p.rho_major, p.rho_minor, seed, amp)
    return p


def small_throat_problem(n=24, seed=7, amp=1e-3, rho_in=2.05, gap=2.0):
    """The 40^3 layout scaled to an n^3 box (sphere radius 14 n/40, edge set so
    that neighbouring spheres leave `gap` lattice units between them)."""
    c = ((n - 1) / 2.0,) * 3
    r = 14.0 * n / 40.0
    sph = tetra_throat(c, 2.0 * r + gap, r)
    p = Problem(nx=n, ny=n, nz=n, bc=(BC_WALLS, BC_WALLS, BC_RESERVOIR), spheres=sph,
                prism_ids=(0, 1, 2), rho_in_nw=rho_in, rho_out_w=2.0, z_front=2,
                probe=_probe_near(c))
    p.rho_init = layered_density(n, n, n, p.z_front, p.rho_major, p.rho_minor, seed, amp)
    return p



def three_sphere_throat(R=32.0, margin=6, seed=3, amp=1e-3, rho_in=2.0):
    """The paper's example throat (Sec. 2.2.2): three equal spheres of radius
    R (lattice units) in mutual contact, centres on one plane normal to z, the
    prism over their triangle as the closure, and no fourth sphere.  The
    non-wetting bath is at z = 0 and the wetting one at z = nz - 1, `margin`
    open planes beyond the spheres on each side.  The invasion probe sits on
    the prism axis 3 lu past the plane of the centres."""
    x0 = y0 = 1.0
    h = math.sqrt(3.0) * R
    nx = int(math.ceil(x0 + 2.0 * R)) + 2
    ny = int(math.ceil(y0 + h)) + 2
    zt = margin + int(math.ceil(R)) + 1
    nz = zt + int(math.ceil(R)) + margin + 2
    sph = np.array([[x0, y0, zt, R], [x0 + 2.0 * R, y0, zt, R], [x0 + R, y0 + h, zt, R]])
    axis = (x0 + R, y0 + h / 3.0)
    p = Problem(nx=nx, ny=ny, nz=nz, bc=(BC_WALLS, BC_WALLS, BC_RESERVOIR), spheres=sph,
                prism_ids=(0, 1, 2), rho_in_nw=rho_in, rho_out_w=2.0, z_front=margin,
                probe=_probe_near((axis[0], axis[1], zt + 3)))
    p.rho_init = layered_density(nx, ny, nz, p.z_front, p.rho_major, p.rho_minor, seed, amp)
    return p


def constriction_problem(nx=20, ny=3, nz=36, gap=6.0, zc=14, seed=5, amp=1e-3):
    """A quasi-two-dimensional throat: a slab periodic in x and y (ny nodes
    thick) holding a periodic row of spheres centred on its mid-plane at
    z = zc, one per period nx, of radius (nx - gap)/2, so that a slit `gap`
    lattice units wide (half-way walls) opens between neighbours.  Below and
    above the row the slab is open from side to side, so no solid touches
    either bath.  The non-wetting phase fills z <= 3 next to the inlet bath;
    the probe sits on the slit's axis 5 nodes past its narrowest section, in
    the open region beyond it.  Small enough for the oracle to drain in
    seconds, with a genuine entry pressure near the two-dimensional Laplace
    value 2 gamma / gap of a perfectly wetting slit."""
    R = (nx - gap) / 2.0
    yc = (ny - 1) / 2.0
    xc = -0.5  # the slit is centred on x = (nx - 1) / 2
    # the sphere and its periodic image, so that every node of the slab sees
    # the solid it is nearest to
    sph = np.array([[xc, yc, zc, R], [xc + nx, yc, zc, R]])
    p = Problem(nx=nx, ny=ny, nz=nz, bc=(BC_PERIODIC, BC_PERIODIC, BC_RESERVOIR), spheres=sph,
                rho_in_nw=2.0, rho_out_w=2.0, z_front=3,
                probe=(int(round((nx - 1) / 2.0)), int(round(yc)), zc + 5))
    p.rho_init = layered_density(nx, ny, nz, p.z_front, p.rho_major, p.rho_minor, seed, amp)
    return p


def throat_incircle(spheres, ids=(0, 1, 2)):
    """Radius and centre of the circle in the xy-plane tangent to the three
    throat circles (sphere cross-sections through their centres): the
    inscribed opening used by the incircle estimate of the entry pressure."""
    from scipy.optimize import fsolve
    c = np.asarray(spheres, dtype=np.float64)[list(ids)]
    P = c[:, :2]
    R = c[:, 3]

    def eqs(v):
        return [np.hypot(v[0] - P[i, 0], v[1] - P[i, 1]) - (v[2] + R[i]) for i in range(3)]

    cen = P.mean(axis=0)
    r0 = np.mean(np.hypot(*(P - cen).T)) - R.mean()
    sol = fsolve(eqs, [cen[0], cen[1], max(r0, 0.5)], full_output=True)
    v = sol[0]
    return float(v[2]), (float(v[0]), float(v[1]))


# interfacial tension of the model at G = 0.9, tau = 1, majority density 2
# (lattice units), from the Laplace-law fit of static cylinders pinned in the
# oracle tests; it only sets the scale of the capillary-pressure ramps
GAMMA_LAPLACE = 0.190


def pc_ramp(gamma, r_ins, n, lo=0.1, hi=1.5):
    """n equally spaced capillary pressures from lo to hi times the incircle
    estimate 2 gamma / r_ins of a perfectly wetting throat."""
    p_hat = 2.0 * gamma / r_ins
    return np.linspace(lo, hi, n) * p_hat
