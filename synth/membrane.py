"""Fully resolved drainage sample of a periodic packing between two baths,
with a porous membrane in front of the wetting outlet (Sec. 3: the full-LBM
drainage against which the hybrid method is validated).

Input generation only: a sphere list and the lattice layout.  The packing's
periodic cell (side L) is resolved at `res` nodes per packing length; x and y
stay periodic, as in the pore network of the same packing (synth.network).
Along z the lattice holds, from the non-wetting bath at z = 0:

  * a buffer of `margin` planes filled with the non-wetting phase, then the
    planes that the slab's spheres reach into,
  * the packing slab: packing height L maps to the slab's first plane, height
    0 to the plane just past its last, so the network's inlet face (z = L)
    meets the non-wetting side,
  * the membrane plane on the slab's outlet face (packing height 0), where the
    pore network's outlet reservoir begins,
  * the planes that the slab's spheres reach into past the membrane, then
    `outlet` open planes and the wetting bath at z = nz - 1.

The slab is cut from the periodic packing: every sphere image (shifts of L
along x, y and z) that meets 0 <= z <= L is kept whole, so its caps reach
past the two faces: into the inlet buffer, which is sized to stay open
beyond them, and behind the membrane, where they lie in the wetting layer.
The membrane is one plane of radius-1 spheres centred on the nodes with even
x and y: it leaves single-node holes at odd (x, y), which pass the wetting
phase and hold the non-wetting one far above the entry pressures of the
packing's throats.
"""
import math

import numpy as np

from .spec import BC_PERIODIC, BC_RESERVOIR, Problem


def membrane_sample(x, r, L, res=12.0, margin=3, outlet=3):
    """Problem and layout of the drainage sample (see the module docstring).

    Returns (problem, info) with info = dict(scale: lattice units per packing
    length, slab: (z_first, z_last) lattice planes of the packing slab,
    membrane_z: lattice plane of the membrane, n_spheres: sphere images that
    meet the slab (before the x/y images), n_membrane: membrane spheres,
    L: the cell side)."""
    x = np.asarray(x, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    n = int(round(L * res))
    n += n & 1                              # even: the membrane pattern has period 2
    s = n / L
    reach = int(math.ceil(2.0 * float(r.max()) * s))  # a kept image spans up to 2r past a face
    z_first = 1 + reach + margin            # first slab plane
    slab_planes = int(math.ceil(L * s))
    z_last = z_first + slab_planes - 1
    membrane_z = z_last + 1
    nz = membrane_z + reach + outlet + 2
    pts, rad = [], []
    n_slab = 0
    for sz in (-1, 0, 1):
        meets = (x[:, 2] + L * sz + r > 0.0) & (x[:, 2] + L * sz - r < L)
        n_slab += int(meets.sum())
        for sx in (-1, 0, 1):
            for sy in (-1, 0, 1):
                c = x[meets] + L * np.array([sx, sy, sz])
                X, Y = c[:, 0] * s, c[:, 1] * s
                Z = z_first + (L - c[:, 2]) * s
                R = r[meets] * s
                keep = (X + R > -1.0) & (X - R < n + 1.0) & (Y + R > -1.0) & (Y - R < n + 1.0)
                pts.append(np.column_stack([X[keep], Y[keep], Z[keep]]))
                rad.append(R[keep])
    C = np.concatenate(pts)
    R = np.concatenate(rad)
    g = np.arange(0, n, 2, dtype=np.float64)
    MX, MY = np.meshgrid(g, g, indexing="xy")
    M = np.column_stack([MX.ravel(), MY.ravel(), np.full(MX.size, float(membrane_z)),
                         np.ones(MX.size)])
    sph = np.vstack([np.column_stack([C, R]), M])
    p = Problem(nx=n, ny=n, nz=nz, bc=(BC_PERIODIC, BC_PERIODIC, BC_RESERVOIR), spheres=sph,
                prism_ids=None, rho_in_nw=2.0, rho_out_w=2.0, z_front=margin,
                probe=None)
    info = dict(scale=s, slab=(z_first, z_last), membrane_z=membrane_z,
                n_spheres=n_slab, n_membrane=int(M.shape[0]), L=float(L))
    return p, info



def lattice_points(xyz, info):
    """Lattice coordinates (float) of packing points xyz [m][3] in the sample
    built by membrane_sample: x and y wrapped into the periodic cell and
    scaled, z flipped onto the slab."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    L, s = info["L"], info["scale"]
    X = np.mod(xyz[:, 0], L) * s
    Y = np.mod(xyz[:, 1], L) * s
    Z = info["slab"][0] + (L - xyz[:, 2]) * s
    return np.column_stack([X, Y, Z])
