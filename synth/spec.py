"""Problem description: the statement of one subdomain run.

The fields follow the paper's statement of the problem (Sec. 2): geometry
(spheres and the throat prism), component densities, relaxation times (Eq. 1),
interaction strengths (Eq. 4-5, adhesion for perfect wetting) and the inlet /
outlet bath densities that set the capillary pressure (Sec. 2.2.2).
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

BC_PERIODIC = 0
BC_WALLS = 1
BC_RESERVOIR = 2


@dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    bc: Tuple[int, int, int] = (BC_WALLS, BC_WALLS, BC_RESERVOIR)
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))  # [n][cx,cy,cz,r]
    prism_ids: Optional[Tuple[int, int, int]] = None
    tau: Tuple[float, float] = (1.0, 1.0)           # (w, nw)
    G: float = 0.9
    G_ads: Tuple[float, float] = (-0.4, 0.4)        # (w, nw)
    rho_major: float = 2.0
    # minority density of a bulk phase: coexistence partner of rho_major = 2 at
    # tau = 1, G = 0.9 for velocity-shift forcing (root of
    # (tau - 1/2) ln(rho_major/rho_minor) = tau G (rho_major - rho_minor))
    rho_minor: float = 0.0609883
    rho_in_nw: float = 2.0
    rho_out_w: float = 2.0
    rho_init: Optional[np.ndarray] = None           # [2][nz][ny][nx] float64
    z_front: int = 2
    probe: Optional[Tuple[int, int, int]] = None

    @property
    def n_nodes(self):
        return self.nx * self.ny * self.nz

    def spheres_array(self):
        s = np.ascontiguousarray(np.asarray(self.spheres, dtype=np.float64).reshape(-1, 4))
        return s

    def rho_init_array(self):
        if self.rho_init is None:
            return None
        r = np.ascontiguousarray(np.asarray(self.rho_init, dtype=np.float64))
        if r.shape != (2, self.nz, self.ny, self.nx):
            raise ValueError("rho_init must have shape (2, nz, ny, nx)")
        return r
