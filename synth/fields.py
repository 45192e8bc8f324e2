"""Initial density fields (inputs to a run: the state at t = 0)."""
import numpy as np

from .rng import uniform_pm


def _perturb(rho, seed, amp):
    # Additive perturbation, one SplitMix64 draw per (component, node), drawn
    # in the order x fastest, then y, then z, then component.
    if seed is None or amp == 0.0:
        return rho
    return rho + uniform_pm(seed, rho.size, amp).reshape(rho.shape)


def layered_density(nx, ny, nz, z_front, rho_major, rho_minor, seed=None, amp=1e-3):
    """Non-wetting fluid in the planes z <= z_front, wetting fluid above."""
    rho = np.empty((2, nz, ny, nx))
    nw = (np.arange(nz) <= z_front)[:, None, None]
    rho[0] = np.where(nw, rho_minor, rho_major)
    rho[1] = np.where(nw, rho_major, rho_minor)
    return _perturb(rho, seed, amp)


def flat_interface_density(nx, ny, nz, split, rho_major, rho_minor, seed=None, amp=0.0):
    """Wetting fluid in x < split, non-wetting fluid in x >= split."""
    rho = np.empty((2, nz, ny, nx))
    w = (np.arange(nx) < split)[None, None, :]
    rho[0] = np.where(w, rho_major, rho_minor)
    rho[1] = np.where(w, rho_minor, rho_major)
    return _perturb(rho, seed, amp)


def droplet_density(nx, ny, nz, center, radius, rho_major, rho_minor, seed=None, amp=0.0,
                    inner=0):
    """A ball of component `inner` (0 = wetting) of the given radius in the
    other component; node (x, y, z) is inside when its squared distance to the
    centre is at most radius**2."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d2 = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2
    ball = d2 <= radius * radius
    rho = np.empty((2, nz, ny, nx))
    rho[inner] = np.where(ball, rho_major, rho_minor)
    rho[1 - inner] = np.where(ball, rho_minor, rho_major)
    return _perturb(rho, seed, amp)
