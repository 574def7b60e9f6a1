"""Site grids (radial shells x angular points) and seeded test charges.

The paper builds each site's real-space basis as a product of a radial grid and
an angular grid (Appendix D.1.a).  Here the angular sets are Lebedev rules
(26/50/86/110 points) from SciPy and the radial grids are uniform; both are
*inputs* to the library, which never generates them itself.

Point ordering inside a site is radial-major: p = i * n_ang + a, at
position centre + r_i * Omega_a.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.integrate import lebedev_rule

_LEBEDEV_DEGREE = {6: 3, 14: 5, 26: 7, 38: 9, 50: 11, 74: 13, 86: 15, 110: 17, 146: 19, 170: 21}


def angular_rule(npts: int):
    """Unit vectors [npts, 3] and weights [npts] (sum 4 pi)."""
    if npts not in _LEBEDEV_DEGREE:
        raise ValueError(f"no Lebedev rule with {npts} points")
    x, w = lebedev_rule(_LEBEDEV_DEGREE[npts])
    x = np.ascontiguousarray(x.T)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x, np.asarray(w, float)


@dataclass
class Site:
    centre: np.ndarray        # [3] Cartesian (bohr)
    radii: np.ndarray         # [n_rad]
    rad_w: np.ndarray         # [n_rad] radial weights u_i ~ r_i^2 dr
    ang_xyz: np.ndarray       # [n_ang, 3]
    ang_w: np.ndarray         # [n_ang]

    @property
    def n_rad(self) -> int:
        return self.radii.shape[0]

    @property
    def n_ang(self) -> int:
        return self.ang_w.shape[0]

    @property
    def npts(self) -> int:
        return self.n_rad * self.n_ang

    def points(self) -> np.ndarray:
        p = self.radii[:, None, None] * self.ang_xyz[None, :, :]
        return (p + self.centre[None, None, :]).reshape(-1, 3)


def uniform_radial(r0: float, r1: float, n: int):
    r = np.linspace(r0, r1, n)
    dr = (r1 - r0) / (n - 1) if n > 1 else r1
    return r, r * r * dr


def make_site(centre, n_rad: int, n_ang: int, r_max: float = 4.0, r_min=None) -> Site:
    r0 = r_max / n_rad if r_min is None else r_min
    r, u = uniform_radial(r0, r_max, n_rad)
    x, w = angular_rule(n_ang)
    return Site(centre=np.asarray(centre, float), radii=r, rad_w=u, ang_xyz=x, ang_w=w)


def gaussian_charge(site: Site, rng: np.random.Generator, sigma: float = 0.5,
                    max_offset: float = 0.5) -> np.ndarray:
    """Unit Gaussian test charge (width sigma) centred within max_offset of the site centre,
    sampled at the site's points; float64 [npts]."""
    while True:
        d = rng.uniform(-max_offset, max_offset, size=3)
        if np.dot(d, d) <= max_offset ** 2:
            break
    c = site.centre + d
    p = site.points()
    r2 = ((p - c[None, :]) ** 2).sum(1)
    return (2 * np.pi * sigma ** 2) ** -1.5 * np.exp(-r2 / (2 * sigma ** 2))
