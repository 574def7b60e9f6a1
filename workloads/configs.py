"""The five synthetic workloads (tiny, production, precision, batching, differentiation).

Each builder returns a :class:`Workload` holding band energies, orbitals at the
site points and (optionally) on the cell grid, the site geometry and seeded
test charges.  All randomness comes from NumPy PCG64 seeded with the workload
index (tiny = 0 ... differentiation = 4).  Shapes follow the paper's workloads
scaled to synthetic crystals: sites of radial shells x angular points, 1-8
k-points, tens to thousands of bands, 16-32 energy nodes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import crystal as cx
from . import sites as sx


@dataclass
class Workload:
    name: str
    energies: np.ndarray            # [nk, nb] float64
    nocc: int
    spin: int
    sites: list                     # [Site]
    psi_site: torch.Tensor          # complex128 [nk, nb, sum npts]
    psi_grid: torch.Tensor | None   # complex128 [nk, nb, ngrid^3] or None
    ngrid: int
    grid_dV: float
    n_terms: int                    # number of energy quadrature nodes for this workload
    bands: cx.Bands
    rho_test: np.ndarray | None = None   # [sum npts] test charges (one per site, concatenated)
    meta: dict = field(default_factory=dict)

    @property
    def nk(self):
        return self.energies.shape[0]

    @property
    def nb(self):
        return self.energies.shape[1]

    @property
    def site_offsets(self):
        o = [0]
        for s in self.sites:
            o.append(o[-1] + s.npts)
        return o

    @property
    def nrows(self):
        return self.site_offsets[-1]


def _assemble(name, bands, sites, ngrid, n_terms, with_grid, rng_charge=None, device="cpu"):
    pts = np.concatenate([s.points() for s in sites])
    psi_site = torch.stack([cx.psi_at_points(bands, pts, k) for k in range(bands.nk)])
    psi_grid = None
    if with_grid:
        psi_grid = torch.stack([cx.psi_on_grid(bands, ngrid, k) for k in range(bands.nk)])
    rho = None
    if rng_charge is not None:
        rho = np.concatenate([sx.gaussian_charge(s, rng_charge) for s in sites])
    return Workload(name=name, energies=bands.energies, nocc=bands.nocc, spin=2, sites=sites,
                    psi_site=psi_site, psi_grid=psi_grid, ngrid=ngrid,
                    grid_dV=bands.crystal.omega / ngrid ** 3, n_terms=n_terms, bands=bands,
                    rho_test=rho, meta={"npw": bands.meta["npw"], "gap_raw": bands.gap_raw,
                                        "scissor": bands.scissor})


def tiny(with_grid=True, device="cpu", seed=0, nb=128, nocc=8) -> Workload:
    """a = 10 bohr, 2 random wells, Gamma, |G|^2 <= 6 bohr^-2, 128 bands (8 occupied),
    16^3 grid, one site of 8 shells (0.1-2 bohr) x 26 angular points, 16 nodes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cr = cx.random_cell(10.0, 2, rng)
    bands = cx.solve_bands(cr, 6.0, np.zeros((1, 3)), nb, nocc, device=device)
    site = sx.make_site(cr.cart[0], 8, 26, r_max=2.0, r_min=0.1)
    return _assemble("tiny", bands, [site], 16, 16, with_grid, rng, device)


def production(with_grid=True, device="cpu", seed=1, nsites=2) -> Workload:
    """8-atom diamond-type cell a = 10.2 bohr, 2x2x2 k, |G|^2 <= 23.2 bohr^-2 (~2000 PWs),
    64 occupied + 512 unoccupied bands, 24^3 grid, sites of 16 shells x 50 points, 24 nodes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cr = cx.diamond_cell(10.2, rng)
    bands = cx.solve_bands(cr, 23.2, cx.kgrid(cr.a, 2), 576, 64, device=device)
    sites = [sx.make_site(cr.cart[i], 16, 50) for i in range(nsites)]
    return _assemble("production", bands, sites, 24, 24, with_grid, rng, device)


def differentiation(with_grid=False, device="cpu", seed=4) -> Workload:
    """The production cell with 4 sites and seeded Gaussian test charges (width 0.5 bohr)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cr = cx.diamond_cell(10.2, rng)
    bands = cx.solve_bands(cr, 23.2, cx.kgrid(cr.a, 2), 576, 64, device=device)
    sites = [sx.make_site(cr.cart[i], 16, 50) for i in range(4)]
    return _assemble("differentiation", bands, sites, 24, 24, with_grid, rng, device)


def _supercell(seed, gamma_only, device, nb=2304, nocc=256):
    rng = np.random.Generator(np.random.PCG64(seed))
    cr = cx.diamond_cell(10.2, rng, reps=2)                        # 64 wells, a = 20.4
    gcut2 = cx.cutoff_for_count(cr.a, int(math.ceil(1.25 * nb)))
    kpts = np.zeros((1, 3)) if gamma_only else cx.kgrid(cr.a, 2)
    bands = cx.solve_bands(cr, gcut2, kpts, nb, nocc, device=device)
    return rng, cr, bands


def precision(with_grid=True, device="cpu", gamma_only=False, seed=2) -> Workload:
    """64-well supercell a = 20.4 bohr, Gamma or 2x2x2 k, 256 + 2048 bands, 48^3 grid,
    one site of 32 shells x 110 points, 32 nodes."""
    rng, cr, bands = _supercell(seed, gamma_only, device)
    site = sx.make_site(cr.cart[0], 32, 110)
    return _assemble("precision", bands, [site], 48, 32, with_grid, rng, device)


def batching(with_grid=True, device="cpu", seed=3, nsites=64) -> Workload:
    """The supercell with 64 sites of uneven grids: shells uniform in 8..32, angular
    points from {26, 50, 86, 110}; 2x2x2 k."""
    rng, cr, bands = _supercell(seed, False, device)
    nrad = rng.integers(8, 33, size=nsites)
    nang = rng.choice([26, 50, 86, 110], size=nsites)
    sites = [sx.make_site(cr.cart[i], int(nrad[i]), int(nang[i])) for i in range(nsites)]
    return _assemble("batching", bands, sites, 48, 28, with_grid, rng, device)


def free_electron(a=10.0, gcut2=6.0, nocc=7, nb=123, ngrid=16, n_rad=4, n_ang=26):
    """Plane waves at Gamma (no potential) with closed shells on both sides of the gap:
    orbitals e^{iG.r}/sqrt(Omega), energies |G|^2/2, no eigensolver involved."""
    gv = cx.gvectors(a, gcut2)[:nb]
    b = 2 * math.pi / a
    G = gv * b
    E = 0.5 * (G ** 2).sum(1)
    site = sx.make_site(np.array([0.3, -0.2, 0.1]) * a, n_rad, n_ang, r_max=2.0)
    pts = site.points()
    omega = a ** 3
    psi_site = np.exp(1j * pts @ G.T).T / math.sqrt(omega)
    gp = cx.grid_points(a, ngrid)
    psi_grid = np.exp(1j * gp @ G.T).T / math.sqrt(omega)
    return dict(G=G, E=E[None, :], nocc=nocc, site=site, pts=pts, omega=omega,
                psi_site=psi_site[None], psi_grid=psi_grid[None], grid_pts=gp,
                dV=omega / ngrid ** 3)


BUILDERS = {"tiny": tiny, "production": production, "precision": precision,
            "batching": batching, "differentiation": differentiation}
