"""Seeded synthetic crystals: plane-wave Hamiltonian -> band energies and orbitals.

This module only *makes inputs*.  It holds none of the screening method's
arithmetic (no Green's function, no polarizability, no quadrature, no W); both
the CPU oracle and the GPU library consume what it produces.

Model (a stand-in for the DFT wave functions the paper reads from a plane-wave
code, Sec. VI.A-B): a cubic cell of side ``a`` holding Gaussian wells
    V(r) = -sum_atoms U_a exp(-|r - R_a|^2 / (2 sigma^2)),
whose Fourier coefficients per cell volume Omega are
    V(G) = -sum_a U_a (2 pi sigma^2)^{3/2} / Omega * exp(-sigma^2 |G|^2 / 2) * exp(-i G.R_a).
At each k the dense Hamiltonian H_{GG'} = |k+G|^2/2 delta_{GG'} + V(G-G') is
diagonalised in FP64; orbitals follow the Bloch form of Eq. (bloch),
    psi_bk(r) = Omega^{-1/2} sum_G C_bk(G) exp(i (k+G).r),
normalised to one over the cell (the 1/N_k convention of the discretised g).
They are evaluated on the cell's FFT grid (inverse FFT) and at arbitrary site
points (direct phase-matrix sum).

Everything is computed with torch in float64/complex128 so that large
workloads can be synthesised directly on a GPU; small ones run on the CPU.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch


@dataclass
class Crystal:
    a: float                      # cubic lattice constant (bohr)
    frac: np.ndarray              # [natom, 3] fractional positions
    depth: np.ndarray             # [natom] well depths U_a (Ha)
    sigma: float = 1.0            # well width (bohr)

    @property
    def omega(self) -> float:
        return self.a ** 3

    @property
    def cart(self) -> np.ndarray:
        return self.frac * self.a


@dataclass
class Bands:
    """Orbitals and energies of one synthetic crystal on one k-set."""
    crystal: Crystal
    kpts: np.ndarray              # [nk, 3] Cartesian k (bohr^-1)
    energies: np.ndarray          # [nk, nb] float64 (Ha), scissor already applied
    nocc: int
    gvec: np.ndarray              # [npw, 3] integer G (units of 2 pi / a)
    coef: list                    # per k: torch complex128 [npw, nb]
    gap_raw: float                # global gap before the scissor (Ha)
    scissor: float                # shift added to every unoccupied energy (Ha)
    meta: dict = field(default_factory=dict)

    @property
    def nk(self) -> int:
        return self.energies.shape[0]

    @property
    def nb(self) -> int:
        return self.energies.shape[1]


def gvectors(a: float, gcut2: float) -> np.ndarray:
    """Integer vectors n with |2 pi n / a|^2 <= gcut2, sorted by length then lexicographically."""
    b = 2.0 * math.pi / a
    nmax = int(math.floor(math.sqrt(gcut2) / b)) + 1
    r = np.arange(-nmax, nmax + 1)
    n = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    g2 = (n * n).sum(1) * b * b
    keep = g2 <= gcut2 * (1 + 1e-12)
    n = n[keep]
    g2 = g2[keep]
    order = np.lexsort((n[:, 2], n[:, 1], n[:, 0], np.round(g2, 10)))
    return n[order]


def cutoff_for_count(a: float, target: int) -> float:
    """Smallest shell cutoff |G|^2 giving at least ``target`` plane waves (closed shells)."""
    b = 2.0 * math.pi / a
    nmax = int(math.ceil((3.0 * target / (4.0 * math.pi)) ** (1.0 / 3.0))) + 2
    r = np.arange(-nmax, nmax + 1)
    n = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    s = np.sort((n * n).sum(1))
    return float(s[target - 1]) * b * b


def kgrid(a: float, nkdiv: int) -> np.ndarray:
    """Gamma-centred nkdiv^3 Monkhorst-Pack-type grid, Cartesian (bohr^-1)."""
    b = 2.0 * math.pi / a
    f = np.arange(nkdiv) / nkdiv
    k = np.stack(np.meshgrid(f, f, f, indexing="ij"), -1).reshape(-1, 3)
    return k * b


def _hamiltonian(cr: Crystal, gvec: np.ndarray, k: np.ndarray, device) -> torch.Tensor:
    b = 2.0 * math.pi / cr.a
    G = torch.as_tensor(gvec, dtype=torch.float64, device=device) * b
    kk = torch.as_tensor(k, dtype=torch.float64, device=device)
    kin = 0.5 * ((G + kk) ** 2).sum(1)
    dG = G[:, None, :] - G[None, :, :]                          # [npw, npw, 3]
    dG2 = (dG ** 2).sum(-1)
    pref = -(2.0 * math.pi * cr.sigma ** 2) ** 1.5 / cr.omega
    H = torch.zeros(dG2.shape, dtype=torch.complex128, device=device)
    env = torch.exp(-0.5 * cr.sigma ** 2 * dG2)
    for R, U in zip(cr.cart, cr.depth):
        Rt = torch.as_tensor(R, dtype=torch.float64, device=device)
        ph = -(dG * Rt).sum(-1)
        H += (pref * float(U)) * env * torch.polar(torch.ones_like(ph), ph)
    del dG, dG2, env
    H += torch.diag(kin).to(torch.complex128)
    return H


def solve_bands(cr: Crystal, gcut2: float, kpts: np.ndarray, nb: int, nocc: int,
                gap_floor: float = 0.05, device="cpu") -> Bands:
    """Diagonalise H(k) for every k, keep the lowest ``nb`` bands.

    The lowest ``nocc`` bands at every k are occupied.  If the global gap
    min_k e_{nocc,k} - max_k e_{nocc-1,k} is below ``gap_floor`` every
    unoccupied energy is shifted up (a scissor, as the paper applies to its
    valence spectra) so that the gap equals the floor; orbitals are unchanged.
    """
    gvec = gvectors(cr.a, gcut2)
    if gvec.shape[0] < nb:
        raise ValueError(f"{gvec.shape[0]} plane waves < {nb} bands")
    energies, coefs = [], []
    for k in kpts:
        H = _hamiltonian(cr, gvec, k, device)
        w, v = torch.linalg.eigh(H)
        del H
        w = w[:nb]
        v = v[:, :nb].contiguous()
        # deterministic gauge: the largest-magnitude coefficient of each band is real positive
        idx = v.abs().argmax(0)
        ph = v[idx, torch.arange(nb, device=v.device)]
        v = v * (ph.abs() / ph)[None, :]
        energies.append(w.double().cpu().numpy())
        coefs.append(v)
    E = np.stack(energies)
    gap = float(E[:, nocc:].min() - E[:, :nocc].max())
    shift = max(0.0, gap_floor - gap)
    E[:, nocc:] += shift
    return Bands(crystal=cr, kpts=np.asarray(kpts, float), energies=E, nocc=nocc, gvec=gvec,
                 coef=coefs, gap_raw=gap, scissor=shift, meta={"npw": int(gvec.shape[0])})


def psi_on_grid(bands: Bands, ngrid: int, ik: int, band_slice=slice(None)) -> torch.Tensor:
    """psi_bk on the ngrid^3 cell grid, flattened C-order; complex128 [nb, ngrid^3]."""
    cr = bands.crystal
    C = bands.coef[ik][:, band_slice]
    dev = C.device
    nbs = C.shape[1]
    gv = bands.gvec
    if np.abs(gv).max() * 2 >= ngrid:
        raise ValueError("FFT grid too small for the plane-wave sphere")
    idx = torch.as_tensor((gv % ngrid) @ np.array([ngrid * ngrid, ngrid, 1]), device=dev)
    box = torch.zeros((nbs, ngrid ** 3), dtype=torch.complex128, device=dev)
    box[:, idx] = C.T
    u = torch.fft.ifftn(box.view(nbs, ngrid, ngrid, ngrid), dim=(1, 2, 3), norm="forward")
    # Bloch phase exp(i k.r) on the grid points r = a * j / ngrid
    f = torch.arange(ngrid, device=dev, dtype=torch.float64) * (cr.a / ngrid)
    k = torch.as_tensor(bands.kpts[ik], device=dev, dtype=torch.float64)
    ph = (k[0] * f)[:, None, None] + (k[1] * f)[None, :, None] + (k[2] * f)[None, None, :]
    u = u * torch.polar(torch.ones_like(ph), ph)[None] / math.sqrt(cr.omega)
    return u.reshape(nbs, -1)


def grid_points(a: float, ngrid: int) -> np.ndarray:
    f = np.arange(ngrid) * (a / ngrid)
    return np.stack(np.meshgrid(f, f, f, indexing="ij"), -1).reshape(-1, 3)


def psi_at_points(bands: Bands, points: np.ndarray, ik: int, chunk: int = 4096) -> torch.Tensor:
    """psi_bk at arbitrary Cartesian points by the direct phase-matrix sum; complex128 [nb, npts]."""
    cr = bands.crystal
    C = bands.coef[ik]
    dev = C.device
    b = 2.0 * math.pi / cr.a
    kG = torch.as_tensor(bands.gvec * b + bands.kpts[ik][None, :], device=dev, dtype=torch.float64)
    out = []
    for s in range(0, points.shape[0], chunk):
        p = torch.as_tensor(points[s:s + chunk], device=dev, dtype=torch.float64)
        ph = p @ kG.T                                            # [np, npw]
        P = torch.polar(torch.ones_like(ph), ph)
        out.append((P @ C).T)
    return torch.cat(out, 1) / math.sqrt(cr.omega)


def diamond_cell(a: float, rng: np.random.Generator, reps: int = 1) -> Crystal:
    base = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], float)
    base = np.concatenate([base, base + 0.25])
    frac = []
    for i in range(reps):
        for j in range(reps):
            for l in range(reps):
                frac.append((base + np.array([i, j, l])) / reps)
    frac = np.concatenate(frac)
    depth = rng.uniform(1.0, 3.0, size=frac.shape[0])
    return Crystal(a=a * reps, frac=frac, depth=depth)


def random_cell(a: float, natom: int, rng: np.random.Generator) -> Crystal:
    frac = rng.uniform(0.0, 1.0, size=(natom, 3))
    depth = rng.uniform(1.0, 3.0, size=natom)
    return Crystal(a=a, frac=frac, depth=depth)


def valence_density(psi: torch.Tensor, nocc: int, spin: int = 2) -> torch.Tensor:
    """Electron density at the points of psi [nk, nb, npts]: (spin / nk) sum_k sum_{n < nocc}
    |psi_nk|^2 (the density a plane-wave calculation hands over with its orbitals)."""
    return spin / psi.shape[0] * (psi[:, :nocc].abs() ** 2).sum((0, 1))
