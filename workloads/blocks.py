"""Seeded stand-ins for site x site chi0 blocks, the input of the per-site solve stages (W,
the ALDA W, the induced potential) when those are tested on their own.

A block is  -(s / m) sum_j f_j f_j^T  over m Gaussian blobs
    f_j(p) = exp(-|p - c_j|^2 / (2 sigma_j^2)),
with centres c_j uniform in a cube of half-width 3 bohr around the site centre and widths
sigma_j uniform in [0.7, 1.5] bohr, evaluated at the site's points.  Such a block is
symmetric, negative semidefinite and smooth over the site, as a static chi0 block is; the
default strength gives dielectric eigenvalues up to a few units on the site grids used here.
Library and oracle both take these blocks as given inputs.
"""
from __future__ import annotations

import numpy as np


def chi0_like_block(site, rng: np.random.Generator, m: int = 48,
                    strength: float = 0.05) -> np.ndarray:
    """[npts, npts] float64 block for one site (points in the site's radial-major order)."""
    p = site.points() - site.centre[None, :]
    c = rng.uniform(-3.0, 3.0, size=(m, 3))
    sig = rng.uniform(0.7, 1.5, size=m)
    f = np.exp(-((p[:, None, :] - c[None, :, :]) ** 2).sum(-1) / (2.0 * sig ** 2))
    blk = -(f @ f.T) * (strength / m)
    return 0.5 * (blk + blk.T)


def chi0_like_blocks(sites, seed: int, m: int = 48, strength: float = 0.05):
    """One block per site, from one seeded stream; returns (list of blocks, flat
    concatenation in site order)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    blocks = [chi0_like_block(s, rng, m, strength) for s in sites]
    return blocks, np.concatenate([b.ravel() for b in blocks])
