"""Orbitals at arbitrary points from plane-wave coefficients (oracle; test infrastructure).

Sec. VI, "Projecting the wave functions": a Bloch state stored as plane-wave coefficients,
Eq. (bloch),

    psi_bk(r) = e^{i k.r} u_bk(r) = sum_G C_bk(G) e^{i (k+G).r},

is evaluated at the site points by the direct method: the phase matrix
P_k(r, G) = e^{i (k+G).r}, common to every band at one k, times the coefficients,
psi_k(r, b) = sum_G P_k(r, G) C_k(G, b).  Here the coefficients are normalised to one
over the cell, so the orbitals carry the factor Omega^{-1/2} (unit norm over the cell).

Plain NumPy in complex128; one matrix product per k.  Parity: pinned in
``tests/test_oracle_pins.py`` against the inverse FFT of the same coefficients at the cell's
grid points, Bloch's theorem under a lattice translation, Parseval's identity on the grid,
and explicit loops on a tiny case.
"""
from __future__ import annotations

import numpy as np


def phase_matrix(k, gvec, points):
    """P_k(r, G) = exp(i (k+G).r): complex128 [npts, npw].  k [3], gvec [npw, 3] (Cartesian,
    bohr^-1), points [npts, 3] (Cartesian, bohr)."""
    kg = np.asarray(gvec, dtype=np.float64) + np.asarray(k, dtype=np.float64)[None, :]
    return np.exp(1j * (np.asarray(points, dtype=np.float64) @ kg.T))


def project(coef, kpts, gvec, points, omega):
    """psi [nk, nb, npts] from coef [nk, nb, npw] (C_bk(G)), kpts [nk, 3], gvec [npw, 3],
    points [npts, 3], cell volume omega."""
    coef = np.asarray(coef, dtype=np.complex128)
    out = np.empty((coef.shape[0], coef.shape[1], len(points)), dtype=np.complex128)
    for ik in range(coef.shape[0]):
        out[ik] = coef[ik] @ phase_matrix(kpts[ik], gvec, points).T
    return out / np.sqrt(omega)
