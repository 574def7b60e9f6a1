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


# --------------------------------------------------------------------------------------------
# The FFT route of the same section: u_bk on the FFT grid x (the Fourier dual of G, optionally
# oversampled), cubic Lagrange interpolation from the grid to the points, then the Bloch phase:
#     u_bk(x_j) = sum_G C_bk(G) exp(i G.x_j),   u_bk(r) = Interp[u_bk(x)],
#     psi_bk(r) = exp(i k.r) u_bk(r) / sqrt(Omega).
# With lattice vectors a_d (rows of `cell`) and Miller indices m (G = sum_d m_d b_d), the grid
# points are x_j = sum_d (j_d / N_d) a_d and G.x_j = 2 pi sum_d m_d j_d / N_d, so u on the grid
# is the unnormalised inverse DFT of C placed at m mod N.

def fft_grid(coef_b, gidx, nfft):
    """u on the [N0, N1, N2] grid from one band's coefficients coef_b [npw] at Miller indices
    gidx [npw, 3] (numpy.fft, unnormalised inverse)."""
    box = np.zeros(tuple(nfft), dtype=np.complex128)
    g = np.asarray(gidx) % np.asarray(nfft)[None, :]
    box[g[:, 0], g[:, 1], g[:, 2]] = coef_b
    return np.fft.ifftn(box) * float(np.prod(nfft))


def lagrange_cubic(t):
    """Weights of the nodes at offsets -1, 0, 1, 2 for a point at offset t from node 0."""
    nodes = (-1.0, 0.0, 1.0, 2.0)
    w = []
    for a in range(4):
        v = 1.0
        for b in range(4):
            if b != a:
                v *= (t - nodes[b]) / (nodes[a] - nodes[b])
        w.append(v)
    return np.array(w)


def stencils(cell, points, nfft):
    """Per point: the first of the four grid nodes in each dimension (floor of the grid
    coordinate minus one) and the weights [3, 4] (cached once per point set)."""
    A = np.asarray(cell, dtype=np.float64)
    frac = np.linalg.solve(A.T, np.asarray(points, dtype=np.float64).T).T   # r = frac @ A
    g = frac * np.asarray(nfft)[None, :]
    i0 = np.floor(g).astype(np.int64)
    t = g - i0
    w = np.stack([[lagrange_cubic(t[p, d]) for d in range(3)] for p in range(len(points))])
    return i0 - 1, w


def project_fft(coef, kpts, cell, gidx, points, omega, nfft):
    """psi [nk, nb, npts] by the FFT route (see above)."""
    coef = np.asarray(coef, dtype=np.complex128)
    nk, nb = coef.shape[:2]
    base, w = stencils(cell, points, nfft)
    N = np.asarray(nfft)
    out = np.empty((nk, nb, len(points)), dtype=np.complex128)
    for ik in range(nk):
        ph = np.exp(1j * (np.asarray(points) @ np.asarray(kpts[ik])))
        for b in range(nb):
            u = fft_grid(coef[ik, b], gidx, nfft)
            for p in range(len(points)):
                acc = 0.0 + 0.0j
                for a in range(4):
                    for c in range(4):
                        for e in range(4):
                            j = (base[p] + np.array([a, c, e])) % N
                            acc += w[p, 0, a] * w[p, 1, c] * w[p, 2, e] * u[j[0], j[1], j[2]]
                out[ik, b, p] = ph[p] * acc
    return out / np.sqrt(omega)


def interpolation_bound(coef, gidx, nfft, omega, samples=256):
    """Bound on |psi_fft(r) - psi_direct(r)| at any point, for each band of coef [..., npw]: with
    delta(theta) = max_t |sum_a w_a(t) e^{i theta (n_a - t)} - 1| the cubic interpolant's error on
    one plane wave of phase step theta per grid spacing, a plane wave G with steps
    theta_d = 2 pi m_d / N_d is reproduced within prod_d (1 + delta(theta_d)) - 1 (tensor
    product), so the error is at most Omega^-1/2 sum_G |C(G)| (prod_d (1 + delta_d) - 1)."""
    t = (np.arange(samples) + 0.5) / samples
    W = np.stack([lagrange_cubic(x) for x in t])                  # [samples, 4]
    nodes = np.array([-1.0, 0.0, 1.0, 2.0])

    def delta(theta):
        ph = np.exp(1j * theta * (nodes[None, :] - t[:, None]))
        return float(np.abs((W * ph).sum(1) - 1.0).max())
    m = np.asarray(gidx)
    f = np.ones(len(m))
    for d in range(3):
        cache = {int(v): delta(2 * np.pi * v / nfft[d]) for v in np.unique(m[:, d])}
        f *= 1.0 + np.array([cache[int(v)] for v in m[:, d]])
    return (np.abs(np.asarray(coef)) @ (f - 1.0)) / np.sqrt(omega)
