"""Spherical-basis projection and the per-site dielectric solve (oracle; test infrastructure).

Sec. VI.E: chi0 between the points of one site is expanded in real spherical
harmonics Y_L (L = (l, m), l <= lmax), the Coulomb operator is diagonal in L,
    v_L(r, r') = 4 pi / (2l + 1) * r_<^l / r_>^(l+1),
and the screened interaction follows from W = eps^-1 v with eps = 1 - v chi0
(equivalently W = v + v chi v with chi = (1 - chi0 v)^-1 chi0, Eqs. reducible
and W).  Radial integrals become sums with weights u_i ~ r_i^2 dr, angular
ones sums with weights w_a (sum 4 pi).

Discretised (basis index (L, i), L-major: idx = L * n_rad + i):
    X_{(L,i),(L',j)} = sum_{a,b} w_a Y_L(a) chi0(r_i a, r_j b) Y_L'(b) w_b
    V_{(L,i),(L',j)} = delta_LL' 4 pi / (2l+1) min(r_i,r_j)^l / max(r_i,r_j)^(l+1)
    D = diag(u_i)
    W = solve(I - V D X D, V)
Test-charge loss: rho_L(r_i) = sum_a w_a Y_L(a) rho(r_i a); L = rho_L^T D W D rho_L.
Induced density and potential of a spherical perturbation (the short-range part of a
potential partitioned by a shell of charge, Eq. partition):
    rho = (I - X D V D)^-1 X D v1,   v_ind = V D rho,   v1 in the L = 00 channel.

Real spherical harmonics, orthonormal on the unit sphere, in the order
L = l^2 + l + m:
    Y_00 = 1/(2 sqrt(pi))
    Y_1,-1 = c1 y, Y_10 = c1 z, Y_11 = c1 x,                       c1 = sqrt(3/(4 pi))
    Y_2,-2 = c2 x y, Y_2,-1 = c2 y z, Y_20 = c20 (3 z^2 - 1),
    Y_21 = c2 x z, Y_22 = c2/2 (x^2 - y^2),                         c2 = sqrt(15/(4 pi)),
                                                                    c20 = sqrt(5/(16 pi))
"""
from __future__ import annotations

import math

import numpy as np


def real_ylm(xyz: np.ndarray, lmax: int = 2) -> np.ndarray:
    """[(lmax+1)^2, npts] real spherical harmonics at unit vectors xyz [npts, 3]."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    out = [np.full_like(x, 0.5 / math.sqrt(math.pi))]
    if lmax >= 1:
        c1 = math.sqrt(3.0 / (4.0 * math.pi))
        out += [c1 * y, c1 * z, c1 * x]
    if lmax >= 2:
        c2 = math.sqrt(15.0 / (4.0 * math.pi))
        c20 = math.sqrt(5.0 / (16.0 * math.pi))
        out += [c2 * x * y, c2 * y * z, c20 * (3 * z * z - 1), c2 * x * z, 0.5 * c2 * (x * x - y * y)]
    if lmax > 2:
        raise ValueError("lmax <= 2")
    return np.stack(out)


def projector(site, lmax=2) -> np.ndarray:
    """P [(nL * n_rad), (n_rad * n_ang)] with P_{(L,i),(i',a)} = delta_ii' w_a Y_L(a)."""
    Y = real_ylm(site.ang_xyz, lmax) * site.ang_w[None, :]        # [nL, n_ang]
    nL, nang = Y.shape
    nr = site.n_rad
    P = np.zeros((nL, nr, nr, nang))
    for i in range(nr):
        P[:, i, i, :] = Y
    return P.reshape(nL * nr, nr * nang)


def coulomb(site, lmax=2) -> np.ndarray:
    r = site.radii
    rl = np.minimum(r[:, None], r[None, :])
    rg = np.maximum(r[:, None], r[None, :])
    nr = r.shape[0]
    nL = (lmax + 1) ** 2
    V = np.zeros((nL, nr, nL, nr))
    for l in range(lmax + 1):
        blk = 4.0 * math.pi / (2 * l + 1) * rl ** l / rg ** (l + 1)
        for m in range(-l, l + 1):
            L = l * l + l + m
            V[L, :, L, :] = blk
    return V.reshape(nL * nr, nL * nr)


def radial_weights(site, lmax=2) -> np.ndarray:
    return np.tile(site.rad_w, (lmax + 1) ** 2)


def project(chi0_ss, site, lmax=2):
    P = projector(site, lmax)
    return P @ chi0_ss @ P.T


def screen_W(chi0_ss, site, lmax=2):
    """W [n, n] for one site from its site x site chi0 block."""
    X = project(chi0_ss, site, lmax)
    V = coulomb(site, lmax)
    d = radial_weights(site, lmax)
    eps = np.eye(V.shape[0]) - V @ (d[:, None] * X * d[None, :])
    return np.linalg.solve(eps, V)


def screen_W_via_chi(chi0_ss, site, lmax=2):
    """The same W through the reducible chi of Eq. reducible: chi = (I - X D V D)^-1 X,
    W = V + V D chi D V (Eq. W)."""
    X = project(chi0_ss, site, lmax)
    V = coulomb(site, lmax)
    D = np.diag(radial_weights(site, lmax))
    chi = np.linalg.solve(np.eye(V.shape[0]) - X @ D @ V @ D, X)
    return V + V @ D @ chi @ D @ V


def charge_moments(rho, site, lmax=2):
    return projector(site, lmax) @ rho


def test_charge_loss(W, rho, site, lmax=2) -> float:
    rl = charge_moments(rho, site, lmax) * radial_weights(site, lmax)
    return float(rl @ W @ rl)


def shell_potential(radii, q, r_shell):
    """The short-range part v1 = v_ext - v2 of the partition by a shell of charge
    (Eq. partition), for v_ext = q / x centred on the site: q (1/r - 1/R_S) inside the shell
    and zero outside."""
    r = np.asarray(radii, dtype=np.float64)
    return np.where(r < r_shell, q * (1.0 / r - 1.0 / r_shell), 0.0)


def induced(chi0_ss, site, v1, lmax=2, l0_only=False):
    """Induced density and potential of a spherical perturbation v1(r_i) (Sec. VI,
    construction of chi and W):
        chi = S^-1 chi0 with S = 1 - chi0 v          (discretised chi = (I - X D V D)^-1 X)
        rho_L(r_i) = sum_j chi_{(L,i),(00,j)} u_j v1_00(r_j),   v1_00 = sqrt(4 pi) v1
        v_L(r_i)   = sum_j V_L(r_i, r_j) u_j rho_L(r_j)
    (v1_00 is the Y_00 coefficient of the spherical v1).  l0_only: the paper's default,
    chi restricted to its 00;00 block.  Returns rho, v as [(L,i)] vectors, L-major (zero
    outside L = 00 when l0_only)."""
    X = project(chi0_ss, site, lmax)
    V = coulomb(site, lmax)
    d = radial_weights(site, lmax)
    nr = site.n_rad
    n = X.shape[0]
    m = nr if l0_only else n
    X, V, d = X[:m, :m], V[:m, :m], d[:m]
    D = np.diag(d)
    chi = np.linalg.solve(np.eye(m) - X @ D @ V @ D, X)
    v1vec = np.zeros(m)
    v1vec[:nr] = math.sqrt(4.0 * math.pi) * np.asarray(v1, dtype=np.float64)
    rho = chi @ D @ v1vec
    vind = V @ D @ rho
    rho_out, v_out = np.zeros(n), np.zeros(n)
    rho_out[:m], v_out[:m] = rho, vind
    return rho_out, v_out
