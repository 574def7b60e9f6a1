"""ALDA vertex correction of the site-local screening (oracle; test infrastructure).

App. (ALDA): with the local exchange-correlation potential as first-order self-energy, the
reducible polarizability becomes (Eq. chi-alda)
    chi~ = (1 - chi0 (v + f_xc))^-1 chi0,
with the contact kernel of Eq. kxc_alda, f_xc(r, r') = delta(r - r') dv_xc/dn at n(r), the
second derivative of the LDA exchange-correlation energy density taken by a 5-point finite
difference with density steps of 0.01 e/bohr^3.  The LDA: Slater exchange and the
Vosko-Wilk-Nusair (1980) paramagnetic fit to the Ceperley-Alder correlation energy, all in
Hartree atomic units.

In the radial x real-Y_lm basis of ``oracle.screen`` (operators compose as A D B) the contact
kernel is block-diagonal in the shell index:
    F_{(L,i),(L',i)} = sum_a w_a Y_L(a) f_xc(r_i a) Y_L'(a),    K = F D^-1,
and the screened interaction for the ALDA polarizability is
    W~ = V + V D chi~ D V,   chi~ = (I - X D (V + K) D)^-1 X.

Parity: the exchange part is pinned against its closed-form second derivative, the
correlation form against its high- and low-density limits (its fit constants are the
published ones and are not pinned to printed values: "parity unpinned" for those), the
finite difference against a finer one, and W~ against W for f_xc = 0 and against a second
route through eps; see ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import math

import numpy as np

from . import screen as sc

# VWN paramagnetic fit to the Ceperley-Alder data, Hartree: A, x0, b, c
VWN_A, VWN_X0, VWN_B, VWN_C = 0.0310907, -0.10498, 3.72744, 12.9352
FD_STEP = 0.01


def eps_x(n):
    """Exchange energy per electron of the uniform gas: -(3/4) (3 n / pi)^(1/3)."""
    return -0.75 * np.cbrt(3.0 * np.asarray(n, dtype=np.float64) / math.pi)


def eps_c(n):
    """VWN correlation energy per electron, x = sqrt(r_s), X(x) = x^2 + b x + c."""
    n = np.asarray(n, dtype=np.float64)
    rs = np.cbrt(3.0 / (4.0 * math.pi * n))
    x = np.sqrt(rs)
    A, x0, b, c = VWN_A, VWN_X0, VWN_B, VWN_C
    Q = math.sqrt(4.0 * c - b * b)
    X = x * x + b * x + c
    X0 = x0 * x0 + b * x0 + c
    at = np.arctan(Q / (2.0 * x + b))
    return A * (np.log(x * x / X) + 2.0 * b / Q * at
                - b * x0 / X0 * (np.log((x - x0) ** 2 / X) + 2.0 * (b + 2.0 * x0) / Q * at))


def e_xc(n):
    """Exchange-correlation energy per volume n (eps_x + eps_c)."""
    n = np.asarray(n, dtype=np.float64)
    return n * (eps_x(n) + eps_c(n))


def fxc(n, h=FD_STEP, energy=e_xc):
    """f_xc(n) = d^2 e / dn^2 (e = e_xc by default) by the 5-point central difference with
    step h; where n < 4h the step shrinks to n/4 so that every density in the stencil stays
    positive (a reading: the paper does not say); zero for n <= 0."""
    n = np.asarray(n, dtype=np.float64)
    out = np.zeros_like(n)
    pos = n > 0
    nn = n[pos]
    hh = np.minimum(h, nn / 4.0)
    out[pos] = (-energy(nn + 2 * hh) + 16 * energy(nn + hh) - 30 * energy(nn)
                + 16 * energy(nn - hh) - energy(nn - 2 * hh)) / (12.0 * hh * hh)
    return out


def contact_matrix(site, f_points, lmax=2):
    """F [(nL n_rad), (nL n_rad)]: F_{(L,i),(L',i)} = sum_a w_a Y_L(a) f(r_i a) Y_L'(a), for
    f at the site's points (radial-major, [n_rad * n_ang])."""
    Y = sc.real_ylm(site.ang_xyz, lmax)                 # [nL, n_ang]
    nL = Y.shape[0]
    nr, na = site.n_rad, site.n_ang
    f = np.asarray(f_points, dtype=np.float64).reshape(nr, na)
    F = np.zeros((nL, nr, nL, nr))
    for i in range(nr):
        F[:, i, :, i] = (Y * (site.ang_w * f[i])[None, :]) @ Y.T
    return F.reshape(nL * nr, nL * nr)


def screen_W_alda(chi0_ss, site, density, lmax=2, f_points=None):
    """W~ = V + V D chi~ D V with chi~ = (I - X D (V + K) D)^-1 X, K = F D^-1, for the
    density at the site's points (or the kernel values f_points given directly)."""
    X = sc.project(chi0_ss, site, lmax)
    V = sc.coulomb(site, lmax)
    d = sc.radial_weights(site, lmax)
    D = np.diag(d)
    f = fxc(density) if f_points is None else f_points
    K = contact_matrix(site, f, lmax) / d[None, :]
    n = V.shape[0]
    chi = np.linalg.solve(np.eye(n) - X @ D @ (V + K) @ D, X)
    return V + V @ D @ chi @ D @ V
