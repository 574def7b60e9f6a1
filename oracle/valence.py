"""Valence screened interaction W(x, x') inside r_m from per-point local screening (oracle;
test infrastructure).

Sec. V.A ("Screening for valence-level BSE", Eq. rpa-val): for valence spectra the screening
sites are the points x of the real-space grid.  At each x the external charge is a sphere of
the grid's discretisation volume V_x = Omega / N_x (radius R_x = (3 V_x / 4 pi)^(1/3)),
here of unit charge spread uniformly, whose potential is
    v_ext(r) = (3 - r^2 / R_x^2) / (2 R_x)   (r < R_x),     1 / r   (r >= R_x).
The shell of charge at R_S splits it (Eq. partition): v2 = 1/R_S inside the shell, 1/r beyond,
and v1 = v_ext - v2.  The screened potential W^[x] = eps^-1 v1 + eps^-1 v2 (Eq. W1): the first
part from the local RPA response of the site (the induced-potential solve of oracle.screen,
v1 in the L = 00 channel), the second with the long-wavelength limit of the model screening,
v2 / eps_inf (eps_inf = 1 leaves v2 bare).  So
    W^[x](x + d) = v_ext(|d|) + sum_L v_ind,L(|d|) Y_L(d/|d|) - (1 - 1/eps_inf) v2(|d|),
with v_ind,L the induced potential's radial functions on the site's shells, read at |d| by
4-point (cubic) Lagrange interpolation on the shells nearest to |d|.
    W(x, x') = (W^[x](x') + W^[x'](x)) / 2           for 0 < |x - x'| <= r_m,
    W(x, x)  = (3 / R_x^3) int_0^R_x W^[x]_00(r) r^2 dr,
the l = 0 (spherically averaged) part integrated over the discretisation sphere: the bare
sphere gives 6 / (5 R_x) exactly, the rest is integrated by 8-point Gauss-Legendre on
[0, R_x].  Beyond r_m the paper uses the HLL model, which is out of scope here: those entries
are zero.  Nearest periodic images: d = c' - c - A^T round(A^-T (c' - c)) for lattice vectors
A (rows), or the plain difference without a lattice.
"""
from __future__ import annotations

import math

import numpy as np

from . import screen as sc


def sphere_potential(r, R):
    """Potential of a unit charge spread uniformly over a sphere of radius R."""
    r = np.asarray(r, dtype=np.float64)
    inside = (3.0 - (r / R) ** 2) / (2.0 * R)
    return np.where(r < R, inside, 1.0 / np.maximum(r, 1e-300))


def shell_v2(r, r_shell):
    """v2 of the partition by a shell of charge at R_S (Eq. partition), unit charge."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < r_shell, 1.0 / r_shell, 1.0 / np.maximum(r, 1e-300))


def lagrange4(xs, ys, x):
    """Cubic Lagrange interpolation of samples (xs ascending, at least 4) at x: the four
    nodes nearest to x (clamped at the ends, so it extrapolates beyond them)."""
    n = len(xs)
    i = int(np.searchsorted(xs, x)) - 2
    i = min(max(i, 0), n - 4)
    nodes = xs[i:i + 4]
    vals = ys[..., i:i + 4]
    out = 0.0
    for a in range(4):
        w = 1.0
        for b in range(4):
            if b != a:
                w *= (x - nodes[b]) / (nodes[a] - nodes[b])
        out = out + w * vals[..., a]
    return out


def site_potential(chi0_ss, site, R_x, r_shell, lmax=2):
    """v1 at the site's shells and the induced potential [(L, i)] (L-major) of the sphere's
    v1, through oracle.screen.induced (full l <= lmax response)."""
    v1 = sphere_potential(site.radii, R_x) - shell_v2(site.radii, r_shell)
    _, vind = sc.induced(chi0_ss, site, v1, lmax)
    return vind.reshape((lmax + 1) ** 2, site.n_rad)


def nearest_image(d, cell):
    if cell is None:
        return d
    A = np.asarray(cell, dtype=np.float64)
    f = np.linalg.solve(A.T, d)
    return d - A.T @ np.round(f)


def valence_W(chi0_blocks, sites, centres, vx, r_shell, eps_inf=1.0, r_m=2.0, cell=None,
              lmax=2):
    """Dense [N, N] W(x, x') for sites centred at the points x (centres [N, 3])."""
    N = len(sites)
    R_x = (3.0 * vx / (4.0 * math.pi)) ** (1.0 / 3.0)
    vind = [site_potential(c, s, R_x, r_shell, lmax) for c, s in zip(chi0_blocks, sites)]
    gx, gw = np.polynomial.legendre.leggauss(8)
    W = np.zeros((N, N))

    def one_way(a, d):
        r = float(np.linalg.norm(d))
        Y = sc.real_ylm((d / r)[None, :], lmax)[:, 0]
        vi = lagrange4(sites[a].radii, vind[a], r)
        v2 = float(shell_v2(np.array(r), r_shell))
        return float(sphere_potential(np.array(r), R_x)) + float(vi @ Y) - (1 - 1 / eps_inf) * v2

    for a in range(N):
        # self term: bare sphere 6/(5 R_x), the shell's v2 inside R_S, and the induced l = 0
        # part (Y_00 = 1/sqrt(4 pi)) averaged over the discretisation sphere
        rr = 0.5 * R_x * (gx + 1.0)
        ww = 0.5 * R_x * gw
        v00 = np.array([lagrange4(sites[a].radii, vind[a][0], r) for r in rr]) / math.sqrt(4 * math.pi)
        W[a, a] = (6.0 / (5.0 * R_x) + 3.0 / R_x ** 3 * float((ww * v00 * rr * rr).sum())
                   - (1 - 1 / eps_inf) / r_shell)
        for b in range(N):
            if b == a:
                continue
            d = nearest_image(np.asarray(centres[b], float) - np.asarray(centres[a], float), cell)
            if np.linalg.norm(d) > r_m:
                continue
            W[a, b] = 0.5 * (one_way(a, d) + one_way(b, -d))
    return W
