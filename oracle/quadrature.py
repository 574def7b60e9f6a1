"""Energy-axis quadrature rules as separable non-negative terms (oracle; test infrastructure).

The static polarizability needs, for every occupied band n (x_n = mu - e_n > 0)
and unoccupied band m (y_m = e_m - mu > 0), the factor 1/(e_m - e_n) = 1/(x_n + y_m).
The paper reaches it through an integral along the imaginary energy axis
(Eq. chi1, Appendix D.1.b).  Every rule below approximates it by
    K_nm = sum_l c_l * alpha_l(n) * beta_l(m),   c_l, alpha_l, beta_l >= 0,
so that the band sums factor into per-term Green's functions.

Imaginary time:  1/(x+y) = int_0^inf exp(-x tau) exp(-y tau) d tau, with the
    Gauss-Legendre nodes (a_j, w_j) on (0, 1) mapped by tau = C a/(1-a),
    weight C w/(1-a)^2.  alpha = exp(-x tau_j), beta = exp(-y tau_j), c = weight.

Paper's single-grid frequency rule (Appendix D.1.b): nodes t_j = zeta a_j/(1-a_j)
    with prefactor zeta w_j / (pi (1-a_j)^2), zeta the geometric mean of the
    smallest and largest |mu - e|.  The integrand at -t is the complex conjugate
    of the one at +t, so the real-axis integral is twice the real part of the
    half-line one; the real part of 1/((x+it)(-y+it)) is
    -[x y + t^2] / ((x^2+t^2)(y^2+t^2)), which splits into two separable
    non-negative terms per node: p(t) = x/(x^2+t^2) and q(t) = t/(x^2+t^2).
"""
from __future__ import annotations

import math

import numpy as np

HARTREE_EV = 27.211386245988
METAL_FLOOR = 0.5 / HARTREE_EV      # 0.5 eV added in quadrature to the smallest |mu - e|


def gauss_legendre_01(n: int):
    """Gauss-Legendre nodes and weights shifted and scaled to (0, 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def mid_gap(E: np.ndarray, nocc: int) -> float:
    """mu in the middle of the global gap over all k (Sec. VI.D)."""
    return 0.5 * (E[:, :nocc].max() + E[:, nocc:].min())


def regularised(d: np.ndarray, delta: float) -> np.ndarray:
    """The metallic regularisation of Sec. VI.D applied to offsets d = mu - e: the offset keeps
    its sign and takes delta in quadrature, d -> sign(d) sqrt(d^2 + delta^2); delta = 0 leaves
    it unchanged."""
    d = np.asarray(d, dtype=np.float64)
    if delta <= 0:
        return d
    return np.sign(d) * np.sqrt(d * d + delta * delta)


def offsets(E: np.ndarray, nocc: int, mu: float, delta: float = 0.0):
    """x = mu - e_occ > 0 and y = e_unocc - mu > 0, regularised by delta (Sec. VI.D).

    Which side of mu a band lies on decides whether it is occupied.  Here the lowest nocc
    bands at every k are the occupied ones, so every one of them must lie below mu and every
    other band above it; a band on the other side would make the occupied count depend on k,
    which this form does not express (ValueError)."""
    x = mu - E[:, :nocc]
    y = E[:, nocc:] - mu
    if not (x.min() > 0 and y.min() > 0):
        raise ValueError("a band lies on the other side of mu than its occupation says")
    # y = e - mu is minus the offset mu - e: regularise the offset, then flip the sign
    return regularised(x, delta), -regularised(-y, delta)


def imag_time_terms(x, y, n: int, scale: float):
    """Returns c [n], alpha [n, nk, nocc], beta [n, nk, nunocc], tau [n]."""
    a, w = gauss_legendre_01(n)
    tau = scale * a / (1.0 - a)
    c = scale * w / (1.0 - a) ** 2
    alpha = np.exp(-x[None, :, :] * tau[:, None, None])
    beta = np.exp(-y[None, :, :] * tau[:, None, None])
    return c, alpha, beta, tau


def imag_time_error(scale: float, n: int, dmin: float, dmax: float, nsample: int = 512) -> float:
    """max over log-spaced Delta in [dmin, dmax] of |Delta * K(Delta) - 1| for the imaginary-time rule."""
    a, w = gauss_legendre_01(n)
    tau = scale * a / (1.0 - a)
    c = scale * w / (1.0 - a) ** 2
    d = np.exp(np.linspace(math.log(dmin), math.log(dmax), nsample))
    K = (c[None, :] * np.exp(-d[:, None] * tau[None, :])).sum(1)
    return float(np.abs(d * K - 1.0).max())


def auto_scale(x, y, n: int) -> float:
    """Scale C = kappa / sqrt(Dmin Dmax) with kappa = 10^(j/40), j = -80..100, chosen to
    minimise the worst relative error over [Dmin, Dmax] (smallest kappa on ties)."""
    dmin = float(x.min() + y.min())
    dmax = float(x.max() + y.max())
    g = math.sqrt(dmin * dmax)
    best, best_s = None, None
    for j in range(-80, 101):
        s = 10.0 ** (j / 40.0) / g
        e = imag_time_error(s, n, dmin, dmax)
        if best is None or e < best:
            best, best_s = e, s
    return best_s


def imag_time_terms_iw(x, y, n: int, scale: float, omega: float):
    """The same rule for the polarizability at imaginary frequency i omega, whose even part
    needs Delta / (Delta^2 + omega^2) = int_0^inf cos(omega tau) exp(-Delta tau) d tau: the
    coefficients take the factor cos(omega tau_l) (and may be negative)."""
    c, alpha, beta, tau = imag_time_terms(x, y, n, scale)
    return c * np.cos(omega * tau), alpha, beta, tau


def imag_time_error_iw(scale: float, n: int, dmin: float, dmax: float, omega: float,
                       nsample: int = 512) -> float:
    """max over log-spaced Delta in [dmin, dmax] of |K(Delta) / k(Delta) - 1|, with
    k = Delta / (Delta^2 + omega^2) and K the cos-weighted rule."""
    a, w = gauss_legendre_01(n)
    tau = scale * a / (1.0 - a)
    c = scale * w / (1.0 - a) ** 2 * np.cos(omega * tau)
    d = np.exp(np.linspace(math.log(dmin), math.log(dmax), nsample))
    K = (c[None, :] * np.exp(-d[:, None] * tau[None, :])).sum(1)
    return float(np.abs(K * (d * d + omega * omega) / d - 1.0).max())


def auto_scale_iw(x, y, n: int, omega: float) -> float:
    """auto_scale with the imaginary-frequency error model (the static scan at omega = 0)."""
    if omega == 0.0:
        return auto_scale(x, y, n)
    dmin = float(x.min() + y.min())
    dmax = float(x.max() + y.max())
    g = math.sqrt(dmin * dmax)
    best, best_s = None, None
    for j in range(-80, 101):
        s = 10.0 ** (j / 40.0) / g
        e = imag_time_error_iw(s, n, dmin, dmax, omega)
        if best is None or e < best:
            best, best_s = e, s
    return best_s


def zeta(E: np.ndarray, mu: float, metallic: bool = False) -> float:
    """Geometric mean of the smallest and largest |mu - e| over all bands and k."""
    d = np.abs(mu - E)
    lo = d.min()
    if metallic:
        lo = math.sqrt(lo * lo + METAL_FLOOR ** 2)
    return math.sqrt(lo * d.max())


def freq_terms(x, y, n: int, z: float):
    """Paper's single-grid rule folded to t > 0: 2n terms (p-terms then q-terms).
    Returns c [2n], alpha [2n, nk, nocc], beta [2n, nk, nunocc], t [n]."""
    a, w = gauss_legendre_01(n)
    t = z * a / (1.0 - a)
    cj = z * w / (math.pi * (1.0 - a) ** 2)
    t3 = t[:, None, None]
    px = x[None] / (x[None] ** 2 + t3 ** 2)
    qx = t3 / (x[None] ** 2 + t3 ** 2)
    py = y[None] / (y[None] ** 2 + t3 ** 2)
    qy = t3 / (y[None] ** 2 + t3 ** 2)
    c = np.concatenate([cj, cj])
    alpha = np.concatenate([px, qx])
    beta = np.concatenate([py, qy])
    return c, alpha, beta, t


def kernel(c, alpha, beta, k: int, kp: int) -> np.ndarray:
    """K_nm for occupied bands at k and unoccupied bands at kp: sum_l c_l alpha_l(k,n) beta_l(kp,m)."""
    return np.einsum("l,ln,lm->nm", c, alpha[:, k, :], beta[:, kp, :])


def auto_nodes(x, y, tol: float, nmin: int = 24, nmax: int = 32):
    """The smallest node count n in [nmin, nmax] whose imaginary-time rule (with its own
    auto_scale) keeps the worst per-pair relative error over [Dmin, Dmax] at or below tol; nmax
    if none does.  Returns (n, scale, error)."""
    dmin = float(x.min() + y.min())
    dmax = float(x.max() + y.max())
    for n in range(nmin, nmax + 1):
        s = auto_scale(x, y, n)
        e = imag_time_error(s, n, dmin, dmax)
        if e <= tol or n == nmax:
            return n, s, e
