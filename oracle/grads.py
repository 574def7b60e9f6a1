"""Reference gradients of the test-charge loss (oracle; test infrastructure).

Loss: L = sum_sites rho_L^T D W D rho_L with W from the site x site chi0 block
(``oracle.screen``).  Back through the solve, dL/dX = D W^T Gbar W^T D with
Gbar = (D rho_L)(D rho_L)^T, so on the site points the sensitivity
Lambda = dL/dchi0 = P^T (dL/dX) P is the rank-one g g^T with
g = P^T D W D rho_L (W symmetric).

With P_f = -2 s / N_k^2 and, per site, the band-pair matrix element
    M_{nk,mk'} = sum_p g(p) psi_nk*(p) psi_mk'(p),
the loss's dependence on chi0 is Q = P_f sum |M|^2 K_{nk,mk'} and
    dL/de_nk  = P_f sum_{m,k'} |M|^2 dK/de_nk
    dL/de_mk' = P_f sum_{n,k}  |M|^2 dK/de_mk'
    grad psi_nk(p)  = 2 P_f g(p) sum_{m,k'} conj(M) K psi_mk'(p)
    grad psi_mk'(p) = 2 P_f g(p) sum_{n,k}  M K psi_nk(p)
(complex gradients as dL/dRe + i dL/dIm).  Exact denominators: K = 1/Delta,
dK/de_n = 1/Delta^2, dK/de_m = -1/Delta^2.  Imaginary-time terms with mu and
the nodes held fixed: dK/de_n = sum_l c_l tau_l alpha beta, dK/de_m = -that.  With the
metallic regularisation each offset's derivative carries the chain factor of its square root.

At imaginary frequency (complex kernel z = K_e + i K_o per pair, chi0 = P_f sum
Re[z rho(r) conj(rho(c))] with rho = psi_nk* psi_mk'), for a linear functional
L = sum_{r,c} Lambda(r, c) chi0(r, c) with an arbitrary real Lambda per site block:
    M = rho^T Lambda conj(rho),   L = P_f sum Re[z M],   dL/de = P_f sum Re[(dz/de) M]
    grad psi_nk(p)  = P_f sum_{m,k'} psi_mk'(p) [z (Lambda conj(rho))(p) + conj(z) (Lambda^T conj(rho))(p)]
    grad psi_mk'(p) = P_f sum_{n,k}  psi_nk(p)  [z (Lambda^T rho)(p) + conj(z) (Lambda rho)(p)]
(``linear_grads_iw``; Wirtinger derivatives, gradients as dL/dRe + i dL/dIm).
"""
from __future__ import annotations

import numpy as np

from . import chi0 as cz
from . import quadrature as q
from . import screen as sc


def site_slices(sites):
    o, out = 0, []
    for s in sites:
        out.append(slice(o, o + s.npts))
        o += s.npts
    return out


def loss(psi_site, E, nocc, spin, sites, rho, kern, lmax=2):
    """Test-charge loss and the per-site W; kern as in oracle.chi0."""
    total, Ws = 0.0, []
    for s, sl in zip(sites, site_slices(sites)):
        ps = psi_site[:, :, sl]
        chi = cz.pair_sum(ps, ps, nocc, spin, kern)[0]
        W = sc.screen_W(chi, s, lmax)
        Ws.append(W)
        total += sc.test_charge_loss(W, rho[sl], s, lmax)
    return total, Ws


def _chain(E, nocc, mu, delta):
    """Regularised offsets X, Y (Sec. VI.D) and their derivatives with respect to the band
    energy, mu fixed: X = sqrt((mu - e)^2 + delta^2) gives dX/de = -(mu - e)/X, and
    Y = sqrt((e - mu)^2 + delta^2) gives dY/de = (e - mu)/Y (-1 and +1 when delta = 0)."""
    X, Y = q.offsets(E, nocc, mu, delta)
    return X, Y, -(mu - E[:, :nocc]) / X, (E[:, nocc:] - mu) / Y


def _kernels_exact(E, nocc, mu, delta):
    x, y, dx, dy = _chain(E, nocc, mu, delta)

    def K(k, kp):
        d = x[k][:, None] + y[kp][None, :]
        return 1.0 / d, -dx[k][:, None] / d ** 2, -dy[kp][None, :] / d ** 2
    return K


def _kernels_time(E, nocc, mu, n, scale, delta=0.0):
    x, y, dx, dy = _chain(E, nocc, mu, delta)
    c, al, be, tau = q.imag_time_terms(x, y, n, scale)

    def K(k, kp):
        base = np.einsum("l,ln,lm->nm", c, al[:, k], be[:, kp])
        # d exp(-x tau)/de = -tau exp(-x tau) dx/de, likewise for y
        d = np.einsum("l,ln,lm->nm", c * tau, al[:, k], be[:, kp])
        return base, -d * dx[k][:, None], -d * dy[kp][None, :]
    return K


def loss_and_grads(psi_site, E, nocc, spin, sites, rho, kind="exact", n_terms=None,
                   scale=None, lmax=2, delta=0.0, with_W=False):
    """Returns (loss, dL/dE [nk, nb], dL/dpsi_site complex [nk, nb, npts]), and the per-site W
    as a fourth item when with_W; delta is the metallic regularisation of Sec. VI.D (mu
    mid-gap and fixed)."""
    mu = q.mid_gap(E, nocc)
    if kind == "exact":
        kfun = _kernels_exact(E, nocc, mu, delta)
        kern = cz.exact_kernel(E, nocc, mu, delta)
    elif kind == "time":
        kfun = _kernels_time(E, nocc, mu, n_terms, scale, delta)
        c, al, be = cz.terms_for(E, nocc, "time", n_terms, scale, mu, delta)
        kern = cz.quad_kernel(c, al, be)
    else:
        raise ValueError(kind)
    L, Ws = loss(psi_site, E, nocc, spin, sites, rho, kern, lmax)
    nk = E.shape[0]
    Pf = -2.0 * spin / nk ** 2
    dE = np.zeros_like(E)
    dpsi = np.zeros_like(psi_site)
    for s, sl, W in zip(sites, site_slices(sites), Ws):
        Wsym = 0.5 * (W + W.T)
        d = sc.radial_weights(s, lmax)
        rl = sc.charge_moments(rho[sl], s, lmax)
        g = sc.projector(s, lmax).T @ (d * (Wsym @ (d * rl)))
        po = psi_site[:, :nocc, sl]
        pu = psi_site[:, nocc:, sl]
        for k in range(nk):
            for kp in range(nk):
                M = (np.conj(po[k]) * g[None, :]) @ pu[kp].T          # [nocc, nu]
                Km, dKn, dKm = kfun(k, kp)
                M2 = (M * np.conj(M)).real
                dE[k, :nocc] += Pf * (M2 * dKn).sum(1)
                dE[kp, nocc:] += Pf * (M2 * dKm).sum(0)
                dpsi[k, :nocc, sl] += 2 * Pf * g[None, :] * ((np.conj(M) * Km) @ pu[kp])
                dpsi[kp, nocc:, sl] += 2 * Pf * g[None, :] * ((M * Km).T @ po[k])
    if with_W:
        return L, dE, dpsi, Ws
    return L, dE, dpsi


def iw_terms(E, nocc, n, scale, omega, mu=None):
    """Imaginary-time terms at i omega: (cc, cs, alpha, beta, tau) with cc = c cos(omega tau),
    cs = c sin(omega tau) (oracle.quadrature)."""
    if mu is None:
        mu = q.mid_gap(E, nocc)
    x, y = q.offsets(E, nocc, mu)
    c, al, be, tau = q.imag_time_terms(x, y, n, scale)
    return c * np.cos(omega * tau), c * np.sin(omega * tau), al, be, tau


def linear_loss_iw(psi_site, nocc, spin, sites, lam_blocks, cc, cs, al, be):
    """L = sum_sites sum_{r,c} Lambda_s(r, c) chi0_iw(r, c) with the quadrature chi0."""
    total = 0.0
    for sl, lam in zip(site_slices(sites), lam_blocks):
        ps = psi_site[:, :, sl]
        total += float((lam * cz.chi0_iw_quad(ps, ps, nocc, spin, cc, cs, al, be)).sum())
    return total


def linear_grads_iw(psi_site, E, nocc, spin, sites, lam_blocks, n, scale, omega, mu=None):
    """(L, dL/dE [nk, nb], dL/dpsi_site complex [nk, nb, npts]) for the linear functional of
    chi0(i omega) above; mu and the nodes held fixed."""
    cc, cs, al, be, tau = iw_terms(E, nocc, n, scale, omega, mu)
    nk = E.shape[0]
    Pf = -2.0 * spin / nk ** 2
    dE = np.zeros_like(E)
    dpsi = np.zeros_like(psi_site)
    L = 0.0
    for sl, lam in zip(site_slices(sites), lam_blocks):
        po = psi_site[:, :nocc, sl]
        pu = psi_site[:, nocc:, sl]
        for k in range(nk):
            for kp in range(nk):
                z = (np.einsum("l,ln,lm->nm", cc, al[:, k], be[:, kp])
                     + 1j * np.einsum("l,ln,lm->nm", cs, al[:, k], be[:, kp]))
                dz = (np.einsum("l,ln,lm->nm", cc * tau, al[:, k], be[:, kp])
                      + 1j * np.einsum("l,ln,lm->nm", cs * tau, al[:, k], be[:, kp]))
                rho = np.conj(po[k])[:, None, :] * pu[kp][None, :, :]     # [nocc, nu, p]
                lr_c = np.conj(rho) @ lam.T           # (Lambda conj(rho))(p)
                ltr_c = np.conj(rho) @ lam            # (Lambda^T conj(rho))(p)
                M = np.einsum("nmp,nmp->nm", rho, lr_c)
                L += Pf * float((z * M).real.sum())
                dE[k, :nocc] += Pf * (dz * M).real.sum(1)
                dE[kp, nocc:] -= Pf * (dz * M).real.sum(0)
                dpsi[k, :nocc, sl] += Pf * np.einsum(
                    "mp,nmp->np", pu[kp], z[:, :, None] * lr_c + np.conj(z)[:, :, None] * ltr_c)
                lt_r = rho @ lam                      # (Lambda^T rho)(p)
                l_r = rho @ lam.T                     # (Lambda rho)(p)
                dpsi[kp, nocc:, sl] += Pf * np.einsum(
                    "np,nmp->mp", po[k], z[:, :, None] * lt_r + np.conj(z)[:, :, None] * l_r)
    return L, dE, dpsi
