"""Static RPA polarizability as a brute-force band-pair sum (oracle; test infrastructure).

Definition used (Eq. chi1 with the k-discretised Green's function of Sec. VI.D,
N_k^-1 per g, spin sum -> factor s):

    chi0(r, r') = -(2 s / N_k^2) sum_{k,k'} sum_{n occ} sum_{m unocc}
                  Re[ psi_nk*(r) psi_mk'(r) psi_mk'*(r') psi_nk(r') ] * K_{nk,mk'}

with K = 1/(e_mk' - e_nk) (the exact result of the imaginary-axis integral for
one band pair; pairs on the same side of mu integrate to zero) or a quadrature
kernel K = sum_l c_l alpha_l(nk) beta_l(mk') from ``oracle.quadrature``.

Pair densities rho_nm(p) = psi_n*(p) psi_m(p) make the sum a product of
(rows x pairs) and (pairs x cols) matrices; nothing is factored further.
"""
from __future__ import annotations

import numpy as np

from . import quadrature as q


def exact_kernel(E, nocc, mu=None, delta=0.0):
    """Returns kernel(k, kp) -> [nocc, nunocc] array of 1/(x_nk + y_mkp)."""
    if mu is None:
        mu = q.mid_gap(E, nocc)
    x, y = q.offsets(E, nocc, mu, delta)

    def K(k, kp):
        return 1.0 / (x[k][:, None] + y[kp][None, :])
    return K


def quad_kernel(c, alpha, beta):
    def K(k, kp):
        return q.kernel(c, alpha, beta, k, kp)
    return K


def pair_sum(psi_rows, psi_cols, nocc, spin, kern, nblock=16):
    """chi0 over all rows x cols.  psi_*: complex [nk, nb, npts]; returns float64 [nrows, ncols].

    Also returns the largest |Im| of the same sum taken without the real part; it
    vanishes for time-reversal-symmetric orbitals on k-sets closed under k -> -k,
    where the full band sum is real before the real part is taken."""
    acc = pair_acc(psi_rows, psi_cols, nocc, kern, nblock)
    pref = -2.0 * spin / psi_rows.shape[0] ** 2
    return pref * acc.real, float(np.abs(acc.imag).max() * abs(pref))


def pair_acc(psi_rows, psi_cols, nocc, kern, nblock=16):
    """sum_{k,k'} sum_{n occ, m unocc} P_nm(r, r') K_nm(k, k') (complex, no prefactor), with
    P = psi_nk*(r) psi_mk'(r) psi_mk'*(r') psi_nk(r')."""
    nk = psi_rows.shape[0]
    nr, nc = psi_rows.shape[2], psi_cols.shape[2]
    acc = np.zeros((nr, nc), dtype=np.complex128)
    for k in range(nk):
        for kp in range(nk):
            Kmat = kern(k, kp)                                   # [nocc, nu]
            for n0 in range(0, nocc, nblock):
                n1 = min(nocc, n0 + nblock)
                # rho[r, n, m] = conj(psi_nk(r)) psi_mkp(r)
                rr = np.conj(psi_rows[k, n0:n1, :])[:, None, :] * psi_rows[kp, None, nocc:, :]
                rc = np.conj(psi_cols[k, n0:n1, :])[:, None, :] * psi_cols[kp, None, nocc:, :]
                rr = rr * Kmat[n0:n1, :, None]
                nu = rr.shape[1]
                acc += rr.reshape((n1 - n0) * nu, nr).T @ np.conj(rc.reshape((n1 - n0) * nu, nc))
    return acc


def chi0_iw_exact(psi_rows, psi_cols, E, nocc, omega, spin=2, mu=None):
    """chi0(r, r'; i omega): each occupied x unoccupied pair contributes
    P / (i omega - Delta) - conj(P) / (i omega + Delta) (the two orderings of the pair), i.e.
        chi0 = -(2 s / N_k^2) sum [Delta Re P - omega Im P] / (Delta^2 + omega^2),
    Delta = e_mk' - e_nk.  The omega Im P part is odd in omega and vanishes for
    time-reversal-symmetric orbital sets.  Returns (chi0, the largest |odd part|)."""
    if mu is None:
        mu = q.mid_gap(E, nocc)
    x, y = q.offsets(E, nocc, mu)

    def k_even(k, kp):
        d = x[k][:, None] + y[kp][None, :]
        return d / (d * d + omega * omega)

    def k_odd(k, kp):
        d = x[k][:, None] + y[kp][None, :]
        return omega / (d * d + omega * omega)

    pref = -2.0 * spin / psi_rows.shape[0] ** 2
    ev = pair_acc(psi_rows, psi_cols, nocc, k_even)
    od = pair_acc(psi_rows, psi_cols, nocc, k_odd)
    odd = -pref * od.imag
    return pref * ev.real + odd, float(np.abs(odd).max())


def chi0_iw_quad(psi_rows, psi_cols, nocc, spin, cc, cs, alpha, beta):
    """chi0(i omega) with the time rule: sum_l (cc_l + i cs_l) alpha_l beta_l approximates
    (Delta + i omega) / (Delta^2 + omega^2) (cc = c cos(omega tau), cs = c sin(omega tau)),
    and chi0 = -(2 s / N_k^2) sum Re[(K_e + i K_o) P] as in chi0_iw_exact."""
    pref = -2.0 * spin / psi_rows.shape[0] ** 2
    ev = pair_acc(psi_rows, psi_cols, nocc, quad_kernel(cc, alpha, beta))
    od = pair_acc(psi_rows, psi_cols, nocc, quad_kernel(cs, alpha, beta))
    return pref * (ev.real - od.imag)


def chi0_exact(psi_rows, psi_cols, E, nocc, spin=2, mu=None, delta=0.0):
    return pair_sum(psi_rows, psi_cols, nocc, spin, exact_kernel(E, nocc, mu, delta))[0]


def chi0_quad(psi_rows, psi_cols, nocc, spin, c, alpha, beta):
    return pair_sum(psi_rows, psi_cols, nocc, spin, quad_kernel(c, alpha, beta))[0]


def pair_sum_entries(psi_r, psi_c, nocc, spin, kern):
    """chi0 at individual entries: psi_r, psi_c complex [nk, nb, E] hold the orbitals at the
    row point and the column point of each entry; returns float64 [E]."""
    nk = psi_r.shape[0]
    out = np.zeros(psi_r.shape[2], dtype=np.complex128)
    for k in range(nk):
        a = np.conj(psi_r[k, :nocc]) * psi_c[k, :nocc]               # [nocc, E]
        for kp in range(nk):
            b = psi_r[kp, nocc:] * np.conj(psi_c[kp, nocc:])         # [nu, E]
            Kmat = kern(k, kp)
            out += np.einsum("ne,ne->e", a, Kmat @ b)
    return -2.0 * spin / nk ** 2 * out.real


def chi0_iw_quad_entries(psi_r, psi_c, nocc, spin, cc, cs, alpha, beta):
    """chi0_iw_quad at individual entries (psi_r, psi_c as in pair_sum_entries)."""
    nk = psi_r.shape[0]
    ev = np.zeros(psi_r.shape[2], dtype=np.complex128)
    od = np.zeros(psi_r.shape[2], dtype=np.complex128)
    Ke, Ko = quad_kernel(cc, alpha, beta), quad_kernel(cs, alpha, beta)
    for k in range(nk):
        a = np.conj(psi_r[k, :nocc]) * psi_c[k, :nocc]               # [nocc, E]
        for kp in range(nk):
            b = psi_r[kp, nocc:] * np.conj(psi_c[kp, nocc:])         # [nu, E]
            ev += np.einsum("ne,ne->e", a, Ke(k, kp) @ b)
            od += np.einsum("ne,ne->e", a, Ko(k, kp) @ b)
    return -2.0 * spin / nk ** 2 * (ev.real - od.imag)


def chi0_iw_exact_entries(psi_r, psi_c, E, nocc, omega, spin=2, mu=None):
    """chi0_iw_exact at individual entries (psi_r, psi_c as in pair_sum_entries): the even
    kernel Delta / (Delta^2 + omega^2) on Re P and the odd kernel omega / (Delta^2 + omega^2)
    on Im P, per band pair."""
    if mu is None:
        mu = q.mid_gap(E, nocc)
    x, y = q.offsets(E, nocc, mu)
    nk = psi_r.shape[0]
    ev = np.zeros(psi_r.shape[2], dtype=np.complex128)
    od = np.zeros(psi_r.shape[2], dtype=np.complex128)
    for k in range(nk):
        a = np.conj(psi_r[k, :nocc]) * psi_c[k, :nocc]               # [nocc, E]
        for kp in range(nk):
            b = psi_r[kp, nocc:] * np.conj(psi_c[kp, nocc:])         # [nu, E]
            d = x[k][:, None] + y[kp][None, :]
            den = d * d + omega * omega
            ev += np.einsum("ne,ne->e", a, (d / den) @ b)
            od += np.einsum("ne,ne->e", a, (omega / den) @ b)
    return -2.0 * spin / nk ** 2 * (ev.real - od.imag)


def chi0_exact_entries(psi_r, psi_c, E, nocc, spin=2, mu=None, delta=0.0):
    return pair_sum_entries(psi_r, psi_c, nocc, spin, exact_kernel(E, nocc, mu, delta))


def chi0_quad_entries(psi_r, psi_c, nocc, spin, c, alpha, beta):
    return pair_sum_entries(psi_r, psi_c, nocc, spin, quad_kernel(c, alpha, beta))


def terms_for(E, nocc, kind, n, scale=None, mu=None, delta=0.0):
    """Quadrature terms for band energies E: kind 'time' (imaginary time) or 'freq' (paper)."""
    if mu is None:
        mu = q.mid_gap(E, nocc)
    x, y = q.offsets(E, nocc, mu, delta)
    if kind == "time":
        if scale is None or scale <= 0:
            scale = q.auto_scale(x, y, n)
        c, al, be, _ = q.imag_time_terms(x, y, n, scale)
        return c, al, be
    if kind.startswith("time_iw:"):        # "time_iw:<omega>": (c cos, c sin, alpha, beta)
        omega = float(kind.split(":", 1)[1])
        if scale is None or scale <= 0:
            scale = q.auto_scale_iw(x, y, n, omega)
        cc, al, be, tau = q.imag_time_terms_iw(x, y, n, scale, omega)
        c0, _, _, _ = q.imag_time_terms(x, y, n, scale)
        return cc, c0 * np.sin(omega * tau), al, be
    if kind == "freq":
        z = q.zeta(E, mu, metallic=delta > 0) if scale is None or scale <= 0 else scale
        c, al, be, _ = q.freq_terms(x, y, n, z)
        return c, al, be
    raise ValueError(kind)
