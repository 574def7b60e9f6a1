"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: adaptive
numerical integration, a plane-wave closed form, brute-force loops, exact
invariants of the static RPA polarizability (symmetry, sign, sum rule, gauge,
translation, k-set replication), the push-through identity between the two
forms of W in the paper, and finite differences of the loss.
"""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

from oracle import chi0 as cz
from oracle import grads as gr
from oracle import quadrature as q
from oracle import screen as sc
from tests.conftest import workload
from workloads import configs, sites as sx


# --------------------------------------------------------------------------- quadrature
@pytest.mark.parametrize("x,y", [(0.02, 0.03), (0.3, 1.7), (1.0, 0.05)])
def test_pair_identity_adaptive_integration(x, y):
    """Per band pair, the imaginary-axis integral of Eq. chi1 gives -1/(x+y); both separable
    integrands used by the rules integrate to 1/(x+y) (scipy adaptive quadrature)."""
    full = integrate.quad(lambda t: ((x * y + t * t) / ((x * x + t * t) * (y * y + t * t))),
                          0, np.inf, epsabs=0, epsrel=1e-13, limit=500)[0] / math.pi
    time = integrate.quad(lambda s: math.exp(-(x + y) * s), 0, np.inf, epsabs=0, epsrel=1e-13)[0]
    # the complex integrand of Eq. chi1 over the whole imaginary axis, integrated numerically
    re = integrate.quad(lambda t: (1.0 / ((x + 1j * t) * (-y + 1j * t))).real, -np.inf, np.inf,
                        epsabs=0, epsrel=1e-13, limit=500)[0] / (2 * math.pi)
    im = integrate.quad(lambda t: (1.0 / ((x + 1j * t) * (-y + 1j * t))).imag, -np.inf, np.inf,
                        epsabs=1e-14, limit=500)[0]
    assert abs(full * (x + y) - 1) < 1e-11
    assert abs(time * (x + y) - 1) < 1e-11
    assert abs(re * (x + y) + 1) < 1e-10
    assert abs(im) < 1e-10
    # same-sign pairs integrate to zero
    same = integrate.quad(lambda t: (1.0 / ((x + 1j * t) * (y + 1j * t))).real, -np.inf, np.inf,
                          epsabs=1e-13, limit=500)[0]
    assert abs(same) < 1e-9


@pytest.mark.parametrize("kind", ["time", "freq"])
def test_rules_converge_to_adaptive_integral(kind):
    """The oracle's separable rules approach the adaptively integrated 1/(x+y), with the
    error shrinking as nodes are added, at R = Dmax/Dmin = 50."""
    xs = np.array([[0.025, 0.1, 0.6]])
    ys = np.array([[0.025, 0.3, 0.65]])
    ref = np.array([[integrate.quad(lambda s: math.exp(-(a + b) * s), 0, np.inf, epsrel=1e-14)[0]
                     for b in ys[0]] for a in xs[0]])
    errs = []
    for n in (8, 16, 32):
        if kind == "time":
            c, al, be, _ = q.imag_time_terms(xs, ys, n, q.auto_scale(xs, ys, n))
        else:
            E = np.concatenate([-xs, ys], 1)
            c, al, be, _ = q.freq_terms(xs, ys, n, q.zeta(E, 0.0))
        K = q.kernel(c, al, be, 0, 0)
        assert np.all(c >= 0) and np.all(al >= 0) and np.all(be >= 0)
        errs.append(np.abs(K / ref - 1).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-9


def test_gauss_legendre_01_exact_for_polynomials():
    a, w = q.gauss_legendre_01(8)
    for p in range(16):
        assert abs((w * a ** p).sum() - 1.0 / (p + 1)) < 1e-14


def test_time_rule_scale_choice_is_optimal_on_scan():
    x = np.array([[0.03, 0.2, 0.9]])
    y = np.array([[0.02, 0.5, 1.1]])
    s = q.auto_scale(x, y, 16)
    e0 = q.imag_time_error(s, 16, 0.05, 2.0)
    for f in (0.5, 0.8, 1.25, 2.0):
        assert q.imag_time_error(s * f, 16, 0.05, 2.0) >= e0 * 0.999


# --------------------------------------------------------------------------- chi0 structure
def _brute_chi0(psi_r, psi_c, E, nocc, spin):
    """Six nested loops over the definition (tiny sizes only)."""
    nk, nb, nr = psi_r.shape
    nc = psi_c.shape[2]
    mu = 0.5 * (E[:, :nocc].max() + E[:, nocc:].min())
    out = np.zeros((nr, nc))
    for i in range(nr):
        for j in range(nc):
            s = 0.0
            for k in range(nk):
                for kp in range(nk):
                    for n in range(nocc):
                        for m in range(nocc, nb):
                            v = (np.conj(psi_r[k, n, i]) * psi_r[kp, m, i]
                                 * np.conj(psi_c[kp, m, j]) * psi_c[k, n, j])
                            s += v.real / (E[kp, m] - E[k, n])
            out[i, j] = -2 * spin / nk ** 2 * s
    assert mu is not None
    return out


def test_node_count_picked_from_the_energy_range(tiny):
    """auto_nodes: the chosen rule meets the bound and one node fewer does not (on the same
    error model), and the bound holds for every actual band pair of the tiny workload, whose
    kernel is summed term by term against the exact 1/(x + y)."""
    w = tiny
    mu = q.mid_gap(w.energies, w.nocc)
    x, y = q.offsets(w.energies, w.nocc, mu)
    dmin, dmax = x.min() + y.min(), x.max() + y.max()
    for tol in (1e-6, 1e-9, 1e-11):
        n, s, e = q.auto_nodes(x, y, tol, 12, 32)
        assert e <= tol
        if n > 12:
            assert q.imag_time_error(q.auto_scale(x, y, n - 1), n - 1, dmin, dmax) > tol
        c, al, be, _ = q.imag_time_terms(x, y, n, s)
        K = q.kernel(c, al, be, 0, 0)
        pair = np.abs(K * (x[0][:, None] + y[0][None, :]) - 1.0).max()
        assert pair <= 1.05 * e
    # a band-energy range that no count in range meets: the largest count
    n, s, e = q.auto_nodes(x, y, 1e-30, 20, 24)
    assert n == 24 and e > 1e-30


def test_pair_sum_matches_brute_force_loops():
    rng = np.random.default_rng(7)
    nk, nb, nocc, nr, nc = 2, 6, 2, 3, 4
    pr = rng.normal(size=(nk, nb, nr)) + 1j * rng.normal(size=(nk, nb, nr))
    pc = rng.normal(size=(nk, nb, nc)) + 1j * rng.normal(size=(nk, nb, nc))
    E = np.sort(rng.uniform(-1, 1, size=(nk, nb)), axis=1)
    E[:, nocc:] += 2.0
    got = cz.chi0_exact(pr, pc, E, nocc, spin=2)
    ref = _brute_chi0(pr, pc, E, nocc, 2)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # and the entry-wise form
    ent = cz.chi0_exact_entries(pr[:, :, [0, 2, 1]], pc[:, :, [3, 0, 1]], E, nocc, 2)
    assert np.abs(ent - ref[[0, 2, 1], [3, 0, 1]]).max() < 1e-12 * np.abs(ref).max()


def test_free_electron_closed_form():
    """V = 0 at Gamma: psi = e^{iG.r}/sqrt(Omega), e = |G|^2/2, closed shells on both sides;
    chi0(r,r') = -(2s/Omega^2) sum_{G occ, G' unocc} cos((G'-G).(r-r')) / (e' - e)."""
    fe = configs.free_electron()
    G, E, nocc, omega = fe["G"], fe["E"], fe["nocc"], fe["omega"]
    pts, gp = fe["pts"], fe["grid_pts"][::37]
    got = cz.chi0_exact(fe["psi_site"], fe["psi_site"][:, :, :], E, nocc)
    got_g = cz.chi0_exact(fe["psi_site"], fe["psi_grid"][:, :, ::37], E, nocc)
    dG = G[None, nocc:, :] - G[:nocc, None, :]                       # [occ, unocc, 3]
    den = E[0, nocc:][None, :] - E[0, :nocc][:, None]

    def closed(r, rp):
        d = r[:, None, :] - rp[None, :, :]
        ph = np.einsum("nmx,ijx->ijnm", dG, d)
        return -4.0 / omega ** 2 * (np.cos(ph) / den).sum((2, 3))
    ref = closed(pts, pts)
    ref_g = closed(pts, gp)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(got_g - ref_g).max() < 1e-12 * np.abs(ref_g).max()


def test_replicated_kset_invariance(tiny):
    """Passing the same k-point twice must leave chi0 unchanged: pins the N_k^-2 factor of the
    double k-sum (one power per Green's function)."""
    w = tiny
    ps = w.psi_site.numpy()[:, :, :40]
    a = cz.chi0_exact(ps, ps, w.energies, w.nocc)
    ps2 = np.concatenate([ps, ps])
    E2 = np.concatenate([w.energies, w.energies])
    b = cz.chi0_exact(ps2, ps2, E2, w.nocc)
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


def test_structure_tiny(tiny):
    """Symmetry, vanishing imaginary part, negative semidefiniteness, gauge invariance and
    the charge sum rule on the cell grid at Gamma."""
    w = tiny
    ps = w.psi_site.numpy()
    pg = w.psi_grid.numpy()
    kern = cz.exact_kernel(w.energies, w.nocc)
    ss, im = cz.pair_sum(ps, ps, w.nocc, 2, kern)
    scale = np.abs(ss).max()
    assert np.abs(ss - ss.T).max() < 1e-14 * scale
    assert im < 1e-14 * scale
    lam = np.linalg.eigvalsh(ss)
    assert lam.max() <= 1e-12 * abs(lam.min())
    # gauge: psi_n -> e^{i theta_n} psi_n
    th = np.random.default_rng(3).uniform(0, 2 * np.pi, size=(1, w.nb, 1))
    g = cz.chi0_exact(ps * np.exp(1j * th), ps * np.exp(1j * th), w.energies, w.nocc)
    assert np.abs(g - ss).max() < 1e-13 * scale
    # sum rule: sum_r' chi0(r, r') dV = 0 (orbitals orthonormal on the alias-free grid)
    sg = cz.chi0_exact(ps, pg, w.energies, w.nocc)
    rowsum = sg.sum(1) * w.grid_dV
    assert np.abs(rowsum).max() < 1e-12 * np.abs(sg).max() * pg.shape[2] * w.grid_dV
    # NSD of the grid x grid block
    gg = cz.chi0_exact(pg[:, :, ::5], pg[:, :, ::5], w.energies, w.nocc)
    lg = np.linalg.eigvalsh(gg)
    assert lg.max() <= 1e-12 * abs(lg.min())


def test_translation_and_mu_independence():
    """chi0(r+R, r'+R) = chi0(r, r') for a lattice vector R with k-points; the
    imaginary-time quadrature is independent of mu inside the gap."""
    w = workload("production", with_grid=False)
    cr = w.bands.crystal
    from workloads import crystal as cx
    pts = w.sites[0].points()[::53]
    shift = np.array([cr.a, -cr.a, 2 * cr.a])
    pa = torch.stack([cx.psi_at_points(w.bands, pts, k) for k in range(w.nk)]).numpy()
    pb = torch.stack([cx.psi_at_points(w.bands, pts + shift, k) for k in range(w.nk)]).numpy()
    E, nocc = w.energies, w.nocc
    a = cz.chi0_exact(pa, pa, E, nocc)
    b = cz.chi0_exact(pb, pb, E, nocc)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()
    mu0 = q.mid_gap(E, nocc)
    gap = E[:, nocc:].min() - E[:, :nocc].max()
    c1 = cz.chi0_quad(pa, pa, nocc, 2, *cz.terms_for(E, nocc, "time", 16, scale=3.0, mu=mu0))
    c2 = cz.chi0_quad(pa, pa, nocc, 2, *cz.terms_for(E, nocc, "time", 16, scale=3.0,
                                                     mu=mu0 + 0.3 * gap))
    assert np.abs(c1 - c2).max() < 1e-13 * np.abs(c1).max()


@pytest.mark.parametrize("kind,n,tol", [("time", 16, 2e-6), ("time", 32, 1e-9), ("freq", 32, 1e-8)])
def test_quadrature_chi0_converges_to_exact(tiny, kind, n, tol):
    w = tiny
    ps = w.psi_site.numpy()
    ex = cz.chi0_exact(ps, ps, w.energies, w.nocc)
    c, al, be = cz.terms_for(w.energies, w.nocc, kind, n)
    qu = cz.chi0_quad(ps, ps, w.nocc, 2, c, al, be)
    assert np.abs(qu - ex).max() < tol * np.abs(ex).max()
    lam = np.linalg.eigvalsh(qu)
    assert lam.max() <= 1e-12 * abs(lam.min())


# --------------------------------------------------------------------------- W
def test_real_ylm_orthonormal_under_lebedev():
    for n in (26, 50, 110):
        x, wgt = sx.angular_rule(n)
        Y = sc.real_ylm(x)
        S = (Y * wgt[None, :]) @ Y.T
        assert np.abs(S - np.eye(9)).max() < 1e-13


def test_real_ylm_values_against_scipy():
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(1)
    v = rng.normal(size=(5, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    theta = np.arccos(v[:, 2])
    phi = np.arctan2(v[:, 1], v[:, 0])
    Y = sc.real_ylm(v)
    for l in range(3):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                ref = c.real
            elif m > 0:
                ref = math.sqrt(2) * (-1) ** m * c.real
            else:
                ref = math.sqrt(2) * (-1) ** m * c.imag
            assert np.abs(Y[l * l + l + m] - ref).max() < 1e-13


def test_W_special_cases(tiny):
    site = tiny.sites[0]
    n = site.npts
    V = sc.coulomb(site)
    assert np.abs(sc.screen_W(np.zeros((n, n)), site) - V).max() == 0.0
    # one shell, isotropic chi0: only the L = 00 channel is non-zero -> scalar solve
    one = sx.make_site(np.zeros(3), 1, 26, r_max=1.5)
    chi = -0.3 * np.ones((26, 26))
    W = sc.screen_W(chi, one, lmax=2)
    x00 = (one.ang_w.sum() / (2 * math.sqrt(math.pi))) ** 2 * -0.3
    v00 = 4 * math.pi / 1.5
    u = one.rad_w[0]
    assert abs(W[0, 0] - v00 / (1 - v00 * u * x00 * u)) < 1e-13 * v00
    assert np.abs(W[1:, 1:] - sc.coulomb(one)[1:, 1:]).max() < 1e-13


def test_W_push_through_and_screening_bound(tiny):
    w = tiny
    ps = w.psi_site.numpy()
    site = w.sites[0]
    chi = cz.chi0_exact(ps, ps, w.energies, w.nocc)
    W1 = sc.screen_W(chi, site)
    W2 = sc.screen_W_via_chi(chi, site)
    assert np.abs(W1 - W2).max() < 1e-12 * np.abs(W1).max()
    assert np.abs(W1 - W1.T).max() < 1e-12 * np.abs(W1).max()
    rho = w.rho_test
    Lw = sc.test_charge_loss(W1, rho, site)
    Lv = sc.test_charge_loss(sc.coulomb(site), rho, site)
    assert 0 < Lw <= Lv


def test_gaussian_self_energy_converges():
    """A unit Gaussian (sigma 0.5) at the site centre: rho^T D V D rho -> 1/(sigma sqrt(pi))."""
    sig = 0.5
    errs = []
    for nr in (40, 160):
        s = sx.make_site(np.zeros(3), nr, 26, r_max=4.0)
        r2 = (s.points() ** 2).sum(1)
        rho = (2 * math.pi * sig ** 2) ** -1.5 * np.exp(-r2 / (2 * sig ** 2))
        e = sc.test_charge_loss(sc.coulomb(s), rho, s)
        errs.append(abs(e - 1 / (sig * math.sqrt(math.pi))))
    assert errs[1] < errs[0] and errs[1] < 5e-3


# --------------------------------------------------------------------------- gradients
def test_reference_gradients_finite_differences():
    """Exact-denominator reference gradients vs central differences of the oracle loss
    (h = 1e-5 Ha for energies; a directional derivative for the orbitals)."""
    w = workload("tiny")
    nb = 40
    E = w.energies[:, :nb].copy()
    ps = w.psi_site.numpy()[:, :nb, :].copy()
    sites, rho, nocc = w.sites, w.rho_test, w.nocc
    kern = lambda EE: cz.exact_kernel(EE, nocc)
    L, dE, dpsi = gr.loss_and_grads(ps, E, nocc, 2, sites, rho, "exact")
    h = 1e-5
    for (k, b) in [(0, 0), (0, 5), (0, 7), (0, 8), (0, 20), (0, 39)]:
        Ep, Em = E.copy(), E.copy()
        Ep[k, b] += h
        Em[k, b] -= h
        fd = (gr.loss(ps, Ep, nocc, 2, sites, rho, kern(Ep))[0]
              - gr.loss(ps, Em, nocc, 2, sites, rho, kern(Em))[0]) / (2 * h)
        assert abs(fd - dE[k, b]) < 1e-6 * np.abs(dE).max() + 1e-9 * abs(L)
    rng = np.random.default_rng(5)
    Vd = rng.normal(size=ps.shape) + 1j * rng.normal(size=ps.shape)
    Vd /= np.abs(Vd).max()
    hp = 1e-5 * np.abs(ps).max()
    Lp = gr.loss(ps + hp * Vd, E, nocc, 2, sites, rho, kern(E))[0]
    Lm = gr.loss(ps - hp * Vd, E, nocc, 2, sites, rho, kern(E))[0]
    fd = (Lp - Lm) / (2 * hp)
    an = float(np.real(np.conj(dpsi) * Vd).sum())
    assert abs(fd - an) < 1e-6 * abs(an)


def test_quadrature_gradients_finite_differences():
    w = workload("tiny")
    nb = 40
    E = w.energies[:, :nb].copy()
    ps = w.psi_site.numpy()[:, :nb, :].copy()
    sites, rho, nocc = w.sites, w.rho_test, w.nocc
    n, scale = 16, 4.0

    def Lq(EE, pp):
        c, al, be = cz.terms_for(EE, nocc, "time", n, scale, mu=q.mid_gap(E, nocc))
        return gr.loss(pp, EE, nocc, 2, sites, rho, cz.quad_kernel(c, al, be))[0]
    L, dE, dpsi = gr.loss_and_grads(ps, E, nocc, 2, sites, rho, "time", n, scale)
    h = 1e-5
    for (k, b) in [(0, 1), (0, 7), (0, 8), (0, 30)]:
        Ep, Em = E.copy(), E.copy()
        Ep[k, b] += h
        Em[k, b] -= h
        fd = (Lq(Ep, ps) - Lq(Em, ps)) / (2 * h)
        assert abs(fd - dE[k, b]) < 1e-6 * np.abs(dE).max()


# ------------------------------------------------------------------ orbital projection
from oracle import project as pj  # noqa: E402


def _random_pw(rng, a, nmax, nb, nk=1):
    n = np.stack(np.meshgrid(*[np.arange(-nmax, nmax + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    gvec = n * (2 * np.pi / a)
    coef = rng.normal(size=(nk, nb, len(n))) + 1j * rng.normal(size=(nk, nb, len(n)))
    coef /= np.linalg.norm(coef, axis=2, keepdims=True)       # unit norm over the cell
    return n, gvec, coef


def test_projection_matches_inverse_fft_on_grid_points():
    """At the points of an N^3 grid, sum_G C(G) e^{i(k+G).x} is N^3 e^{ik.x} times the inverse
    FFT of C placed at G mod N (numpy.fft), for k off Gamma too."""
    rng = np.random.default_rng(31)
    a, N, nmax = 7.0, 12, 3
    n, gvec, coef = _random_pw(rng, a, nmax, nb=3, nk=2)
    kpts = np.array([[0.0, 0.0, 0.0], [0.5, -0.25, 0.5]]) * (2 * np.pi / a)
    j = np.stack(np.meshgrid(*[np.arange(N)] * 3, indexing="ij"), -1).reshape(-1, 3)
    x = j * (a / N)
    psi = pj.project(coef, kpts, gvec, x, a ** 3)
    for ik in range(2):
        for b in range(3):
            box = np.zeros((N, N, N), dtype=np.complex128)
            box[n[:, 0] % N, n[:, 1] % N, n[:, 2] % N] = coef[ik, b]
            ref = np.fft.ifftn(box).reshape(-1) * N ** 3 * np.exp(1j * (x @ kpts[ik]))
            ref /= np.sqrt(a ** 3)
            assert np.abs(psi[ik, b] - ref).max() < 1e-12 * np.abs(ref).max()


def test_projection_bloch_and_parseval():
    """psi(r + a e_d) = e^{i k_d a} psi(r) for each lattice direction, and the grid sum of
    |psi|^2 dV equals sum_G |C|^2 = 1 when the grid resolves every G."""
    rng = np.random.default_rng(32)
    a, nmax = 6.5, 2
    n, gvec, coef = _random_pw(rng, a, nmax, nb=2)
    k = np.array([0.3, -0.2, 0.45]) * (2 * np.pi / a)
    r = rng.uniform(-3, 9, size=(17, 3))
    psi = pj.project(coef, k[None], gvec, r, a ** 3)[0]
    for d in range(3):
        sh = r.copy()
        sh[:, d] += a
        psi_t = pj.project(coef, k[None], gvec, sh, a ** 3)[0]
        assert np.abs(psi_t - np.exp(1j * k[d] * a) * psi).max() < 1e-12
    N = 2 * nmax + 2
    j = np.stack(np.meshgrid(*[np.arange(N)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pg = pj.project(coef, k[None], gvec, j * (a / N), a ** 3)[0]
    norm = (np.abs(pg) ** 2).sum(1) * (a / N) ** 3
    assert np.abs(norm - 1.0).max() < 1e-12


def test_fft_route_exact_at_grid_points_and_cubic_weights():
    """The FFT route at the FFT grid's own points (weights 0, 1, 0, 0) equals the direct phase
    matrix sum to rounding, on a sheared (non-orthogonal) cell and off Gamma; the Lagrange
    weights sum to one and reproduce t, t^2, t^3."""
    rng = np.random.default_rng(41)
    cell = np.array([[6.0, 0.0, 0.0], [1.5, 5.5, 0.0], [0.5, -1.0, 6.5]])
    B = 2 * np.pi * np.linalg.inv(cell).T                      # reciprocal vectors (rows)
    n = np.stack(np.meshgrid(*[np.arange(-2, 3)] * 3, indexing="ij"), -1).reshape(-1, 3)
    gvec = n @ B
    coef = rng.normal(size=(2, 2, len(n))) + 1j * rng.normal(size=(2, 2, len(n)))
    kpts = np.array([[0.0, 0.0, 0.0], [0.25, -0.5, 0.125]]) @ B
    N = (10, 12, 9)
    j = rng.integers(0, 40, size=(15, 3))
    pts = (j / np.array(N)) @ cell
    omega = abs(np.linalg.det(cell))
    f = pj.project_fft(coef, kpts, cell, n, pts, omega, N)
    d = pj.project(coef, kpts, gvec, pts, omega)
    assert np.abs(f - d).max() < 1e-12 * np.abs(d).max()
    for t in (0.0, 0.3, 0.77):
        w = pj.lagrange_cubic(t)
        nodes = np.array([-1.0, 0.0, 1.0, 2.0])
        for p in range(4):
            assert abs((w * nodes ** p).sum() - t ** p) < 1e-14


def test_fft_route_within_derived_interpolation_bound():
    """At random points the FFT route differs from the direct sum by no more than the derived
    bound of the cubic tensor-product interpolation (oracle.project.interpolation_bound), the
    bound is tight within a factor of 30, and the error falls at least tenfold when the grid
    is oversampled twice as much (fourth-order interpolation)."""
    rng = np.random.default_rng(42)
    a, nmax = 7.0, 3
    n, gvec, coef = _random_pw(rng, a, nmax, nb=2, nk=1)
    cell = np.eye(3) * a
    k = np.array([[0.1, 0.2, -0.3]])
    pts = rng.uniform(-2, 9, size=(24, 3))
    d = pj.project(coef, k, gvec, pts, a ** 3)
    errs = []
    for N in (28, 56):
        f = pj.project_fft(coef, k, cell, n, pts, a ** 3, (N, N, N))
        for b in range(2):
            e = np.abs(f[0, b] - d[0, b]).max()
            bound = pj.interpolation_bound(coef[0, b], n, (N, N, N), a ** 3)
            assert e <= bound and bound < 30 * e
        errs.append(np.abs(f - d).max())
    assert errs[1] < errs[0] / 10


def test_projection_explicit_loops():
    """Two bands, a handful of plane waves and points, by explicit loops over G."""
    import cmath
    rng = np.random.default_rng(33)
    gvec = rng.normal(size=(5, 3))
    k = rng.normal(size=3) * 0.1
    pts = rng.normal(size=(3, 3)) * 2
    coef = rng.normal(size=(1, 2, 5)) + 1j * rng.normal(size=(1, 2, 5))
    omega = 11.0
    got = pj.project(coef, k[None], gvec, pts, omega)
    for b in range(2):
        for p in range(3):
            s = 0j
            for g in range(5):
                ph = sum((k[c] + gvec[g, c]) * pts[p, c] for c in range(3))
                s += coef[0, b, g] * cmath.exp(1j * ph)
            assert abs(got[0, b, p] - s / math.sqrt(omega)) < 1e-13


# ------------------------------------------------------------------ induced potential
def test_shell_partition_potential():
    """v1 + v2 = q / x (Eq. partition): v2 = q/R_S inside the shell, q/x outside."""
    r = np.array([0.1, 0.5, 1.0, 1.49, 1.5, 2.0, 3.7])
    q, rs = 1.3, 1.5
    v1 = sc.shell_potential(r, q, rs)
    v2 = np.where(r < rs, q / rs, q / r)
    assert np.abs(v1 + v2 - q / r).max() < 1e-14 * q / r.min()
    assert np.all(v1[r >= rs] == 0.0) and np.all(v1[r < rs] > 0.0)


def test_induced_pins(tiny):
    """Induced density and potential of a spherical perturbation:
    - no response (chi0 = 0) gives zero;
    - v1 + v_ind equals eps^-1 v1, solved with eps = I - V D X D instead of through chi;
    - a weak response agrees with the Dyson iteration rho = X D (v1 + V D rho);
    - v1^T D rho <= 0 (chi is negative semidefinite);
    - an isotropic chi0 responds in L = 00 only, where the l = 0 solve is exact."""
    w = tiny
    ps = w.psi_site.numpy()
    site = w.sites[0]
    chi = cz.chi0_exact(ps, ps, w.energies, w.nocc)
    v1 = sc.shell_potential(site.radii, 1.0, 1.2)
    n = (site.n_rad) * 9
    r0, z0 = sc.induced(np.zeros_like(chi), site, v1)
    assert np.abs(r0).max() == 0.0 and np.abs(z0).max() == 0.0
    rho, vind = sc.induced(chi, site, v1)
    X = sc.project(chi, site)
    V = sc.coulomb(site)
    D = np.diag(sc.radial_weights(site))
    v1vec = np.zeros(n)
    v1vec[:site.n_rad] = math.sqrt(4 * math.pi) * v1
    tot = np.linalg.solve(np.eye(n) - V @ D @ X @ D, v1vec)
    assert np.abs(v1vec + vind - tot).max() < 1e-12 * np.abs(tot).max()
    assert v1vec @ D @ rho <= 0.0
    # weak response: the Dyson series converges
    small = 0.05 * chi
    rs_, _ = sc.induced(small, site, v1)
    Xs = sc.project(small, site)
    it = np.zeros(n)
    for _ in range(200):
        it = Xs @ D @ (v1vec + V @ D @ it)
    assert np.abs(it - rs_).max() < 1e-12 * np.abs(rs_).max()
    # isotropic response: only L = 00
    rr = np.repeat(np.arange(site.n_rad), site.n_ang)
    iso = -0.2 * np.exp(-np.abs(rr[:, None] - rr[None, :]))
    full, vf = sc.induced(iso, site, v1)
    l0, vl0 = sc.induced(iso, site, v1, l0_only=True)
    assert np.abs(full[site.n_rad:]).max() < 1e-12 * np.abs(full).max()
    assert np.abs(full - l0).max() < 1e-12 * np.abs(full).max()
    assert np.abs(vf - vl0).max() < 1e-12 * np.abs(vf).max()


# ------------------------------------------------------------------ ALDA vertex
from oracle import alda as ax  # noqa: E402


def test_lda_exchange_kernel_closed_form():
    """The 5-point difference of the exchange energy n eps_x(n) against its closed-form
    second derivative -(1/3) (3/pi)^(1/3) n^(-2/3)."""
    n = np.array([0.2, 0.5, 1.0, 3.0])
    fd = ax.fxc(n, energy=lambda m: m * ax.eps_x(m))
    exact = -(1.0 / 3.0) * (3.0 / math.pi) ** (1 / 3) * n ** (-2 / 3)
    assert np.abs(fd / exact - 1).max() < 1e-5


def test_vwn_correlation_limits():
    """eps_c < 0 and rising to 0 at low density; d eps_c / d ln r_s -> A at high density (the
    form's logarithmic term)."""
    rs = np.array([0.5, 1.0, 2.0, 5.0, 10.0, 100.0, 1e4])
    n = 3.0 / (4.0 * math.pi * rs ** 3)
    ec = ax.eps_c(n)
    assert np.all(ec < 0) and np.all(np.diff(ec) > 0) and abs(ec[-1]) < 1e-3
    r1, r2 = 1e-10, 1e-9
    n1, n2 = 3.0 / (4.0 * math.pi * r1 ** 3), 3.0 / (4.0 * math.pi * r2 ** 3)
    slope = (ax.eps_c(n2) - ax.eps_c(n1)) / math.log(r2 / r1)
    assert abs(slope / ax.VWN_A - 1) < 1e-3


def test_fxc_difference_step_and_contact_matrix():
    """The 0.01 step agrees with a 0.001 step; for a constant f the contact matrix is f I
    (the Lebedev rule integrates products of l <= 2 harmonics exactly)."""
    n = np.array([0.2, 0.3, 1.0])
    assert np.abs(ax.fxc(n) / ax.fxc(n, h=1e-3) - 1).max() < 1e-5
    site = sx.make_site(np.zeros(3), 3, 26, r_max=2.0)
    F = ax.contact_matrix(site, np.full(site.npts, -0.7))
    assert np.abs(F + 0.7 * np.eye(F.shape[0])).max() < 1e-13


def test_alda_W_pins(tiny):
    """W~ through eps (I - (V D + F) X D) agrees with W~ through chi~; a zero kernel gives
    the RPA W back, and the density's kernel changes it."""
    w = tiny
    ps = w.psi_site.numpy()
    site = w.sites[0]
    chi = cz.chi0_exact(ps, ps, w.energies, w.nocc)
    from workloads import crystal as cx
    dens = cx.valence_density(w.psi_site, w.nocc).numpy()
    Wa = ax.screen_W_alda(chi, site, dens)
    X = sc.project(chi, site)
    V = sc.coulomb(site)
    d = sc.radial_weights(site)
    D = np.diag(d)
    F = ax.contact_matrix(site, ax.fxc(dens))
    n = V.shape[0]
    Y = np.linalg.solve(np.eye(n) - (V @ D + F) @ X @ D, V)
    Wb = V + V @ D @ X @ D @ Y
    assert np.abs(Wa - Wb).max() < 1e-11 * np.abs(Wa).max()
    W = sc.screen_W(chi, site)
    W0 = ax.screen_W_alda(chi, site, dens, f_points=np.zeros_like(dens))
    assert np.abs(W0 - W).max() < 1e-12 * np.abs(W).max()
    assert np.abs(Wa - W).max() > 1e-6 * np.abs(W).max()


# ------------------------------------------------------------------ chi0 at imaginary frequency
@pytest.mark.parametrize("d,om", [(0.05, 0.02), (0.3, 0.3), (1.7, 0.8), (0.2, 3.0)])
def test_iw_pair_identity(d, om):
    """int_0^inf cos(omega tau) exp(-Delta tau) d tau = Delta / (Delta^2 + omega^2)."""
    val, _ = integrate.quad(lambda t: math.cos(om * t) * math.exp(-d * t), 0, np.inf,
                            limit=400, epsabs=1e-14, epsrel=1e-13)
    assert abs(val - d / (d * d + om * om)) < 1e-11 * d / (d * d + om * om)


def test_chi0_iw_limits_and_symmetry(tiny):
    """omega = 0 gives the static chi0; omega^2 chi0(i omega) tends to the first-moment sum
    -(2s/N_k^2) sum Delta Re P; the odd part vanishes for the Gamma-only tiny workload (a
    real potential: a time-reversal-symmetric set with whole multiplets)."""
    w = tiny
    ps = w.psi_site.numpy()
    E = w.energies
    static = cz.chi0_exact(ps, ps, E, w.nocc)
    z, odd0 = cz.chi0_iw_exact(ps, ps, E, w.nocc, 0.0)
    assert np.abs(z - static).max() < 1e-13 * np.abs(static).max()
    om = 1e4
    big, _ = cz.chi0_iw_exact(ps, ps, E, w.nocc, om)
    mu = q.mid_gap(E, w.nocc)
    x, y = q.offsets(E, w.nocc, mu)
    first = cz.pair_sum(ps, ps, w.nocc, 2, lambda k, kp: x[k][:, None] + y[kp][None, :])[0]
    assert np.abs(om * om * big - first).max() < 1e-7 * np.abs(first).max()
    _, odd = cz.chi0_iw_exact(ps, ps, E, w.nocc, 0.3)
    assert odd < 1e-14 * np.abs(static).max()


def test_iw_time_rule_converges(tiny):
    """The cos-weighted imaginary-time rule approaches chi0(i omega) as nodes are added (its
    accuracy falls as omega tau oscillates faster: small omega only)."""
    w = tiny
    ps = w.psi_site.numpy()
    E = w.energies
    ex, _ = cz.chi0_iw_exact(ps, ps, E, w.nocc, 0.2)
    errs = []
    for n in (16, 32, 48):
        cc, cs, al, be = cz.terms_for(E, w.nocc, "time_iw:0.2", n)
        got = cz.chi0_iw_quad(ps, ps, w.nocc, 2, cc, cs, al, be)
        errs.append(np.abs(got - ex).max() / np.abs(ex).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6


def test_iw_odd_part_with_split_band_sets():
    """Where the band cut splits a degenerate multiplet (production cell, 2x2x2 k) the odd
    part is not zero; the sin-weighted terms reproduce it: the quadrature chi0(i omega)
    approaches the exact one, odd part included, and is not symmetric."""
    p = workload("production", with_grid=False)
    pp = p.psi_site.numpy()[:, :, :120]
    ex, odd = cz.chi0_iw_exact(pp, pp, p.energies, p.nocc, 0.05)
    assert odd > 1e-5 * np.abs(ex).max()
    cc, cs, al, be = cz.terms_for(p.energies, p.nocc, "time_iw:0.05", 48)
    got = cz.chi0_iw_quad(pp, pp, p.nocc, 2, cc, cs, al, be)
    assert np.abs(got - ex).max() < 1e-6 * np.abs(ex).max()
    assert np.abs(got - got.T).max() > 1e-6 * np.abs(got).max()


def test_iw_entries_match_blocks(tiny):
    """The per-entry imaginary-frequency sum equals the block sum at those entries."""
    w = tiny
    ps = w.psi_site.numpy()
    cc, cs, al, be = cz.terms_for(w.energies, w.nocc, "time_iw:0.3", 24)
    blk = cz.chi0_iw_quad(ps, ps, w.nocc, 2, cc, cs, al, be)
    rng = np.random.default_rng(5)
    r = rng.integers(0, ps.shape[2], 40)
    c = rng.integers(0, ps.shape[2], 40)
    ent = cz.chi0_iw_quad_entries(ps[:, :, r], ps[:, :, c], w.nocc, 2, cc, cs, al, be)
    assert np.abs(ent - blk[r, c]).max() < 1e-13 * np.abs(blk).max()


def test_iw_exact_entries_match_blocks():
    """The per-entry exact imaginary-frequency sum equals the block sum at those entries, on
    the production cell where the odd part is not zero (entries and their transposes)."""
    p = workload("production", with_grid=False)
    pp = p.psi_site.numpy()[:, :, :120]
    ex, odd = cz.chi0_iw_exact(pp, pp, p.energies, p.nocc, 0.05)
    assert odd > 1e-5 * np.abs(ex).max()
    rng = np.random.default_rng(6)
    r = rng.integers(0, 120, 30)
    c = rng.integers(0, 120, 30)
    rr, cc = np.concatenate([r, c]), np.concatenate([c, r])
    ent = cz.chi0_iw_exact_entries(pp[:, :, rr], pp[:, :, cc], p.energies, p.nocc, 0.05)
    assert np.abs(ent - ex[rr, cc]).max() < 1e-13 * np.abs(ex).max()
    assert np.abs(ent[:30] - ent[30:]).max() > 1e-6 * np.abs(ex).max()


def test_iw_linear_gradient_central_differences():
    """The reference gradient of L = sum Lambda chi0(i omega) (arbitrary, non-symmetric Lambda;
    complex term coefficients) against central differences of the oracle's own chi0(i omega)
    in the energies and along random complex orbital directions."""
    from workloads import sites as sx
    rng = np.random.default_rng(8)
    nk, nb, nocc, n, omega = 2, 10, 3, 24, 0.3
    sites = [sx.make_site(np.zeros(3), 2, 6), sx.make_site(np.ones(3), 1, 6)]
    npts = sum(s.npts for s in sites)
    ps = rng.standard_normal((nk, nb, npts)) + 1j * rng.standard_normal((nk, nb, npts))
    E = np.sort(rng.uniform(-1, 1, (nk, nb)), axis=1)
    E[:, nocc:] += 0.5
    lam = [rng.standard_normal((s.npts, s.npts)) for s in sites]
    mu = q.mid_gap(E, nocc)
    x, y = q.offsets(E, nocc, mu)
    scale = q.auto_scale_iw(x, y, n, omega)
    L, dE, dpsi = gr.linear_grads_iw(ps, E, nocc, 2, sites, lam, n, scale, omega, mu)

    def Lf(pp, EE):
        cc, cs, al, be, _ = gr.iw_terms(EE, nocc, n, scale, omega, mu)
        return gr.linear_loss_iw(pp, nocc, 2, sites, lam, cc, cs, al, be)
    assert abs(L - Lf(ps, E)) < 1e-12 * abs(L)
    h = 1e-6
    for k in range(nk):
        for b in range(nb):
            Ep, Em = E.copy(), E.copy()
            Ep[k, b] += h
            Em[k, b] -= h
            fd = (Lf(ps, Ep) - Lf(ps, Em)) / (2 * h)
            assert abs(fd - dE[k, b]) < 1e-6 * np.abs(dE).max()
    for _ in range(3):
        V = rng.standard_normal(ps.shape) + 1j * rng.standard_normal(ps.shape)
        fd = (Lf(ps + h * V, E) - Lf(ps - h * V, E)) / (2 * h)
        an = float((np.conj(dpsi) * V).real.sum())
        assert abs(fd - an) < 1e-6 * abs(an)


def test_iw_gradient_at_zero_frequency_is_the_static_loss_gradient():
    """Two independently written reference gradients agree: the imaginary-frequency gradient of
    sum Lambda chi0 at omega = 0, with Lambda = g g^T the sensitivity of the test-charge loss,
    equals the static test-charge-loss gradient (same nodes)."""
    w = workload("tiny")
    nb = 40
    E = w.energies[:, :nb].copy()
    ps = w.psi_site.numpy()[:, :nb, :].copy()
    sites, rho, nocc = w.sites, w.rho_test, w.nocc
    n, scale = 16, 4.0
    _, dE, dpsi = gr.loss_and_grads(ps, E, nocc, 2, sites, rho, "time", n, scale)
    c, al, be = cz.terms_for(E, nocc, "time", n, scale)
    lams = []
    for s, sl in zip(sites, gr.site_slices(sites)):
        chi = cz.chi0_quad(ps[:, :, sl], ps[:, :, sl], nocc, 2, c, al, be)
        W = sc.screen_W(chi, s)
        d = sc.radial_weights(s)
        g = sc.projector(s).T @ (d * (0.5 * (W + W.T) @ (d * sc.charge_moments(rho[sl], s))))
        lams.append(np.outer(g, g))
    _, dE0, dpsi0 = gr.linear_grads_iw(ps, E, nocc, 2, sites, lams, n, scale, 0.0)
    assert np.abs(dE0 - dE).max() < 1e-12 * np.abs(dE).max()
    assert np.abs(dpsi0 - dpsi).max() < 1e-12 * np.abs(dpsi).max()
