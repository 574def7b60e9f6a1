"""More pins of the CPU oracle: the l = 1, 2 Coulomb blocks, the chemical potential and the
frequency-rule scale, and the metallic regularisation of Sec. VI.D.

Each check compares the oracle with something computed another way: the potential of a
Gaussian multipole charge in closed form (Hobson's formula), hand-computed values of the
paper's rules for mu and zeta, adaptive integration of the regularised per-pair integrand of
Eq. chi1, brute-force loops over band pairs, and central differences.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erf

from oracle import chi0 as cz
from oracle import grads as gr
from oracle import quadrature as q
from oracle import screen as sc
from tests.conftest import workload
from workloads import sites as sx


# ------------------------------------------------------------------- Coulomb multipoles
def _d_pow(f, l, r, h):
    """(D^l f)(r) with D = (1/r) d/dr, by nested central differences (step h)."""
    if l == 0:
        return f(r)
    return (_d_pow(f, l - 1, r + h, h) - _d_pow(f, l - 1, r - h, h)) / (2 * h * r)


def _gauss_potential_d(r, sig, l):
    """(D^l phi)(r) for phi(r) = erf(r / (sig sqrt 2)) / r, the potential of a unit Gaussian
    charge of width sig, in closed form (D = (1/r) d/dr)."""
    a = 1.0 / (sig * math.sqrt(2.0))
    e = erf(a * r)
    g = 2.0 * a / math.sqrt(math.pi) * np.exp(-a * a * r * r)
    if l == 0:
        return e / r
    if l == 1:
        return g / r ** 2 - e / r ** 3
    if l == 2:
        return g * (-2.0 * a * a / r ** 2 - 3.0 / r ** 4) + 3.0 * e / r ** 5
    raise ValueError(l)


def test_gaussian_potential_closed_forms():
    """The closed forms of D^l phi used below, against nested central differences of phi."""
    sig = 0.5
    r = np.linspace(0.3, 3.0, 13)
    phi = lambda x: erf(x / (sig * math.sqrt(2.0))) / x
    for l in (1, 2):
        fd = _d_pow(phi, l, r, 1e-3)
        ex = _gauss_potential_d(r, sig, l)
        assert np.abs(fd - ex).max() < 1e-5 * np.abs(ex).max()


def test_coulomb_blocks_against_gaussian_multipoles():
    """Every channel L = (l, m), l <= 2, of the Coulomb matrix against an exact potential.

    For a harmonic homogeneous polynomial h of degree l, h(grad) F(r) = h(x) (D^l F)(r)
    (Hobson).  The charge rho = h_L(grad) g, with g a unit Gaussian and h_L(x) = r^l Y_L(x/r),
    is therefore r^l Y_L (-1/sig^2)^l g(r), and its potential is h_L(grad) phi =
    r^l Y_L (D^l phi)(r).  The oracle's V D (P rho) on a fine radial grid must give the Y_L
    coefficient r^l D^l phi(r); a wrong 4 pi/(2l+1) or a wrong power of r in any block fails
    by a factor of order one."""
    sig = 0.5
    site = sx.make_site(np.zeros(3), 400, 26, r_max=5.0)
    pts = site.points()
    r = np.sqrt((pts ** 2).sum(1))
    Y = sc.real_ylm(pts / r[:, None], 2)                        # [9, npts]
    g = (2 * math.pi * sig ** 2) ** -1.5 * np.exp(-r * r / (2 * sig * sig))
    V = sc.coulomb(site, 2)
    d = sc.radial_weights(site, 2)
    nr = site.n_rad
    rr = site.radii
    inner = rr < 3.0        # away from the truncation of the radial range
    for l in range(3):
        for m in range(-l, l + 1):
            L = l * l + l + m
            rho = r ** l * Y[L] * (-1.0 / sig ** 2) ** l * g
            rl = sc.charge_moments(rho, site, 2)
            v = V @ (d * rl)
            ref = rr ** l * _gauss_potential_d(rr, sig, l)
            got = v[L * nr:(L + 1) * nr]
            err = np.abs(got[inner] - ref[inner]).max() / np.abs(ref[inner]).max()
            assert err < 2e-3, (l, m, err)
            # the other channels receive nothing
            others = np.delete(v, np.s_[L * nr:(L + 1) * nr])
            assert np.abs(others).max() < 1e-10 * np.abs(got).max()


def test_multipole_self_energy_through_the_loss():
    """rho^T D V D rho (the test-charge loss with W = V) for the l = 1 and l = 2 Gaussian
    multipoles against the electrostatic self-energy int rho phi, computed as a radial integral
    of the closed forms by adaptive quadrature."""
    sig = 0.5
    site = sx.make_site(np.zeros(3), 400, 26, r_max=5.0)
    pts = site.points()
    r = np.sqrt((pts ** 2).sum(1))
    Y = sc.real_ylm(pts / r[:, None], 2)
    g = (2 * math.pi * sig ** 2) ** -1.5 * np.exp(-r * r / (2 * sig * sig))
    V = sc.coulomb(site, 2)
    for l, L in ((1, 2), (2, 6)):
        rho = r ** l * Y[L] * (-1.0 / sig ** 2) ** l * g
        got = sc.test_charge_loss(V, rho, site, 2)

        def integrand(x):
            gx = (2 * math.pi * sig ** 2) ** -1.5 * math.exp(-x * x / (2 * sig * sig))
            return x ** 2 * (x ** l * (-1.0 / sig ** 2) ** l * gx) * x ** l * float(
                _gauss_potential_d(np.array([x]), sig, l)[0])
        ref = integrate.quad(integrand, 1e-6, 8.0, epsabs=0, epsrel=1e-11, limit=400)[0]
        assert abs(got - ref) < 3e-3 * abs(ref), (l, got, ref)


# ------------------------------------------------------------- mu and the frequency scale
def test_mid_gap_and_zeta_hand_values():
    """mu is the middle of the global gap over all k (the top occupied and the bottom
    unoccupied level may sit at different k), and the frequency rule's zeta is the geometric
    mean of the smallest and largest |mu - e|, i.e. of half the gap and the larger distance to
    the band bottom or top; metals add 0.5 eV in quadrature to the smallest."""
    E = np.array([[-3.0, -0.2, 0.5, 2.0],
                  [-2.5, -0.6, 0.1, 2.2]])
    mu = q.mid_gap(E, 2)
    assert mu == pytest.approx((-0.2 + 0.1) / 2, abs=1e-15)      # top at k0, bottom at k1
    half_gap = 0.15
    far = max(mu - (-3.0), 2.2 - mu)                                # bottom is farther: 2.95
    assert q.zeta(E, mu) == pytest.approx(math.sqrt(half_gap * far), rel=1e-14)
    ev = 0.5 / 27.211386245988
    assert q.zeta(E, mu, metallic=True) == pytest.approx(
        math.sqrt(math.sqrt(half_gap ** 2 + ev ** 2) * far), rel=1e-14)
    # mirror image: reflecting the spectrum swaps which side is farther
    Er = -E[:, ::-1]
    assert q.mid_gap(Er, 2) == pytest.approx(-mu, abs=1e-15)
    assert q.zeta(Er, -mu) == pytest.approx(q.zeta(E, mu), rel=1e-14)


# ---------------------------------------------------------------- metallic regularisation
def _pair_integral(xb, xbp):
    """(1/2 pi) int dt Re[1 / ((xb + i t)(xbp + i t))] over the real line: the energy integral
    of Eq. chi1 for one band pair with offsets xb = mu - e_b, xbp = mu - e_b' (adaptive
    quadrature; the integrand is even in t after the real part)."""
    f = lambda t: ((xb * xbp - t * t) / ((xb * xb + t * t) * (xbp * xbp + t * t)))
    return integrate.quad(f, 0, np.inf, epsabs=0, epsrel=1e-12, limit=500)[0] / math.pi


@pytest.mark.parametrize("e1,e2", [(-0.3, 0.2), (-0.01, 0.02), (-0.4, -0.1), (0.05, 0.3)])
def test_regularised_pair_integral_keeps_the_sides(e1, e2):
    """With (mu - e) -> +-sqrt((mu - e)^2 + delta^2) (Sec. VI.D) a pair across mu integrates to
    -1/(X + Y) with X, Y the regularised distances (what the oracle's kernel uses), and a pair
    on one side to zero, as without regularisation.  With the sign dropped every offset would be
    positive and pairs across mu would vanish too."""
    mu, delta = 0.0, 0.03
    xb = q.regularised(np.array(mu - e1), delta)
    xbp = q.regularised(np.array(mu - e2), delta)
    val = _pair_integral(float(xb), float(xbp))
    if (mu - e1) * (mu - e2) < 0:
        E = np.array([[e1, e2]])
        X, Yv = q.offsets(E, 1, mu, delta)
        assert val == pytest.approx(-1.0 / (X[0, 0] + Yv[0, 0]), rel=1e-9)
        assert X[0, 0] == pytest.approx(math.hypot(mu - e1, delta), rel=1e-15)
        # with the sign dropped both offsets are positive and the pair would vanish
        xa, xbp_a = math.hypot(mu - e1, delta), math.hypot(mu - e2, delta)
        assert abs(_pair_integral(xa, xbp_a)) < 1e-10
    else:
        assert abs(val) < 1e-10


def test_regularised_chi0_by_brute_force_and_limit():
    """chi0 with delta > 0 on a small two-k band set: the oracle's pair sum against explicit
    loops over every band pair (occupied or not) with the adaptively integrated regularised
    per-pair factor, and the delta -> 0 limit against the unregularised sum."""
    rng = np.random.default_rng(7)
    nk, nb, nocc, npt = 2, 6, 2, 5
    E = np.sort(rng.uniform(-0.5, 0.5, size=(nk, nb)), axis=1)
    E[:, nocc:] += 0.3 - E[:, nocc:].min() + E[:, :nocc].max()      # a gap of 0.3
    psi = rng.normal(size=(nk, nb, npt)) + 1j * rng.normal(size=(nk, nb, npt))
    mu = q.mid_gap(E, nocc)
    delta = 0.07
    got = cz.chi0_exact(psi, psi, E, nocc, spin=2, mu=mu, delta=delta)
    ref = np.zeros((npt, npt))
    for k in range(nk):
        for kp in range(nk):
            for b in range(nb):
                for bp in range(nb):
                    xb = float(q.regularised(np.array(mu - E[k, b]), delta))
                    xbp = float(q.regularised(np.array(mu - E[kp, bp]), delta))
                    if xb * xbp > 0:
                        assert abs(_pair_integral(xb, xbp)) < 1e-10
                        continue
                    if xb < 0:
                        continue                     # each pair once: b below mu, b' above
                    f = _pair_integral(xb, xbp)      # = -1/(X + Y)
                    P = (np.conj(psi[k, b])[:, None] * psi[kp, bp][:, None]
                         * np.conj(psi[kp, bp])[None, :] * psi[k, b][None, :])
                    # (spin 2) the two orderings of the pair give P and conj(P): 2 Re P
                    ref += 2 * 2.0 / nk ** 2 * (f * P).real
    assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max()
    small = cz.chi0_exact(psi, psi, E, nocc, spin=2, mu=mu, delta=1e-7)
    plain = cz.chi0_exact(psi, psi, E, nocc, spin=2, mu=mu)
    assert np.abs(small - plain).max() < 1e-9 * np.abs(plain).max()
    assert np.abs(got - plain).max() > 1e-3 * np.abs(plain).max()    # delta matters here


def test_regularised_time_rule_converges(tiny):
    """The imaginary-time rule with regularised offsets converges to the regularised exact sum
    (tiny workload, site x site)."""
    w = tiny
    ps = w.psi_site.numpy()
    mu = q.mid_gap(w.energies, w.nocc)
    delta = 0.02
    ex = cz.chi0_exact(ps, ps, w.energies, w.nocc, mu=mu, delta=delta)
    errs = []
    for n in (16, 32):
        terms = cz.terms_for(w.energies, w.nocc, "time", n, None, mu, delta)
        qq = cz.chi0_quad(ps, ps, w.nocc, 2, *terms)
        errs.append(np.abs(qq - ex).max() / np.abs(ex).max())
    assert errs[1] < errs[0] and errs[1] < 1e-9


def test_band_on_the_wrong_side_is_refused():
    """The lowest nocc bands are occupied at every k; a band set in which one of them lies above
    mu (or an unoccupied one below) would need k-dependent occupation: refused."""
    E = np.array([[-0.5, 0.2, 0.4], [-0.4, -0.1, 0.5]])     # band 1 at k1 lies below band 1...
    with pytest.raises(ValueError):
        q.offsets(E, 1, 0.0, 0.05)                           # e[1,1] = -0.1 < mu, unoccupied
    with pytest.raises(ValueError):
        q.offsets(E, 2, 0.0, 0.0)                            # e[0,1] = 0.2 > mu, occupied
    x, y = q.offsets(E, 1, -0.2, 0.05)
    assert x.min() > 0 and y.min() > 0


def test_regularised_gradients_finite_differences():
    """Gradients of the test-charge loss with delta > 0 (exact and imaginary-time kernels, mu
    held at the unperturbed mid-gap value) against central differences."""
    w = workload("tiny")
    nb = 40
    E = w.energies[:, :nb].copy()
    ps = w.psi_site.numpy()[:, :nb, :].copy()
    sites, rho, nocc = w.sites, w.rho_test, w.nocc
    mu = q.mid_gap(E, nocc)
    delta, n, scale = 0.03, 16, 4.0

    def L_of(EE, kind):
        if kind == "exact":
            kern = cz.exact_kernel(EE, nocc, mu, delta)
        else:
            kern = cz.quad_kernel(*cz.terms_for(EE, nocc, "time", n, scale, mu, delta))
        return gr.loss(ps, EE, nocc, 2, sites, rho, kern)[0]

    for kind in ("exact", "time"):
        _, dE, _ = gr.loss_and_grads(ps, E, nocc, 2, sites, rho, kind, n, scale, delta=delta)
        h = 1e-5
        for (k, b) in [(0, 0), (0, 7), (0, 8), (0, 25)]:
            Ep, Em = E.copy(), E.copy()
            Ep[k, b] += h
            Em[k, b] -= h
            fd = (L_of(Ep, kind) - L_of(Em, kind)) / (2 * h)
            assert abs(fd - dE[k, b]) < 1e-6 * np.abs(dE).max(), (kind, k, b)


# ---------------------------------------------------------------- valence W(x, x') in r_m
from oracle import valence as va  # noqa: E402


def test_sphere_potential_and_self_term_by_quadrature():
    """The uniformly charged sphere's potential against the radial Coulomb integral of its
    density (adaptive quadrature), and its average over the sphere against 6 / (5 R)."""
    R = 0.4
    rho = 3.0 / (4.0 * math.pi * R ** 3)
    for r in (0.05, 0.2, 0.39, 0.41, 1.3):
        ref = integrate.quad(lambda s: 4 * math.pi * s * s * rho / max(r, s), 0, R,
                             points=[min(r, R)], epsabs=0, epsrel=1e-12)[0]
        assert float(va.sphere_potential(np.array(r), R)) == pytest.approx(ref, rel=1e-10)
    avg = 3 / R ** 3 * integrate.quad(lambda s: float(va.sphere_potential(np.array(s), R)) * s * s,
                                      0, R, epsabs=0, epsrel=1e-13)[0]
    assert avg == pytest.approx(6 / (5 * R), rel=1e-12)


def test_lagrange4_exact_for_cubics():
    rng = np.random.default_rng(3)
    xs = np.sort(rng.uniform(0.1, 3.0, 12))
    c = rng.normal(size=4)
    f = lambda x: c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3
    for x in (0.0, 0.05, 0.7, 1.9, 2.999, 3.4):        # inside and extrapolated at both ends
        assert va.lagrange4(xs, f(xs), x) == pytest.approx(f(x), rel=1e-10, abs=1e-10)


def _valence_sites(nsites=8, spacing=0.625, n_rad=16, n_ang=26, seed=2):
    rng = np.random.default_rng(seed)
    base = np.array([[i, j, k] for i in range(2) for j in range(2) for k in range(2)], float)
    centres = base[:nsites] * spacing + rng.uniform(-0.01, 0.01, (nsites, 3))
    sites = [sx.make_site(c, n_rad, n_ang, r_max=2.0, r_min=0.05) for c in centres]
    return centres, sites


def test_valence_W_bare_limits():
    """chi0 = 0: W(x, x') is the bare potential of the neighbouring sphere's unit charge,
    1/|x - x'| (|x - x'| > R_x), reduced by (1 - 1/eps_inf) times the shell's v2 (1/R_S inside
    the shell); the diagonal is 6/(5 R_x) less the same constant; zero beyond r_m; symmetric."""
    centres, sites = _valence_sites()
    zero = [np.zeros((s.npts, s.npts)) for s in sites]
    vx, R_S = 0.244, 1.5
    R_x = (3 * vx / (4 * math.pi)) ** (1 / 3)
    for eps_inf in (1.0, 2.5):
        W = va.valence_W(zero, sites, centres, vx, R_S, eps_inf, r_m=1.0)
        c = (1 - 1 / eps_inf) / R_S
        for a in range(len(sites)):
            assert W[a, a] == pytest.approx(6 / (5 * R_x) - c, rel=1e-12)
            for b in range(len(sites)):
                if a == b:
                    continue
                d = np.linalg.norm(centres[b] - centres[a])
                ref = 1 / d - c if d <= 1.0 else 0.0
                assert W[a, b] == pytest.approx(ref, rel=1e-12, abs=1e-15)
        assert np.array_equal(W, W.T)


def test_valence_W_periodic_images_and_screening():
    """Sites across the cell boundary meet through the nearest image; with NSD chi0-like blocks
    the induced potential lowers W(x, x') below the bare value at every pair within r_m (a
    positive charge attracts the responding electrons), and the diagonal below 6/(5 R_x)."""
    from workloads import blocks as bx
    a = 4.0
    centres = np.array([[0.2, 0.2, 0.2], [3.8, 0.2, 0.2], [0.2, 3.9, 0.3], [0.9, 0.3, 0.2]])
    sites = [sx.make_site(c, 16, 26, r_max=2.0, r_min=0.05) for c in centres]
    blocks, _ = bx.chi0_like_blocks(sites, seed=5)
    cell = np.eye(3) * a
    vx, R_S = 0.05, 1.5                 # R_x = 0.23 bohr, below every pair distance
    R_x = (3 * vx / (4 * math.pi)) ** (1 / 3)
    W = va.valence_W(blocks, sites, centres, vx, R_S, 1.0, r_m=1.0, cell=cell)
    zero = [np.zeros_like(b) for b in blocks]
    W0 = va.valence_W(zero, sites, centres, vx, R_S, 1.0, r_m=1.0, cell=cell)
    assert W0[0, 1] == pytest.approx(1 / 0.4, rel=1e-12)          # through the x boundary
    assert W0[0, 2] == pytest.approx(1 / math.sqrt(0.3 ** 2 + 0.1 ** 2), rel=1e-12)
    assert W0[1, 3] == 0.0                                       # 1.10 bohr > r_m apart
    pairs = W0 != 0
    assert np.all(W[pairs] < W0[pairs])
    assert np.all(np.diag(W) < 6 / (5 * R_x))
    assert np.array_equal(W, W.T)
