"""GPU parity of chi0 from real orbitals at the Gamma point (Sec. VI.F; lrs_set_orbitals_real).

The synthetic crystals have a real potential, so their Gamma orbitals can be made real: a phase
per band and a real basis of each degenerate set (a unitary change within the set, which leaves
chi0 unchanged, since a set's orbitals carry equal weights).  The tests make them real
(`workloads.realify`, on the device), then compare the library's real-orbital chi0 (FP64 and F16F8)
with the oracle's band-pair sum on the same real orbitals, and with the library's complex path
on the original orbitals.  Error measure: max |gpu - ref| / max |ref|.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import chi0 as cz
from oracle import grads as gr
from oracle import quadrature as q
from tests.conftest import workload
from workloads.realify import realify

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_07834_amd as P
    return P


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def oracle_scale(E, nocc, n):
    mu = q.mid_gap(E, nocc)
    x, y = q.offsets(E, nocc, mu)
    return q.auto_scale(x, y, n)


@pytest.fixture(scope="module")
def tiny_real():
    w = workload("tiny")
    E = w.energies[0]
    (g, s), left = realify(w.energies, [w.psi_grid.to("cuda"), w.psi_site.to("cuda")])
    return dict(w=w, E=E, g=g[0], s=s[0], left=left)


def test_real_orbitals_tiny(P, tiny_real):
    """Tiny workload (Gamma): FP64 and F16F8 chi0 from the real orbitals on the grid and on the
    site block against the oracle with the same real orbitals and terms, and the FP64 result
    against the complex path on the original orbitals (equal to rounding); refusals."""
    T = tiny_real
    w, E = T["w"], T["E"]
    say(f"tiny real orbitals: imaginary part left {T['left']:.1e}")
    assert T["left"] < 1e-12
    n = w.n_terms
    s = oracle_scale(w.energies, w.nocc, n)
    ctx = P.Context(0)
    ctx.set_orbitals_real(E, w.nocc, T["g"], w.grid_dV)
    ctx.set_sites(w.sites, T["s"][None])
    ctx.make_quadrature(P.QUAD_TIME, n, s)
    gr_ = T["g"].cpu().numpy()[None].astype(np.complex128)
    sr_ = T["s"].cpu().numpy()[None].astype(np.complex128)
    terms = cz.terms_for(w.energies, w.nocc, "time", n, s)
    ref_g = cz.chi0_quad(sr_, gr_, w.nocc, 2, *terms)
    ref_s = cz.chi0_quad(sr_, sr_, w.nocc, 2, *terms)
    c2 = P.Context(0)
    c2.set_orbitals(w.energies, w.nocc, w.psi_grid, w.grid_dV)
    c2.set_sites(w.sites, w.psi_site)
    c2.make_quadrature(P.QUAD_TIME, n, s)
    cplx = c2.chi0(-1, P.COLS_GRID, P.FP64).cpu().numpy()
    c2.close()
    for prec, tol in (("fp64", 1e-12), ("f16f8", 1e-4)):
        g = ctx.chi0(-1, P.COLS_GRID, prec).cpu().numpy()
        sb = ctx.site_blocks(ctx.chi0(-1, P.COLS_SITE, prec))[0].cpu().numpy()
        eg, es = rel(g, ref_g), rel(sb, ref_s)
        say(f"  {prec}: grid {eg:.2e} site {es:.2e} vs oracle")
        assert eg < tol and es < tol
        if prec == "fp64":
            ec = rel(g, cplx)
            say(f"  fp64 real vs complex orbitals: {ec:.2e}")
            assert ec < 1e-12
    # imaginary frequency: the odd part of chi0 vanishes for real orbitals
    omega = 0.7
    ctx.make_quadrature_iw(32, 0.0, omega)
    sc = ctx.get_quadrature()["scale"]
    cc, cs, al, be = cz.terms_for(w.energies, w.nocc, f"time_iw:{omega}", 32, sc)
    ref_iw = cz.chi0_iw_quad(sr_, gr_, w.nocc, 2, cc, cs, al, be)
    for prec, tol in (("fp64", 1e-12), ("f16f8", 1e-4)):
        e = rel(ctx.chi0(-1, P.COLS_GRID, prec).cpu().numpy(), ref_iw)
        say(f"  {prec} at i omega = {omega} i: grid {e:.2e} vs oracle")
        assert e < tol
    for bad in ("bf16x2", "fp32"):
        with pytest.raises(P.LrsError) as e:
            ctx.chi0(-1, P.COLS_GRID, bad)
        assert e.value.status == P.LRS_EUNSUPPORTED
    with pytest.raises(P.LrsError) as e:
        ctx.chi0_backward(torch.zeros(w.nrows ** 2, dtype=torch.float64, device="cuda"),
                          P.FP64)
    assert e.value.status == P.LRS_EUNSUPPORTED
    with pytest.raises(P.LrsError) as e:
        ctx.set_sites(w.sites, w.psi_site)              # complex site orbitals
    assert e.value.status == P.LRS_EINVAL
    c3 = P.Context(0)
    with pytest.raises(P.LrsError) as e:
        c3.set_orbitals_real(E, w.nocc, w.psi_grid[0], w.grid_dV)   # complex grid orbitals
    assert e.value.status == P.LRS_EINVAL
    c3.close()
    ctx.close()


def test_real_orbitals_adjoint_tiny(P, tiny_real):
    """The adjoint with real orbitals (tiny workload, Gamma): dL/dE and dL/dpsi of the
    test-charge loss from the F16F8 path, which takes its Green's functions from the forward
    site-block call, against the oracle's gradient on the same real orbitals (whose imaginary
    parts vanish, as the library's do); refused before any Green's functions were kept."""
    T = tiny_real
    w = T["w"]
    n = w.n_terms
    s = oracle_scale(w.energies, w.nocc, n)
    ctx = P.Context(0)
    ctx.set_orbitals_real(T["E"], w.nocc, T["g"], w.grid_dV)
    ctx.set_sites(w.sites, T["s"][None])
    ctx.make_quadrature(P.QUAD_TIME, n, s)
    with pytest.raises(P.LrsError) as e:
        ctx.chi0_backward(torch.zeros(w.nrows ** 2, dtype=torch.float64, device="cuda"),
                          P.F16F8)
    assert e.value.status == P.LRS_EUNSUPPORTED
    chi = ctx.chi0(-1, P.COLS_SITE, P.F16F8)
    ctx.screen_W(chi, rho=torch.as_tensor(w.rho_test, device="cuda"), want_loss=True)
    lam = ctx.screen_W_backward()
    dE, dpsi = ctx.chi0_backward(lam, P.F16F8)
    sr = T["s"].cpu().numpy()[None].astype(np.complex128)
    _, dE_ref, dp_ref = gr.loss_and_grads(sr, w.energies, w.nocc, 2, w.sites, w.rho_test,
                                          "time", n, s)
    eE = rel(dE.cpu().numpy(), dE_ref)
    ep = rel(dpsi.real.cpu().numpy(), dp_ref.real)
    say(f"real-orbital adjoint (f16f8): dE {eE:.2e} dpsi {ep:.2e} vs oracle; max |Im| "
        f"{float(dpsi.imag.abs().max()):.1e} (oracle {np.abs(dp_ref.imag).max():.1e})")
    assert eE < 1e-4 and ep < 1e-4
    assert float(dpsi.imag.abs().max()) == 0.0 and np.abs(dp_ref.imag).max() == 0.0
    ctx.close()


def test_real_orbitals_precision_gamma(P):
    """Precision workload at Gamma (2304 bands, 3520 site rows x 110,592 grid columns, 32
    terms): the site x grid launch from real orbitals in FP64 and F16F8, sampled against the
    oracle on the real orbitals, and timed beside the complex launch of each precision."""
    from workloads import configs
    w = configs.precision(device="cuda", gamma_only=True)
    E = w.energies[0]
    (g, s), left = realify(w.energies, [w.psi_grid, w.psi_site])
    g, s = g[0], s[0]
    say(f"precision at Gamma: real orbitals, imaginary part left {left:.1e}")
    assert left < 1e-10
    n = w.n_terms
    rng = np.random.default_rng(9)
    rows = rng.integers(0, w.nrows, 48)
    cols = rng.integers(0, w.ngrid ** 3, 48)
    ps = s[:, torch.as_tensor(rows, device="cuda")].cpu().numpy()[None].astype(np.complex128)
    pg = g[:, torch.as_tensor(cols, device="cuda")].cpu().numpy()[None].astype(np.complex128)
    out = torch.empty((w.nrows, w.ngrid ** 3), dtype=torch.float64, device="cuda")
    times = {}
    ctx = P.Context(0)
    ctx.set_orbitals(w.energies, w.nocc, w.psi_grid, w.grid_dV)
    ctx.set_sites(w.sites, w.psi_site)
    ctx.make_quadrature(P.QUAD_TIME, n, 0.0)
    scale = ctx.get_quadrature()["scale"]
    for prec in ("f16f8", "fp64"):
        ctx.chi0(-1, P.COLS_GRID, prec, out=out)
        times[prec + " complex"] = ctx.last_kernel_ms()
    ctx.close()
    w.psi_grid = None
    torch.cuda.empty_cache()
    ctx = P.Context(0)
    ctx.set_orbitals_real(E, w.nocc, g, w.grid_dV)
    ctx.set_sites(w.sites, s[None])
    ctx.make_quadrature(P.QUAD_TIME, n, scale)
    terms = cz.terms_for(w.energies, w.nocc, "time", n, scale)
    ref = cz.chi0_quad_entries(ps, pg, w.nocc, 2, *terms)
    for prec, tol in (("f16f8", 1e-4), ("fp64", 1e-12)):
        ctx.chi0(-1, P.COLS_GRID, prec, out=out)
        ctx.chi0(-1, P.COLS_GRID, prec, out=out)
        times[prec + " real"] = ctx.last_kernel_ms()
        got = out[torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")]
        e = rel(got.cpu().numpy(), ref)
        say(f"  {prec} real: {times[prec + ' real']:.0f} ms (complex orbitals "
            f"{times[prec + ' complex']:.0f} ms), vs oracle {e:.2e}")
        assert e < tol
    ctx.close()


def test_real_orbitals_many_k(P):
    """Real orbitals at 8 k-points (production workload: 576 bands, 2 sites of 800 points, 24^3
    grid, 24 terms).  chi0 is defined for any orbital set, so the real parts of the workload's
    orbitals serve as the input: FP64 and F16F8 site x grid and site blocks from the real path,
    sampled against the oracle on the same real orbitals, and the FP64 result against the
    complex path given the same orbitals as complex values."""
    w = workload("production")
    n = w.n_terms
    g = w.psi_grid.real.contiguous()
    s = w.psi_site.real.contiguous()
    ctx = P.Context(0)
    ctx.set_orbitals_real(w.energies, w.nocc, g, w.grid_dV)
    ctx.set_sites(w.sites, s)
    ctx.make_quadrature(P.QUAD_TIME, n, 0.0)
    scale = ctx.get_quadrature()["scale"]
    c2 = P.Context(0)
    c2.set_orbitals(w.energies, w.nocc, g.to(torch.complex128), w.grid_dV)
    c2.set_sites(w.sites, s.to(torch.complex128))
    c2.make_quadrature(P.QUAD_TIME, n, scale)
    cplx = c2.chi0(-1, P.COLS_GRID, P.FP64).cpu().numpy()
    cplx_s = c2.chi0(-1, P.COLS_SITE, P.FP64).cpu().numpy()
    # the adjoint on a seeded dL/dchi0: complex path (F16F8) on the same orbitals
    lam = torch.as_tensor(np.random.default_rng(6).standard_normal(cplx_s.size), device="cuda")
    c2.chi0(-1, P.COLS_SITE, P.F16F8)
    dE_c, dp_c = c2.chi0_backward(lam, P.F16F8)
    c2.close()
    rng = np.random.default_rng(5)
    rows = rng.integers(0, w.nrows, 40)
    cols = rng.integers(0, w.ngrid ** 3, 40)
    sg = s.numpy().astype(np.complex128)
    gg = g.numpy().astype(np.complex128)
    terms = cz.terms_for(w.energies, w.nocc, "time", n, scale)
    ref = cz.chi0_quad_entries(sg[:, :, rows], gg[:, :, cols], w.nocc, 2, *terms)
    site = 1
    o = w.site_offsets[site]
    m = w.site_offsets[site + 1] - o
    ra = rng.integers(0, m, 40)
    rb = rng.integers(0, m, 40)
    ref_s = cz.chi0_quad_entries(sg[:, :, o + ra], sg[:, :, o + rb], w.nocc, 2, *terms)
    for prec, tol in (("fp64", 1e-12), ("f16f8", 1e-4)):
        got = ctx.chi0(-1, P.COLS_GRID, prec).cpu().numpy()
        blk = ctx.site_blocks(ctx.chi0(-1, P.COLS_SITE, prec))[site].cpu().numpy()
        eg = rel(got[rows, cols], ref)
        es = rel(blk[ra, rb], ref_s)
        say(f"  8 k real {prec}: grid {eg:.2e} site {es:.2e} vs oracle")
        assert eg < tol and es < tol
        if prec == "fp64":
            ec = rel(got, cplx)
            ecs = rel(ctx.chi0(-1, P.COLS_SITE, prec).cpu().numpy(), cplx_s)
            say(f"  8 k real vs complex path: grid {ec:.2e} site {ecs:.2e}")
            assert ec < 1e-12 and ecs < 1e-12
    # (the last forward call above is the F16F8 site-block one, so its Green's functions are
    # kept) the real-orbital adjoint against the complex path's
    dE_r, dp_r = ctx.chi0_backward(lam, P.F16F8)
    eE = rel(dE_r.cpu().numpy(), dE_c.cpu().numpy())
    ep = rel(dp_r.real.cpu().numpy(), dp_c.real.cpu().numpy())
    say(f"  8 k real-orbital adjoint vs complex path: dE {eE:.2e} dpsi {ep:.2e}")
    assert eE < 1e-4 and ep < 1e-4
    ctx.close()
