"""GPU parity at full size, in the launch configuration the benchmark times: the precision
workload at 2x2x2 k (3520 site points x 110,592 grid points, 8 k x 2304 bands, 32
imaginary-time terms), site x grid and site x site launches, against the oracle on seeded
sampled entries computed one by one.

Error measure: max |gpu - ref| / max |ref| over the sampled entries.  Bars: FP64 1e-12
against the same terms and 1e-6 against the exact pair sum; BF16X2 / FP16X2 1e-4 against
both.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import chi0 as cz
from oracle import quadrature as q

pytestmark = pytest.mark.gpu

NS = 192


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_07834_amd as P
    from workloads import configs
    say("precision workload, 2x2x2 k, with the grid")
    w = configs.precision(device="cuda")
    rng = np.random.default_rng(31)
    rows = rng.integers(0, w.nrows, NS)
    cols = rng.integers(0, w.ngrid ** 3, NS)
    ps = w.psi_site[:, :, torch.as_tensor(rows, device="cuda")].cpu().numpy()
    pg = w.psi_grid[:, :, torch.as_tensor(cols, device="cuda")].cpu().numpy()
    ctx = P.Context(0)
    ctx.set_orbitals(w.energies, w.nocc, w.psi_grid, w.grid_dV)
    ctx.set_sites(w.sites, w.psi_site)
    w.psi_grid = None
    torch.cuda.empty_cache()
    mu = q.mid_gap(w.energies, w.nocc)
    x, y = q.offsets(w.energies, w.nocc, mu)
    scale = q.auto_scale(x, y, w.n_terms)
    terms = cz.terms_for(w.energies, w.nocc, "time", w.n_terms, scale, mu)
    say(f"  oracle on {NS} sampled entries")
    ref_q = cz.chi0_quad_entries(ps, pg, w.nocc, 2, *terms)
    ref_x = cz.chi0_exact_entries(ps, pg, w.energies, w.nocc, mu=mu)
    out = torch.empty((w.nrows, w.ngrid ** 3), dtype=torch.float64, device="cuda")
    yield dict(P=P, w=w, ctx=ctx, rows=rows, cols=cols, ps=ps, pg=pg, mu=mu, scale=scale,
               terms=terms, ref_q=ref_q, ref_x=ref_x, out=out)
    ctx.close()
    del out
    torch.cuda.empty_cache()


def sampled(F, out):
    return out[torch.as_tensor(F["rows"], device="cuda"),
               torch.as_tensor(F["cols"], device="cuda")].cpu().numpy()


@pytest.mark.parametrize("prec,tq,tx", [("bf16x2", 1e-4, 1e-4), ("fp16x2", 1e-4, 1e-4),
                                        ("f16f8", 1e-4, 1e-4), ("fp64", 1e-12, 1e-6),
                                        ("fp64m3", 1e-12, 1e-6)])
def test_grid_launch_sampled(full, prec, tq, tx):
    """The site x grid launch (the benchmark's headline launch), every precision of the
    bench line, with the library's own scale choice equal to the oracle's."""
    F = full
    P, ctx = F["P"], F["ctx"]
    ctx.make_quadrature(P.QUAD_TIME, F["w"].n_terms, 0.0)
    assert ctx.get_quadrature()["scale"] == F["scale"]
    ctx.chi0(-1, P.COLS_GRID, prec, out=F["out"])
    got = sampled(F, F["out"])
    eq, ex = rel(got, F["ref_q"]), rel(got, F["ref_x"])
    say(f"  grid {prec}: {ctx.last_kernel_ms():.0f} ms, vs same terms {eq:.2e}, vs exact {ex:.2e}")
    assert eq < tq and ex < tx


def test_site_block_sampled_and_symmetric(full):
    """The site x site launch (upper-triangle tiles, mirrored): sampled entries and their
    transposes against the oracle (BF16X2, FP64 and FP64 3M), and the block exactly
    symmetric."""
    F = full
    P, ctx, w = F["P"], F["ctx"], F["w"]
    ctx.make_quadrature(P.QUAD_TIME, w.n_terms, 0.0)
    rng = np.random.default_rng(32)
    r = rng.integers(0, w.nrows, 96)
    c = rng.integers(0, w.nrows, 96)
    rr, cc = np.concatenate([r, c]), np.concatenate([c, r])
    ps_all = w.psi_site.cpu().numpy()
    ref = cz.chi0_quad_entries(ps_all[:, :, rr], ps_all[:, :, cc], w.nocc, 2, *F["terms"])
    for prec, tol in [("bf16x2", 1e-4), ("fp64", 1e-12), ("fp64m3", 1e-12)]:
        blk = ctx.site_blocks(ctx.chi0(-1, P.COLS_SITE, prec))[0]
        e = rel(blk[torch.as_tensor(rr, device="cuda"), torch.as_tensor(cc, device="cuda")]
                .cpu().numpy(), ref)
        say(f"  site block {prec}: {ctx.last_kernel_ms():.0f} ms, vs same terms {e:.2e}")
        assert e < tol
        assert torch.equal(blk, blk.T)


def test_grid_launch_imaginary_frequency(full):
    """chi0(i omega) on the same launch (complex term coefficients), BF16X2, against the
    oracle with the same terms and against the exact pair sum, odd part included."""
    F = full
    P, ctx, w = F["P"], F["ctx"], F["w"]
    omega = 0.1
    ctx.make_quadrature_iw(w.n_terms, 0.0, omega)
    sc = ctx.get_quadrature()["scale"]
    x, y = q.offsets(w.energies, w.nocc, F["mu"])
    assert sc == q.auto_scale_iw(x, y, w.n_terms, omega)
    tiw = cz.terms_for(w.energies, w.nocc, f"time_iw:{omega}", w.n_terms, sc, F["mu"])
    ref_q = cz.chi0_iw_quad_entries(F["ps"], F["pg"], w.nocc, 2, *tiw)
    ref_x = cz.chi0_iw_exact_entries(F["ps"], F["pg"], w.energies, w.nocc, omega, mu=F["mu"])
    ctx.chi0(-1, P.COLS_GRID, "bf16x2", out=F["out"])
    got = sampled(F, F["out"])
    eq, ex = rel(got, ref_q), rel(got, ref_x)
    say(f"  grid bf16x2 at i omega = {omega}i: {ctx.last_kernel_ms():.0f} ms, vs same terms "
        f"{eq:.2e}, vs exact {ex:.2e}")
    assert eq < 1e-4 and ex < 1e-4



def test_gamma_grid_launch_sampled():
    """The precision workload at Gamma (the other half of its "Gamma + 2x2x2 k" k-sets): the
    site x grid launch in BF16X2 and FP64 against the oracle on sampled entries (same terms and
    exact pair sum)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_07834_amd as P
    from workloads import configs
    say("precision workload at Gamma, with the grid")
    w = configs.precision(device="cuda", gamma_only=True)
    rng = np.random.default_rng(35)
    rows = rng.integers(0, w.nrows, NS)
    cols = rng.integers(0, w.ngrid ** 3, NS)
    ps = w.psi_site[:, :, torch.as_tensor(rows, device="cuda")].cpu().numpy()
    pg = w.psi_grid[:, :, torch.as_tensor(cols, device="cuda")].cpu().numpy()
    ctx = P.Context(0)
    ctx.set_orbitals(w.energies, w.nocc, w.psi_grid, w.grid_dV)
    ctx.set_sites(w.sites, w.psi_site)
    w.psi_grid = None
    torch.cuda.empty_cache()
    ctx.make_quadrature(P.QUAD_TIME, w.n_terms, 0.0)
    mu = q.mid_gap(w.energies, w.nocc)
    terms = cz.terms_for(w.energies, w.nocc, "time", w.n_terms, ctx.get_quadrature()["scale"], mu)
    ref_q = cz.chi0_quad_entries(ps, pg, w.nocc, 2, *terms)
    ref_x = cz.chi0_exact_entries(ps, pg, w.energies, w.nocc, mu=mu)
    out = torch.empty((w.nrows, w.ngrid ** 3), dtype=torch.float64, device="cuda")
    for prec, tq, tx in (("bf16x2", 1e-4, 1e-4), ("fp64", 1e-12, 1e-6)):
        ctx.chi0(-1, P.COLS_GRID, prec, out=out)
        got = out[torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")]
        got = got.cpu().numpy()
        eq, ex = rel(got, ref_q), rel(got, ref_x)
        say(f"  Gamma grid {prec}: {ctx.last_kernel_ms():.0f} ms, vs same terms {eq:.2e}, "
            f"vs exact {ex:.2e}")
        assert eq < tq and ex < tx
    ctx.close()
    del out
    torch.cuda.empty_cache()
