"""GPU parity at the largest size: the batching workload's site x grid launch, whose output
is addressed past 2^32 elements, against the oracle on seeded sampled entries.

Error measure: max |gpu - ref| / max |ref| over the sampled entries; bar 1e-4 (BF16X2).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import chi0 as cz

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_batching_grid_launch_sampled():
    """The batching workload's site x grid launch in BF16X2: 64 uneven sites (87,040 rows) x
    110,592 grid columns, 28 terms, 2x2x2 k, run in operand batches of at most 24 GiB; the
    output (9.6e9 entries, 77 GB) is addressed past 2^32 elements.  Three sampled entries per
    site against the oracle with the same terms."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import time

    import paper_2005_07834_amd as P
    from tests.conftest import workload
    from workloads import crystal as cx
    w = workload("batching", with_grid=False, device="cuda")
    ncols = w.ngrid ** 3
    say(f"batching grid launch: {len(w.sites)} sites, {w.nrows} rows x {ncols} columns")
    psi_grid = torch.stack([cx.psi_on_grid(w.bands, w.ngrid, k) for k in range(w.bands.nk)])
    rng = np.random.default_rng(33)
    offs = w.site_offsets
    rows = np.array([offs[k] + rng.integers(0, s.npts) for k, s in enumerate(w.sites)
                     for _ in range(3)])
    cols = rng.integers(0, ncols, rows.size)
    assert (rows.astype(np.int64) * ncols + cols).max() > 2 ** 32
    ps = w.psi_site[:, :, torch.as_tensor(rows, device="cuda")].cpu().numpy()
    pg = psi_grid[:, :, torch.as_tensor(cols, device="cuda")].cpu().numpy()
    ctx = P.Context(0)
    ctx.set_orbitals(w.energies, w.nocc, psi_grid, w.grid_dV)
    ctx.set_sites(w.sites, w.psi_site)
    del psi_grid
    torch.cuda.empty_cache()
    ctx.make_quadrature(P.QUAD_TIME, w.n_terms, 0.0)
    sc = ctx.get_quadrature()["scale"]
    terms = cz.terms_for(w.energies, w.nocc, "time", w.n_terms, sc)
    ref = cz.chi0_quad_entries(ps, pg, w.nocc, 2, *terms)
    out = torch.empty((w.nrows, ncols), dtype=torch.float64, device="cuda")
    t0 = time.time()
    ctx.chi0(-1, P.COLS_GRID, "bf16x2", out=out)
    torch.cuda.synchronize()
    dt = time.time() - t0
    got = out[torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")]
    e = rel(got.cpu().numpy(), ref)
    say(f"  bf16x2: {dt:.1f} s for the call, vs same terms {e:.2e}")
    assert e < 1e-4
    ctx.close()
    del out


def test_batching_fp32_grid_launch_sampled():
    """The batching workload's FP32 variant on the site x grid launch: the largest, the
    smallest and a ragged site (rows not a multiple of the 128-row tile) of the 64 uneven
    sites, each over all 110,592 grid columns with 28 terms, sampled against the oracle with
    the same terms (bar 1e-5)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import time

    import paper_2005_07834_amd as P
    from tests.conftest import workload
    from workloads import crystal as cx
    w = workload("batching", with_grid=False, device="cuda")
    ncols = w.ngrid ** 3
    sizes = [s.npts for s in w.sites]
    pick = [int(np.argmax(sizes)), int(np.argmin(sizes))]
    pick.append(next(k for k, n in enumerate(sizes) if n % 128 and k not in pick))
    say(f"batching FP32 grid launch: sites {pick} ({[sizes[k] for k in pick]} rows)")
    psi_grid = torch.stack([cx.psi_on_grid(w.bands, w.ngrid, k) for k in range(w.bands.nk)])
    rng = np.random.default_rng(34)
    offs = w.site_offsets
    ctx = P.Context(0)
    ctx.set_orbitals(w.energies, w.nocc, psi_grid, w.grid_dV)
    ctx.set_sites(w.sites, w.psi_site)
    ctx.make_quadrature(P.QUAD_TIME, w.n_terms, 0.0)
    terms = cz.terms_for(w.energies, w.nocc, "time", w.n_terms, ctx.get_quadrature()["scale"])
    worst = 0.0
    for k in pick:
        r = rng.integers(0, sizes[k], 8)
        c = rng.integers(0, ncols, 8)
        ps = w.psi_site[:, :, torch.as_tensor(offs[k] + r, device="cuda")].cpu().numpy()
        pg = psi_grid[:, :, torch.as_tensor(c, device="cuda")].cpu().numpy()
        ref = cz.chi0_quad_entries(ps, pg, w.nocc, 2, *terms)
        t0 = time.time()
        out = ctx.chi0(k, P.COLS_GRID, "fp32")
        torch.cuda.synchronize()
        got = out[torch.as_tensor(r, device="cuda"), torch.as_tensor(c, device="cuda")]
        e = rel(got.cpu().numpy(), ref)
        say(f"  site {k} ({sizes[k]} rows): {time.time() - t0:.1f} s, vs same terms {e:.2e}")
        worst = max(worst, e)
        del out
    assert worst < 1e-5
    ctx.close()
    del psi_grid
    torch.cuda.empty_cache()
