"""GPU parity of chi0 from real orbitals at the Gamma point (Sec. VI.F; lrs_set_orbitals_real).

The synthetic crystals have a real potential, so their Gamma orbitals can be made real: a phase
per band and a real basis of each degenerate set (a unitary change within the set, which leaves
chi0 unchanged, since a set's orbitals carry equal weights).  The tests make them real
(`realify`, on the device), then compare the library's real-orbital chi0 (FP64 and F16F8)
with the oracle's band-pair sum on the same real orbitals, and with the library's complex path
on the original orbitals.  Error measure: max |gpu - ref| / max |ref|.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import chi0 as cz
from oracle import quadrature as q
from tests.conftest import workload

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


def realify(E, arrays, tol=1e-8):
    """Real orbitals spanning each degenerate set of complex Gamma orbitals.  arrays: complex
    [nb, P_i] device tensors sampling the same orbitals (the first, a full grid, fixes the
    change of basis); returns their real versions (float64) and the largest imaginary part
    left relative to the largest value, over all arrays."""
    nb = len(E)
    out = [torch.empty_like(a) for a in arrays]
    b = 0
    while b < nb:
        e = b + 1
        while e < nb and abs(E[e] - E[b]) <= tol * max(1.0, abs(E[b])):
            e += 1
        V = arrays[0][b:e]                                    # [d, Ng]
        A = torch.cat([V.real, V.imag])                       # [2d, Ng] real
        _, _, Wh = torch.linalg.svd(A, full_matrices=False)
        W = Wh[: e - b].to(V.dtype)                           # real orthonormal rows
        G = V @ V.conj().T                                    # [d, d], a multiple of I
        C = (W @ V.conj().T) @ torch.linalg.inv(G)            # W = C V
        C = C * torch.sqrt(torch.diagonal(G).real.mean())     # keep the orbitals' norms
        for o, a in zip(out, arrays):
            o[b:e] = C @ a[b:e]
        b = e
    left = max(float(o.imag.abs().max() / o.abs().max()) for o in out)
    return [o.real.contiguous() for o in out], left


def oracle_scale(E, nocc, n):
    mu = q.mid_gap(E, nocc)
    x, y = q.offsets(E, nocc, mu)
    return q.auto_scale(x, y, n)


@pytest.fixture(scope="module")
def tiny_real():
    w = workload("tiny")
    E = w.energies[0]
    (g, s), left = realify(E, [w.psi_grid[0].to("cuda"), w.psi_site[0].to("cuda")])
    return dict(w=w, E=E, g=g, s=s, left=left)


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


def test_real_orbitals_precision_gamma(P):
    """Precision workload at Gamma (2304 bands, 3520 site rows x 110,592 grid columns, 32
    terms): the site x grid launch from real orbitals in FP64 and F16F8, sampled against the
    oracle on the real orbitals, and timed beside the complex launch of each precision."""
    from workloads import configs
    w = configs.precision(device="cuda", gamma_only=True)
    E = w.energies[0]
    (g, s), left = realify(E, [w.psi_grid[0], w.psi_site[0]])
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
