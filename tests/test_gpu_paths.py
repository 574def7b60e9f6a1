"""GPU tests of the differentiable path, the batched launch, graph capture and tuning.

Every comparison goes through the C ABI (via the thin binding) and against the FP64 CPU
oracle or against finite differences of the FP64 GPU path itself.
Error measure: max |gpu - ref| / max |ref| over the compared entries.
"""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import chi0 as cz
from oracle import grads as gr
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
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def oracle_scale(w, n):
    mu = q.mid_gap(w.energies, w.nocc)
    x, y = q.offsets(w.energies, w.nocc, mu)
    return q.auto_scale(x, y, n)


def make_ctx(P, w, n, scale, grid=True):
    ctx = P.Context(0)
    ctx.set_orbitals(w.energies, w.nocc, w.psi_grid if grid else None, w.grid_dV)
    ctx.set_sites(w.sites, w.psi_site)
    ctx.make_quadrature(P.QUAD_TIME, n, scale)
    return ctx


def site_pairs(w, n_per_site, rng, sites=None):
    """Seeded (row, col) pairs inside the site x site blocks: global rows, and the flat index
    of each pair in the site-block layout."""
    offs = w.site_offsets
    blk = np.cumsum([0] + [s.npts ** 2 for s in w.sites])
    rows, cols, flat = [], [], []
    for s in (range(len(w.sites)) if sites is None else sites):
        n = w.sites[s].npts
        i = rng.integers(0, n, n_per_site)
        j = rng.integers(0, n, n_per_site)
        rows += list(offs[s] + i)
        cols += list(offs[s] + j)
        flat += list(blk[s] + i * n + j)
    return np.array(rows), np.array(cols), np.array(flat)


# ------------------------------------------------------------------ differentiation
def test_chi0fn_energies_without_gradient(P):
    """Energies given as an array (or a tensor without requires_grad): the backward pass returns
    no energy gradient, and the orbital gradient equals the one taken with differentiable
    energies."""
    w = workload("tiny")
    n = w.n_terms
    s = oracle_scale(w, n)
    say("Chi0Fn with energies that take no gradient, tiny")
    ctx = P.Context(0)
    lam = None
    grads = []
    for E in (np.asarray(w.energies), torch.tensor(w.energies, dtype=torch.float64),
              torch.tensor(w.energies, dtype=torch.float64, requires_grad=True)):
        psi = w.psi_site.to("cuda").clone().requires_grad_(True)
        chi = P.Chi0Fn.apply(E, psi, ctx, w.nocc, w.sites, n, s)
        if lam is None:
            lam = torch.randn(chi.shape, dtype=torch.float64, device="cuda",
                              generator=torch.Generator("cuda").manual_seed(5))
        (chi * lam).sum().backward()
        grads.append(psi.grad.clone())
        if isinstance(E, torch.Tensor) and E.requires_grad:
            assert E.grad is not None and torch.isfinite(E.grad).all()
    e = max(float((g - grads[2]).abs().max() / grads[2].abs().max()) for g in grads[:2])
    say(f"  dpsi with and without an energy gradient: {e:.2e}")
    assert e == 0.0
    ctx.close()


def test_autograd_gradcheck_tiny(P):
    """Chi0Fn -> ScreenWFn -> sum of losses against torch's numerical Jacobian (FP64 path)."""
    w = workload("tiny")
    n = w.n_terms
    s = oracle_scale(w, n)
    say("autograd gradcheck, tiny")
    ctx = P.Context(0)
    E = torch.tensor(w.energies, dtype=torch.float64, requires_grad=True)
    psi = w.psi_site.to("cuda").clone().requires_grad_(True)
    rho = torch.as_tensor(w.rho_test, device="cuda")

    def f(E_, psi_):
        chi = P.Chi0Fn.apply(E_, psi_, ctx, w.nocc, w.sites, n, s)
        W, loss = P.ScreenWFn.apply(chi, ctx, rho)
        return loss.sum() + 0.1 * (W * W).sum()

    assert torch.autograd.gradcheck(f, (E, psi), eps=1e-6, atol=1e-7, rtol=1e-4,
                                    fast_mode=True)


@pytest.mark.parametrize("prec,tol_l,tol_g", [(None, 1e-12, 1e-9), ("bf16x2", 1e-4, 1e-4),
                                              ("f16f8", 1e-4, 1e-4)])
def test_autograd_matches_oracle_tiny(P, prec, tol_l, tol_g):
    """Loss and gradients through Chi0Fn and ScreenWFn against the oracle: the FP64 path (the
    default), and the split path (BF16X2 forward and adjoint products)."""
    w = workload("tiny")
    n = w.n_terms
    s = oracle_scale(w, n)
    say(f"autograd gradients vs oracle, tiny ({prec or 'fp64'})")
    ctx = P.Context(0)
    E = torch.tensor(w.energies, dtype=torch.float64, requires_grad=True)
    psi = w.psi_site.to("cuda").clone().requires_grad_(True)
    rho = torch.as_tensor(w.rho_test, device="cuda")
    extra = () if prec is None else (prec,)
    chi = P.Chi0Fn.apply(E, psi, ctx, w.nocc, w.sites, n, s, *extra)
    W, loss = P.ScreenWFn.apply(chi, ctx, rho)
    loss.sum().backward()
    L_ref, dE_ref, dpsi_ref = gr.loss_and_grads(w.psi_site.numpy(), w.energies, w.nocc, 2,
                                                w.sites, w.rho_test, "time", n, s)
    eL = abs(loss.sum().item() - L_ref) / abs(L_ref)
    eE = rel(E.grad.numpy(), dE_ref)
    ep = rel(psi.grad.cpu().numpy(), dpsi_ref)
    say(f"  loss {eL:.2e} dE {eE:.2e} dpsi {ep:.2e}")
    assert eL < tol_l and eE < tol_g and ep < tol_g


def test_differentiation_workload_fd_and_oracle(P):
    """Differentiation workload (production cell, 4 sites, 2x2x2 k): the adjoint against
    central finite differences of the FP64 GPU path (energy step 1e-5 Ha; orbitals along a
    seeded direction) and, for site 0, against the oracle's reference gradient."""
    w = workload("differentiation")
    n = w.n_terms
    s = oracle_scale(w, n)
    say("differentiation workload: FD + oracle (site 0)")
    ctx = P.Context(0)
    rho = torch.as_tensor(w.rho_test, device="cuda")
    psi0 = w.psi_site.to("cuda")

    def loss_of(E_, psi_):
        chi = P.Chi0Fn.apply(E_, psi_, ctx, w.nocc, w.sites, n, s)
        return P.ScreenWFn.apply(chi, ctx, rho)[1].sum()

    E = torch.tensor(w.energies, dtype=torch.float64, requires_grad=True)
    psi = psi0.clone().requires_grad_(True)
    L = loss_of(E, psi)
    L.backward()
    dE = E.grad.numpy()
    dpsi = psi.grad
    rng = np.random.default_rng(17)
    no = w.nocc
    picks = [(int(rng.integers(0, w.nk)), b) for b in (no - 1, no - 5, 3, no, no + 7, no + 200)]
    h = 1e-5
    with torch.no_grad():
        for k, b in picks:
            Ep = w.energies.copy()
            Ep[k, b] += h
            Em = w.energies.copy()
            Em[k, b] -= h
            fd = (loss_of(torch.as_tensor(Ep), psi0).item()
                  - loss_of(torch.as_tensor(Em), psi0).item()) / (2 * h)
            err = abs(fd - dE[k, b]) / np.abs(dE).max()
            say(f"  dL/dE[{k},{b}] adjoint {dE[k, b]:.6e} fd {fd:.6e} rel {err:.2e}")
            assert err < 1e-6
        g = torch.Generator(device="cpu").manual_seed(5)
        V = torch.complex(torch.randn(psi0.shape, generator=g, dtype=torch.float64),
                          torch.randn(psi0.shape, generator=g, dtype=torch.float64)).to("cuda")
        V /= V.abs().max()
        hp = 1e-5 * psi0.abs().max().item()
        fd = (loss_of(E.detach(), psi0 + hp * V).item()
              - loss_of(E.detach(), psi0 - hp * V).item()) / (2 * hp)
        ad = torch.sum(dpsi.real * V.real + dpsi.imag * V.imag).item()
        err = abs(fd - ad) / abs(ad)
        say(f"  directional dL/dpsi adjoint {ad:.6e} fd {fd:.6e} rel {err:.2e}")
        assert err < 1e-6

    # site 0 alone against the oracle's reference gradient (same quadrature)
    sl = gr.site_slices(w.sites)[0]
    ctx1 = P.Context(0)
    E1 = torch.tensor(w.energies, dtype=torch.float64, requires_grad=True)
    p1 = psi0[:, :, sl].contiguous().requires_grad_(True)
    chi = P.Chi0Fn.apply(E1, p1, ctx1, w.nocc, w.sites[:1], n, s)
    L1 = P.ScreenWFn.apply(chi, ctx1, rho[sl].contiguous())[1].sum()
    L1.backward()
    say("  oracle reference gradient for site 0 (CPU)")
    L_ref, dE_ref, dpsi_ref, W_ref = gr.loss_and_grads(w.psi_site.numpy()[:, :, sl], w.energies,
                                                       w.nocc, 2, w.sites[:1], w.rho_test[sl],
                                                       "time", n, s, with_W=True)
    eL = abs(L1.item() - L_ref) / abs(L_ref)
    eE = rel(E1.grad.numpy(), dE_ref)
    ep = rel(p1.grad.cpu().numpy(), dpsi_ref)
    say(f"  site 0 vs oracle: loss {eL:.2e} dE {eE:.2e} dpsi {ep:.2e}")
    assert eL < 1e-11 and eE < 1e-8 and ep < 1e-8
    # W of site 0 from the split-precision chi0 and from the FP64 one, element by element
    # against the oracle's W on the same terms
    with torch.no_grad():
        for prec, tol in (("bf16x2", 1e-4), ("fp64", 1e-10)):
            ctx1.set_orbitals(w.energies, w.nocc)
            ctx1.set_sites(w.sites[:1], p1.detach())
            ctx1.make_quadrature(P.QUAD_TIME, n, s)
            Wg, lg = ctx1.screen_W(ctx1.chi0(-1, P.COLS_SITE, prec), rho=rho[sl].contiguous(),
                                   want_loss=True)
            Wg = ctx1.W_blocks(Wg)[0].cpu().numpy()
            eW = rel(Wg, W_ref[0])
            eF = float(np.linalg.norm(Wg - W_ref[0]) / np.linalg.norm(W_ref[0]))
            eLs = abs(lg.item() - L_ref) / abs(L_ref)
            say(f"  site 0 W from {prec} chi0 vs oracle W: max {eW:.2e} frobenius {eF:.2e} "
                f"loss {eLs:.2e}")
            assert eW < tol and eLs < tol


def test_split_adjoint_matches_fp64(P):
    """Differentiation workload (4 sites of 800 points, 2x2x2 k, 24 terms): the adjoint with
    split-precision products (Green's functions in BF16X2, then in F16F8) against the FP64
    adjoint on the same dL/dchi0, per site; each result is bitwise reproducible."""
    w = workload("differentiation")
    n = w.n_terms
    s = oracle_scale(w, n)
    say("split adjoint vs FP64 adjoint (differentiation workload)")
    ctx = make_ctx(P, w, n, s, grid=False)
    chi = ctx.chi0(-1, P.COLS_SITE, P.FP64)
    ctx.screen_W(chi, rho=torch.as_tensor(w.rho_test, device="cuda"), want_loss=True)
    lam = ctx.screen_W_backward()
    dE64, dp64 = ctx.chi0_backward(lam, P.FP64)
    for prec in (P.BF16X2, P.F16F8):
        if prec == P.F16F8:
            ctx.chi0(-1, P.COLS_SITE, prec)      # (the forward call whose operand it reads)
        dEs, dps = ctx.chi0_backward(lam, prec)
        eE = rel(dEs.cpu().numpy(), dE64.cpu().numpy())
        say(f"  precision {prec}: dE {eE:.2e}")
        assert eE < 1e-4
        for k, sl in enumerate(gr.site_slices(w.sites)):
            ep = rel(dps[:, :, sl].cpu().numpy(), dp64[:, :, sl].cpu().numpy())
            say(f"  dpsi site {k}: {ep:.2e}")
            assert ep < 1e-4
        dEs2, dps2 = ctx.chi0_backward(lam, prec)
        assert torch.equal(dEs, dEs2) and torch.equal(dps, dps2)
    ctx.close()


@pytest.mark.parametrize("prec", ["f16f8", "bf16x2", "fp64"])
def test_kept_green_functions_match_recompute(P, prec):
    """The adjoint built from the Green's functions that the forward site-block launch
    keeps equals, bit for bit, the adjoint that recomputes them (differentiation workload, 4
    sites of 800 points; the static rule and chi0 at imaginary frequency); a new quadrature
    drops the kept ones, so the second call recomputes."""
    w = workload("differentiation")
    n = w.n_terms
    s = oracle_scale(w, n)
    ctx = make_ctx(P, w, n, s, grid=False)
    rng = np.random.default_rng(31)
    lam = torch.as_tensor(rng.standard_normal(sum(x.npts ** 2 for x in w.sites)), device="cuda")
    rules = (("static", lambda: ctx.make_quadrature(P.QUAD_TIME, n, s)),
             ("i omega", lambda: ctx.make_quadrature_iw(n, 0.0, 0.3)))
    for name, rule in rules:
        rule()
        ctx.chi0(-1, P.COLS_SITE, prec)               # keeps every term's G_o, G_u
        dE1, dp1 = ctx.chi0_backward(lam, prec)
        rule()                                        # drops them
        dE2, dp2 = ctx.chi0_backward(lam, prec)       # recomputes them
        say(f"kept vs recomputed Green's functions ({prec}, {name}): dE equal "
            f"{torch.equal(dE1, dE2)}, dpsi equal {torch.equal(dp1, dp2)}")
        assert torch.equal(dE1, dE2) and torch.equal(dp1, dp2)
    ctx.close()


# ------------------------------------------------------------------ batching
def test_batching_uneven_sites(P):
    """64 sites with uneven radial x angular grids, 2x2x2 k, 28 terms: all site x site blocks
    in one call (persistent launches over operand batches), sampled against the oracle in
    BF16X2, FP32 and FP64; the BF16X2 call captured into a HIP graph replays to the same bits;
    a much smaller operand budget (more batches) gives the same result."""
    w = workload("batching", with_grid=False, device="cuda")
    n = w.n_terms
    s = oracle_scale(w, n)
    say(f"batching: {len(w.sites)} sites, {w.nrows} points, npts "
        f"{min(x.npts for x in w.sites)}..{max(x.npts for x in w.sites)}")
    rng = np.random.default_rng(23)
    rows, cols, flat = site_pairs(w, 3, rng)
    ps_r = w.psi_site[:, :, torch.as_tensor(rows, device="cuda")].cpu().numpy()
    ps_c = w.psi_site[:, :, torch.as_tensor(cols, device="cuda")].cpu().numpy()
    terms = cz.terms_for(w.energies, w.nocc, "time", n, s)
    ref = cz.chi0_quad_entries(ps_r, ps_c, w.nocc, 2, *terms)
    st = torch.cuda.Stream()   # the context enqueues on st, which the graph captures
    with torch.cuda.stream(st):
        ctx = make_ctx(P, w, n, s, grid=False)
        fidx = torch.as_tensor(flat, device="cuda")
        for prec, tol in [("bf16x2", 1e-4), ("fp32", 1e-5), ("fp64", 1e-12)]:
            out = ctx.chi0(-1, P.COLS_SITE, prec)
            got = out[fidx].cpu().numpy()
            say(f"  {prec}: {ctx.last_kernel_ms():.1f} ms, rel err {rel(got, ref):.3e}")
            assert rel(got, ref) < tol
            if prec == "bf16x2":
                base = out.clone()
        del out
        gout = torch.empty_like(base)
    torch.cuda.synchronize()
    # the whole batched BF16X2 call in a graph
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        ctx.chi0(-1, P.COLS_SITE, "bf16x2", out=gout)
    for i in range(2):
        gout.fill_(3.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say(f"  graph replay {i}: equal {torch.equal(gout, base)}")
        assert torch.equal(gout, base)
    del g, gout
    ctx.close()
    old = os.environ.get("LRS_SITE_OPERAND_BYTES")
    os.environ["LRS_SITE_OPERAND_BYTES"] = str(1 << 30)
    try:
        ctx2 = make_ctx(P, w, n, s, grid=False)
        out2 = ctx2.chi0(-1, P.COLS_SITE, "bf16x2")
        say(f"  bf16x2 with a 1 GiB operand budget: max diff {(out2 - base).abs().max().item():.3e}")
        assert torch.equal(out2, base)
        ctx2.close()
    finally:
        if old is None:
            os.environ.pop("LRS_SITE_OPERAND_BYTES")
        else:
            os.environ["LRS_SITE_OPERAND_BYTES"] = old


def test_batching_adjoint(P):
    """The adjoint over 64 uneven sites (6 terms, a seeded dL/dchi0): split products against
    FP64, and the split result unchanged bit for bit when a small operand budget cuts the
    Green's-function launches into many batches."""
    w = workload("batching", with_grid=False, device="cuda")
    n = 6
    s = oracle_scale(w, n)
    ctx = make_ctx(P, w, n, s, grid=False)
    tot = sum(x.npts ** 2 for x in w.sites)
    g = torch.Generator(device="cuda").manual_seed(29)
    lam = torch.randn(tot, generator=g, dtype=torch.float64, device="cuda")
    say(f"batching adjoint: {len(w.sites)} sites, {tot} block entries")
    dE64, dp64 = ctx.chi0_backward(lam, P.FP64)
    dEs, dps = ctx.chi0_backward(lam, P.BF16X2)
    eE = (dEs - dE64).abs().max().item() / dE64.abs().max().item()
    eP = (dps - dp64).abs().max().item() / dp64.abs().max().item()
    say(f"  split vs FP64: dE {eE:.2e} dpsi {eP:.2e}")
    assert eE < 1e-4 and eP < 1e-4
    ctx.close()
    old = os.environ.get("LRS_SITE_OPERAND_BYTES")
    os.environ["LRS_SITE_OPERAND_BYTES"] = str(64 << 20)
    try:
        ctx2 = make_ctx(P, w, n, s, grid=False)
        dEb, dpb = ctx2.chi0_backward(lam, P.BF16X2)
        say(f"  64 MiB operand budget: max diff dE {(dEb - dEs).abs().max().item():.1e} "
            f"dpsi {(dpb - dps).abs().max().item():.1e}")
        assert torch.equal(dEb, dEs) and torch.equal(dpb, dps)
        ctx2.close()
    finally:
        if old is None:
            os.environ.pop("LRS_SITE_OPERAND_BYTES")
        else:
            os.environ["LRS_SITE_OPERAND_BYTES"] = old


# ------------------------------------------------------------------ graph capture, tuning
def test_graph_capture_replay(P):
    """chi0 site x grid (BF16X2) and site x site (FP64) captured into one graph: every
    replay, with eager work and synchronisation between replays, equals the eager result."""
    w = workload("production")
    n = w.n_terms
    s = oracle_scale(w, n)
    say("graph capture, production")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = make_ctx(P, w, n, s)
        og = torch.empty((w.nrows, w.ngrid ** 3), dtype=torch.float64, device="cuda")
        os_ = torch.empty(sum(x.npts ** 2 for x in w.sites), dtype=torch.float64, device="cuda")
        ctx.chi0(-1, P.COLS_GRID, "bf16x2", out=og)
        ctx.chi0(-1, P.COLS_SITE, "fp64", out=os_)
        ref_g, ref_s = og.clone(), os_.clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        ctx.chi0(-1, P.COLS_GRID, "bf16x2", out=og)
        ctx.chi0(-1, P.COLS_SITE, "fp64", out=os_)
    torch.cuda.synchronize()
    for i in range(3):
        og.fill_(7.0)
        os_.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say(f"  replay {i}: grid equal {torch.equal(og, ref_g)} site equal {torch.equal(os_, ref_s)}"
            f" ({junk.item():.2f})")
        assert torch.equal(og, ref_g) and torch.equal(os_, ref_s)
    # an eager call after the replays still matches
    with torch.cuda.stream(st):
        ctx.chi0(-1, P.COLS_GRID, "bf16x2", out=og)
    torch.cuda.synchronize()
    assert torch.equal(og, ref_g)
    ctx.close()


def test_captured_graph_pins_the_context(P):
    """A captured chi0 call pins the context: calls that would free or replace the buffers the
    graph reads (new terms, new sites, a larger operand) are refused with LRS_ESTATE, eager calls
    that fit the existing buffers run, and replays stay bitwise equal to the eager result, also
    after an eager call in another precision has overwritten the site operand (the graph
    rebuilds it).  After lrs_release_graphs the context accepts new inputs again."""
    w = workload("tiny")
    n = w.n_terms
    s = oracle_scale(w, n)
    say("graph pinning, tiny")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = make_ctx(P, w, n, s)
        o64 = ctx.chi0(-1, P.COLS_SITE, "fp64")
        ref = o64.clone()
        obf = ctx.chi0(-1, P.COLS_SITE, "bf16x2")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        ctx.chi0(-1, P.COLS_SITE, "fp64", out=o64)
    torch.cuda.synchronize()

    def replay_equal():
        o64.fill_(5.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        return torch.equal(o64, ref)

    assert replay_equal()
    for what, call in [("make_quadrature", lambda: ctx.make_quadrature(P.QUAD_TIME, n, s)),
                       ("set_sites", lambda: ctx.set_sites(w.sites, w.psi_site)),
                       ("set_orbitals", lambda: ctx.set_orbitals(w.energies, w.nocc))]:
        with pytest.raises(P.LrsError) as e:
            with torch.cuda.stream(st):
                call()
        assert e.value.status == P.LRS_ESTATE, what
        say(f"  {what} refused while pinned")
    with torch.cuda.stream(st):
        again = ctx.chi0(-1, P.COLS_SITE, "bf16x2")      # fits: overwrites the site operand
    torch.cuda.synchronize()
    assert torch.equal(again, obf)
    assert replay_equal()
    say("  replay after an eager split call: equal")
    # the replay rewrote the site operand with the FP64 one: an eager split call rebuilds its own
    with torch.cuda.stream(st):
        again = ctx.chi0(-1, P.COLS_SITE, "bf16x2")
    torch.cuda.synchronize()
    assert torch.equal(again, obf)
    ctx.release_graphs()
    del g
    with torch.cuda.stream(st):
        ctx.make_quadrature(P.QUAD_TIME, n, s)
        assert torch.equal(ctx.chi0(-1, P.COLS_SITE, "fp64"), ref)
    torch.cuda.synchronize()
    ctx.close()


def test_capture_without_warmup_is_refused(P):
    """Capturing a call whose plan is not built yet returns LRS_ESTATE (nothing is allocated
    or launched under capture); so does capturing the backward pass, which copies host tables
    and synchronises."""
    w = workload("tiny")
    n = w.n_terms
    s = oracle_scale(w, n)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = make_ctx(P, w, n, s)
        out = torch.empty((w.nrows, w.ngrid ** 3), dtype=torch.float64, device="cuda")
        lam = torch.zeros(w.nrows ** 2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    for what, call in [("chi0 without a plan", lambda: ctx.chi0(-1, P.COLS_GRID, "fp32", out=out)),
                       ("chi0 backward", lambda: ctx.chi0_backward(lam))]:
        g = torch.cuda.CUDAGraph()
        err = None
        with torch.cuda.stream(st):
            g.capture_begin()
            try:
                call()
            except P.LrsError as e:
                err = e
            finally:
                g.capture_end()
        assert err is not None and err.status == P.LRS_ESTATE
        say(f"  {what} refused: {err}")
        torch.cuda.synchronize()
    ctx.close()


def test_tune_and_determinism(P, tmp_path):
    """The autotuner picks a variant per (precision, column set); the tuned calls agree with the
    default variant's, repeated calls are bitwise identical, and a second context reads the
    choices back from the cache file."""
    w = workload("production")
    n = w.n_terms
    s = oracle_scale(w, n)
    say("tune + determinism, production")
    cache = tmp_path / "tune.txt"
    os.environ["LRS_TUNE_CACHE"] = str(cache)
    try:
        ctx = make_ctx(P, w, n, s)
        chosen = {}
        for prec in ["bf16x2", "fp64"]:
            a = ctx.chi0(-1, P.COLS_GRID, prec)
            b = ctx.chi0(-1, P.COLS_GRID, prec)
            assert torch.equal(a, b)
            sa = ctx.chi0(-1, P.COLS_SITE, prec)
            ctx.tune(prec)
            for cols in (P.COLS_GRID, P.COLS_SITE):
                chosen[(prec, cols)] = ctx.tuned_variant(prec, cols)
            c = ctx.chi0(-1, P.COLS_GRID, prec)
            sc = ctx.chi0(-1, P.COLS_SITE, prec)
            d = (c - a).abs().max().item() / a.abs().max().item()
            ds = (sc - sa).abs().max().item() / sa.abs().max().item()
            say(f"  {prec}: tuned grid {chosen[(prec, P.COLS_GRID)]} site "
                f"{chosen[(prec, P.COLS_SITE)]}; vs default {d:.2e} / {ds:.2e}")
            tol = 1e-6 if prec == "bf16x2" else 1e-13
            assert d < tol and ds < tol
            assert torch.equal(c, ctx.chi0(-1, P.COLS_GRID, prec))
        ctx.close()
        lines = cache.read_text().splitlines()
        assert len(lines) == 4 and all(" variant=" in x for x in lines)
        ctx2 = make_ctx(P, w, n, s)
        for prec in ["bf16x2", "fp64"]:
            ctx2.tune(prec)                          # from the cache file, nothing timed
            for cols in (P.COLS_GRID, P.COLS_SITE):
                assert ctx2.tuned_variant(prec, cols) == chosen[(prec, cols)]
        assert len(cache.read_text().splitlines()) == 4
        ctx2.close()
    finally:
        os.environ.pop("LRS_TUNE_CACHE", None)


def test_single_site_calls_match_all_sites(P):
    """chi0 for one site (site >= 0) equals that site's rows of the all-sites call (grid
    columns) and its block of the site-block layout, bit for bit."""
    w = workload("production")
    n = w.n_terms
    s = oracle_scale(w, n)
    ctx = make_ctx(P, w, n, s)
    offs = w.site_offsets
    for prec in ["bf16x2", "fp64"]:
        allg = ctx.chi0(-1, P.COLS_GRID, prec)
        alls = ctx.site_blocks(ctx.chi0(-1, P.COLS_SITE, prec))
        for k in range(len(w.sites)):
            g = ctx.chi0(k, P.COLS_GRID, prec)
            b = ctx.chi0(k, P.COLS_SITE, prec).view(w.sites[k].npts, w.sites[k].npts)
            assert torch.equal(g, allg[offs[k]:offs[k + 1]])
            assert torch.equal(b, alls[k])
        say(f"  {prec}: single-site calls equal the all-sites call")
    ctx.close()


def test_size_limits_refused(P):
    """Inputs beyond the documented limits are refused on the host before any launch."""
    import ctypes as C
    w = workload("tiny")
    ctx = P.Context(0)
    ctx.set_orbitals(w.energies, w.nocc, w.psi_grid, w.grid_dV)
    psi = w.psi_site.to("cuda")
    one = np.ones(8, dtype=np.float64)
    xyz = np.zeros((8, 3), dtype=np.float64)
    for nrad, nang in [(4097, 1), (1, 4097), (0, 26)]:
        st = P.lib.lrs_set_sites(ctx.h, 1, np.array([nrad], np.int32).ctypes.data_as(C.c_void_p),
                                 np.array([nang], np.int32).ctypes.data_as(C.c_void_p),
                                 one.ctypes.data_as(C.c_void_p), one.ctypes.data_as(C.c_void_p),
                                 xyz.ctypes.data_as(C.c_void_p), one.ctypes.data_as(C.c_void_p),
                                 C.c_void_p(psi.data_ptr()), 2)
        assert st == P.LRS_EINVAL, (nrad, nang, st)
    st = P.lib.lrs_set_sites(ctx.h, 1, np.array([8], np.int32).ctypes.data_as(C.c_void_p),
                             np.array([26], np.int32).ctypes.data_as(C.c_void_p),
                             one.ctypes.data_as(C.c_void_p), one.ctypes.data_as(C.c_void_p),
                             xyz.ctypes.data_as(C.c_void_p), one.ctypes.data_as(C.c_void_p),
                             C.c_void_p(psi.data_ptr()), 3)
    assert st == P.LRS_EINVAL                     # lmax above 2
    # a site of 50 shells (450 basis functions) is accepted for chi0 but not by the solves
    from workloads import sites as sx
    big = sx.make_site(np.zeros(3), 50, 26)
    g = torch.Generator(device="cuda").manual_seed(5)
    psi_big = torch.complex(torch.randn((1, w.energies.shape[1], big.npts), dtype=torch.float64,
                                        device="cuda", generator=g),
                            torch.randn((1, w.energies.shape[1], big.npts), dtype=torch.float64,
                                        device="cuda", generator=g))
    ctx.set_sites([big], psi_big)
    chi = torch.zeros(big.npts ** 2, dtype=torch.float64, device="cuda")
    for name, call in [("W", lambda: ctx.screen_W(chi)),
                       ("ALDA W", lambda: ctx.screen_W_alda(chi, torch.ones(big.npts, dtype=torch.float64))),
                       ("induced", lambda: ctx.induced_potential(chi))]:
        with pytest.raises(P.LrsError) as e:
            call()
        assert e.value.status == P.LRS_EUNSUPPORTED, name
    say("  size limits refused")
    ctx.close()


@pytest.mark.parametrize("nrad", [36, 48])
def test_solves_large_sites(P, nrad):
    """Sites of 36 and 48 shells x 26 directions (n = 324 and 432 basis functions: the larger
    Gauss-Jordan form, the paper's 48-shell sites) with a seeded negative semidefinite chi0
    block: W and its test-charge loss, and the induced potential (full and l = 0), against the
    oracle's solves on the same block (1e-10)."""
    from oracle import screen as sc
    from workloads import sites as sx
    site = sx.make_site(np.zeros(3), nrad, 26, r_max=6.0)
    n = site.npts
    rng = np.random.default_rng(nrad)
    B = rng.normal(size=(n, 96)) * 0.03
    chi = -(B @ B.T)
    rho = rng.normal(size=n)
    say(f"solves at {nrad} shells ({9 * nrad} basis functions, {n} points)")
    ctx = P.Context(0)
    nb = 4
    ctx.set_orbitals(np.array([[-1.0, -0.5, 0.5, 1.0]]), 2)
    psi = torch.zeros((1, nb, n), dtype=torch.complex128, device="cuda")
    ctx.set_sites([site], psi)
    chi_d = torch.as_tensor(chi.ravel(), device="cuda")
    W, loss = ctx.screen_W(chi_d, rho=torch.as_tensor(rho, device="cuda"), want_loss=True)
    Wref = sc.screen_W(chi, site)
    Lref = sc.test_charge_loss(Wref, rho, site)
    eW = rel(ctx.W_blocks(W)[0].cpu().numpy(), Wref)
    eL = abs(loss.item() / Lref - 1)
    say(f"  W {eW:.2e}, loss {eL:.2e}")
    assert eW < 1e-10 and eL < 1e-10
    for l0 in (False, True):
        rho_i, v_i = ctx.induced_potential(chi_d, q=1.0, r_shell=1.5, l0_only=l0)
        v1 = np.where(site.radii < 1.5, 1.0 / site.radii - 1.0 / 1.5, 0.0)
        rref, vref = sc.induced(chi, site, v1, 2, l0_only=l0)
        er = rel(rho_i.cpu().numpy(), rref)
        ev = rel(v_i.cpu().numpy(), vref)
        say(f"  induced (l0 {l0}): rho {er:.2e} v {ev:.2e}")
        assert er < 1e-10 and ev < 1e-10
    ctx.close()


def test_mfma_rate_probe(P):
    """The sustained matrix-core rate probe: positive and below the datasheet peak of each
    precision's unit (FP64 78.6, FP32 157.3, 16-bit 2500 TFLOP/s), a longer run takes longer,
    and bad arguments are refused."""
    say("matrix-core rate probe")
    ctx = P.Context(0)
    peak = {"fp64": 78.6, "fp32": 157.3, "bf16x2": 2500.0, "fp16x2": 2500.0, "f16f8": 2500.0}
    for prec, top in peak.items():
        ctx.mfma_rate(prec, 200)
        r1, ms1 = ctx.mfma_rate(prec, 2000)
        r2, ms2 = ctx.mfma_rate(prec, 8000)
        say(f"  {prec}: {r2:.1f} TFLOP/s ({ms2:.1f} ms for 8000 rounds, {ms1:.1f} ms for 2000)")
        assert 0 < r2 <= 1.02 * top and ms2 > 2 * ms1
    with pytest.raises(P.LrsError) as e:
        ctx.mfma_rate("fp64", 0)
    assert e.value.status == P.LRS_EINVAL
    assert P.lib.lrs_mfma_rate(ctx.h, 9, 10, None, None) == P.LRS_EINVAL
    ctx.close()
