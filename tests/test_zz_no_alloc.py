"""GPU test of the allocation-free W solve (lrs_screen_W_noalloc) through the C ABI.

Its output is checked against lrs_screen_W's on the same inputs, and both against the oracle,
on two calls in a row (the second with a smaller site set), after an earlier call on other
sites has left the scratch array dirty.  Bars: equal to lrs_screen_W to 1e-14 of max |W| (the
same kernels on the same inputs), within 1e-11 of the oracle; sizes beyond the fixed array are
refused on the host.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import screen as sc
from workloads import blocks as bx
from workloads import sites as sx

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


def _setup(P, ctx, shapes, seed):
    """Sites of the given (n_rad, n_ang) shapes with seeded orbitals, chi0-like blocks and test
    charges (the solve reads only the site geometry from the context)."""
    rng = np.random.default_rng(seed)
    sites = [sx.make_site(rng.uniform(0, 5, 3), nr, na) for nr, na in shapes]
    npts = sum(s.npts for s in sites)
    E = np.array([[-1.0, 0.5, 0.9, 1.4]])
    psi = torch.as_tensor(rng.normal(size=(1, 4, npts)) + 1j * rng.normal(size=(1, 4, npts)))
    ctx.set_orbitals(E, 1)
    ctx.set_sites(sites, psi)
    blocks, flat = bx.chi0_like_blocks(sites, seed=seed + 100)
    rho = np.concatenate([sx.gaussian_charge(s, rng) for s in sites])
    return sites, blocks, torch.as_tensor(flat, device="cuda"), rho


def _check(P, ctx, sites, blocks, chi, rho, label):
    W1, L1 = ctx.screen_W(chi, rho=rho, want_loss=True)
    r = torch.as_tensor(rho, device="cuda")
    # outputs allocated up front; the call itself allocates nothing
    W2 = torch.full_like(W1, float("nan"))
    loss2 = torch.full_like(L1, float("nan"))
    st = P.lib.lrs_screen_W_noalloc(ctx.h, P._ptr(chi), P._ptr(W2), P._ptr(r), P._ptr(loss2))
    assert st == P.LRS_OK, P.lib.lrs_last_error(ctx.h).decode()
    torch.cuda.synchronize()
    e_w = rel(W2.cpu().numpy(), W1.cpu().numpy())
    e_l = rel(loss2.cpu().numpy(), L1.cpu().numpy())
    worst = 0.0
    for k, (site, blk) in enumerate(zip(sites, blocks)):
        ref = sc.screen_W(blk, site)
        worst = max(worst, rel(ctx.W_blocks(W2)[k].cpu().numpy(), ref))
    say(f"  {label}: vs lrs_screen_W W {e_w:.1e} loss {e_l:.1e}; vs oracle {worst:.1e}")
    assert e_w < 1e-14 and e_l < 1e-14 and worst < 1e-11


def test_noalloc_matches_screen_W_on_two_calls(P):
    ctx = P.Context(0)
    say("no-alloc W: dirty the scratch with an unrelated site set")
    sites, blocks, chi, rho = _setup(P, ctx, [(24, 50), (20, 86)], seed=3)
    W, _ = ctx.screen_W_noalloc(chi)
    say("no-alloc W: call 1, three sites up to 288 basis functions")
    sites, blocks, chi, rho = _setup(P, ctx, [(8, 26), (16, 50), (32, 110)], seed=5)
    _check(P, ctx, sites, blocks, chi, rho, "call 1")
    # the W kept for the backward pass belongs to lrs_screen_W, not to the no-alloc call
    lam0 = ctx.screen_W_backward()
    ctx.screen_W_noalloc(chi)
    assert torch.equal(lam0, ctx.screen_W_backward())
    say("no-alloc W: call 2, one smaller site")
    sites, blocks, chi, rho = _setup(P, ctx, [(8, 26)], seed=9)
    _check(P, ctx, sites, blocks, chi, rho, "call 2")
    ctx.close()


def test_noalloc_refuses_beyond_the_array(P):
    ctx = P.Context(0)
    say("no-alloc W: 40 sites of 288 basis functions exceed the 64 MiB array")
    rng = np.random.default_rng(1)
    sites = [sx.make_site(rng.uniform(0, 5, 3), 32, 26) for _ in range(40)]
    npts = sum(s.npts for s in sites)
    ctx.set_orbitals(np.array([[-1.0, 0.5]]), 1)
    ctx.set_sites(sites, torch.zeros((1, 2, npts), dtype=torch.complex128))
    dummy = torch.zeros(16, dtype=torch.float64, device="cuda")
    st = P.lib.lrs_screen_W_noalloc(ctx.h, P._ptr(dummy), P._ptr(dummy), None, None)
    assert st == P.LRS_ENOMEM
    assert "scratch" in P.lib.lrs_last_error(ctx.h).decode()
    ctx.close()
