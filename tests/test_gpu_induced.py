"""GPU parity of the induced density and potential of a spherical perturbation (the
short-range part of a potential split by a shell of charge) against the oracle, full response
and the l = 0 response.

Error measure: max |gpu - ref| / max |ref|; bar 1e-10 with the library's FP64 chi0 against
the oracle's chi0 of the same quadrature, 1e-11 when both start from the same seeded
chi0-like blocks.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import chi0 as cz
from oracle import quadrature as q
from oracle import screen as sc
from tests.conftest import workload
from workloads import blocks as bx

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


def scale_for(w, n):
    mu = q.mid_gap(w.energies, w.nocc)
    x, y = q.offsets(w.energies, w.nocc, mu)
    return q.auto_scale(x, y, n)


@pytest.mark.parametrize("name", ["tiny", "production"])
def test_induced_vs_oracle(P, name):
    """The shell-partitioned point perturbation (q = 1, R_S = 1.2 bohr) and an explicit v1
    profile, full and l = 0 response, at every site; chi0 from the library (FP64) and from
    the oracle (same quadrature)."""
    w = workload(name, with_grid=False)
    n = w.n_terms
    s = scale_for(w, n)
    ctx = P.Context(0)
    ctx.set_orbitals(w.energies, w.nocc, None, w.grid_dV)
    ctx.set_sites(w.sites, w.psi_site)
    ctx.make_quadrature(P.QUAD_TIME, n, s)
    chi = ctx.chi0(-1, P.COLS_SITE, P.FP64)
    ps = w.psi_site.numpy()
    terms = cz.terms_for(w.energies, w.nocc, "time", n, s)
    offs = w.site_offsets
    prof = np.concatenate([np.exp(-x.radii) / x.radii for x in w.sites])
    for v1 in (None, prof):
        for l0 in (False, True):
            rho, vind = ctx.induced_potential(chi, v1=v1, q=1.0, r_shell=1.2, l0_only=l0)
            rho, vind = rho.cpu().numpy(), vind.cpu().numpy()
            o, ro = 0, 0
            er = ev = 0.0
            for k, site in enumerate(w.sites):
                sl = slice(offs[k], offs[k + 1])
                ref_chi = cz.chi0_quad(ps[:, :, sl], ps[:, :, sl], w.nocc, 2, *terms)
                v1s = (sc.shell_potential(site.radii, 1.0, 1.2) if v1 is None
                       else prof[ro:ro + site.n_rad])
                r_ref, v_ref = sc.induced(ref_chi, site, v1s, l0_only=l0)
                nb = len(r_ref)
                er = max(er, rel(rho[o:o + nb], r_ref))
                ev = max(ev, rel(vind[o:o + nb], v_ref))
                o += nb
                ro += site.n_rad
            say(f"  {name} v1={'shell' if v1 is None else 'profile'} l0={l0}: rho {er:.2e} "
                f"v_ind {ev:.2e}")
            assert er < 1e-10 and ev < 1e-10
    ctx.close()


def test_induced_uneven_sites(P):
    """Batching workload (64 sites, 208..3520 points, n up to 288): the library's batched
    solve and the oracle's on the same seeded chi0-like blocks (workloads.blocks), at every
    site."""
    w = workload("batching", with_grid=False, device="cuda")
    ctx = P.Context(0)
    ctx.set_orbitals(w.energies, w.nocc, None, w.grid_dV)
    ctx.set_sites(w.sites, w.psi_site)
    blocks, flat = bx.chi0_like_blocks(w.sites, seed=12)
    chi = torch.as_tensor(flat, device="cuda")
    rho, vind = ctx.induced_potential(chi, q=0.7, r_shell=1.5)
    rho, vind = rho.cpu().numpy(), vind.cpu().numpy()
    nbas = [9 * x.n_rad for x in w.sites]
    bo = np.cumsum([0] + nbas)
    worst = 0.0
    for k, site in enumerate(w.sites):
        r_ref, v_ref = sc.induced(blocks[k], site, sc.shell_potential(site.radii, 0.7, 1.5))
        er = rel(rho[bo[k]:bo[k + 1]], r_ref)
        ev = rel(vind[bo[k]:bo[k + 1]], v_ref)
        worst = max(worst, er, ev)
    say(f"  64 sites: worst rho / v_ind error {worst:.2e}")
    assert worst < 1e-11
    with pytest.raises(P.LrsError) as e:
        ctx.induced_potential(chi, v1=np.full(sum(x.n_rad for x in w.sites), np.nan))
    assert e.value.status == P.LRS_ENONFINITE
    with pytest.raises(P.LrsError) as e:
        ctx.induced_potential(chi, q=1.0, r_shell=0.0)
    assert e.value.status == P.LRS_EINVAL
    ctx.close()


def test_valence_W_vs_oracle(P):
    """Valence W(x, x') within r_m (Sec. V.A, Eq. rpa-val) on 27 grid-point sites of a 3 x 3 x 3
    patch of the tiny cell's 16^3 grid (16 shells x 26 directions each, seeded chi0-like
    blocks), periodic images on: against the oracle element by element (bar 1e-11), for
    eps_inf 1 and 4; the bare limit (chi0 = 0) gives 1/|x - x'| and 6/(5 R_x) on the diagonal."""
    from oracle import valence as va
    from workloads import blocks as bx
    from workloads import sites as sx
    a, ng = 10.0, 16
    h = a / ng
    idx = np.array([[i, j, k] for i in (15, 0, 1) for j in (15, 0, 1) for k in (15, 0, 1)])
    centres = idx * h
    sites = [sx.make_site(c, 16, 26, r_max=2.0, r_min=0.05) for c in centres]
    blocks, flat = bx.chi0_like_blocks(sites, seed=13)
    cell = np.eye(3) * a
    vx = a ** 3 / ng ** 3
    R_S, r_m = 1.5, 1.5
    rng = np.random.default_rng(2)
    psi = torch.as_tensor(rng.normal(size=(1, 4, sum(s.npts for s in sites)))
                          + 1j * rng.normal(size=(1, 4, sum(s.npts for s in sites))))
    ctx = P.Context(0)
    ctx.set_orbitals(np.array([[-1.0, 0.5, 0.9, 1.4]]), 1)
    ctx.set_sites(sites, psi)
    chi = torch.as_tensor(flat, device="cuda")
    for eps_inf in (1.0, 4.0):
        say(f"valence W: 27 sites, eps_inf {eps_inf}")
        got = ctx.valence_W(chi, centres, vx, R_S, eps_inf, r_m, cell).cpu().numpy()
        ref = va.valence_W(blocks, sites, centres, vx, R_S, eps_inf, r_m, cell)
        e = rel(got, ref)
        npairs = int((ref != 0).sum()) - len(sites)
        say(f"  vs oracle {e:.2e} ({npairs} pairs within r_m)")
        assert e < 1e-11 and np.array_equal(got, got.T) and npairs > 100
        assert np.array_equal(got == 0, ref == 0)
    zero = torch.zeros_like(chi)
    W0 = ctx.valence_W(zero, centres, vx, R_S, 1.0, r_m, cell).cpu().numpy()
    R_x = (3 * vx / (4 * np.pi)) ** (1 / 3)
    assert np.abs(np.diag(W0) - 6 / (5 * R_x)).max() < 1e-13 * 6 / (5 * R_x)
    # sites 0 and 1 (grid indices (15, 15, 15) and (15, 15, 0)) are neighbours through the
    # cell boundary, one grid step apart
    assert abs(W0[0, 1] - 1 / h) < 1e-13
    with pytest.raises(P.LrsError) as e:
        ctx.valence_W(chi, centres, vx, R_S, 1.0, 2.5, cell)      # r_m beyond the shells
    assert e.value.status == P.LRS_EINVAL
    ctx.close()
