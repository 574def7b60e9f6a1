"""GPU parity of the orbital projection (plane-wave coefficients -> orbitals at site points,
Eq. bloch, direct phase-matrix method) against the oracle's projection.

Error measure: max |gpu - ref| / max |ref| over the compared entries; bar 1e-12 (FP64 path;
the phases are reduced from arguments up to a few hundred radians, whose rounding alone is
of order 1e-14).
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import project as pj
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


def pw_inputs(w):
    """coef [nk, nb, npw] (torch, CPU), Cartesian k [nk, 3] and G [npw, 3], cell volume."""
    bd = w.bands
    coef = torch.stack([c.T.cpu() for c in bd.coef]).contiguous()
    gcart = bd.gvec * (2.0 * math.pi / bd.crystal.a)
    return coef, np.asarray(bd.kpts, dtype=np.float64), gcart, bd.crystal.omega


@pytest.mark.parametrize("name", ["tiny", "production"])
def test_projection_matches_oracle(P, name):
    """Every band and site point of the tiny (Gamma) and production (2x2x2 k, 2 sites)
    workloads; a second call gives the same bits."""
    w = workload(name, with_grid=False)
    coef, kpts, gcart, omega = pw_inputs(w)
    pts = np.concatenate([s.points() for s in w.sites])
    say(f"projection {name}: nk {coef.shape[0]} nb {coef.shape[1]} npw {coef.shape[2]} "
        f"points {len(pts)}")
    ctx = P.Context(0)
    got = ctx.project_orbitals(kpts, gcart, coef.cuda(), omega, pts)
    ref = pj.project(coef.numpy(), kpts, gcart, pts, omega)
    e = rel(got.cpu().numpy(), ref)
    say(f"  rel err {e:.2e}")
    assert e < 1e-12
    again = ctx.project_orbitals(kpts, gcart, coef.cuda(), omega, pts)
    assert torch.equal(got, again)
    ctx.close()


def test_projection_precision_sampled(P):
    """Precision workload (2x2x2 k, 2304 bands, 2897 plane waves, 3520 site points): all
    bands at 96 seeded points against the oracle, and every point against the site orbitals
    the workload was built with."""
    w = workload("precision", with_grid=False, device="cuda")
    coef, kpts, gcart, omega = pw_inputs(w)
    pts = np.concatenate([s.points() for s in w.sites])
    ctx = P.Context(0)
    torch.cuda.synchronize()
    got = ctx.project_orbitals(kpts, gcart, coef.cuda(), omega, pts)
    rng = np.random.default_rng(41)
    pick = np.sort(rng.choice(len(pts), size=96, replace=False))
    ref = pj.project(coef.numpy(), kpts, gcart, pts[pick], omega)
    e = rel(got[:, :, torch.as_tensor(pick, device="cuda")].cpu().numpy(), ref)
    e_all = rel(got.cpu().numpy(), w.psi_site.cpu().numpy())
    say(f"  precision: sampled vs oracle {e:.2e}, all points vs workload orbitals {e_all:.2e}")
    assert e < 1e-12 and e_all < 1e-12
    ctx.close()


def test_projection_edge_cases_and_errors(P):
    """One band, one point, plane-wave counts off the 16-wide chunk, points far outside the
    cell (large phases), and rejected inputs."""
    rng = np.random.default_rng(42)
    a = 9.0
    ctx = P.Context(0)
    for nb, npw, npts in [(1, 1, 1), (3, 17, 5), (70, 33, 130), (65, 100, 129)]:
        n = rng.integers(-4, 5, size=(npw, 3))
        gcart = n * (2 * math.pi / a)
        kpts = rng.uniform(-0.5, 0.5, size=(2, 3)) * (2 * math.pi / a)
        coef = torch.complex(torch.randn(2, nb, npw, dtype=torch.float64),
                             torch.randn(2, nb, npw, dtype=torch.float64))
        pts = rng.uniform(-60, 60, size=(npts, 3))
        got = ctx.project_orbitals(kpts, gcart, coef.cuda(), a ** 3, pts)
        ref = pj.project(coef.numpy(), kpts, gcart, pts, a ** 3)
        e = rel(got.cpu().numpy(), ref)
        say(f"  nb {nb} npw {npw} npts {npts}: {e:.2e}")
        assert e < 1e-12
    coef = torch.ones(1, 1, 2, dtype=torch.complex128, device="cuda")
    g = np.zeros((2, 3))
    k = np.zeros((1, 3))
    out = torch.empty(1, dtype=torch.complex128, device="cuda")
    st = P.lib.lrs_project_orbitals(ctx.h, 1, 0, 2, P._ptr(k), P._ptr(g), P._ptr(coef), 1.0, 1,
                                    P._ptr(np.zeros((1, 3))), P._ptr(out))
    assert st == P.LRS_EINVAL
    with pytest.raises(P.LrsError) as e:
        ctx.project_orbitals(k, g, coef, -1.0, np.zeros((1, 3)))
    assert e.value.status == P.LRS_EINVAL
    with pytest.raises(P.LrsError) as e:
        ctx.project_orbitals(k, g, coef, 1.0, np.full((1, 3), np.nan))
    assert e.value.status == P.LRS_ENONFINITE
    ctx.close()


# ------------------------------------------------------------------------- the FFT route
def _fft_size(m, over=4):
    """Smallest 2^a 3^b 5^c >= over * (2 m + 1) (the oversampled grid of the FFT route)."""
    n = over * (2 * m + 1)
    while True:
        k = n
        for f in (2, 3, 5):
            while k % f == 0:
                k //= f
        if k == 1:
            return n
        n += 1


def test_fft_projection_tiny_vs_oracle(P):
    """Tiny workload (Gamma, 128 bands, 251 plane waves, 208 site points) on a 32^3 grid: the
    library's FFT route against the oracle's (same grid, numpy FFT, the same cubic
    interpolation) element by element (1e-12), and against the direct sum within the derived
    interpolation bound of each band; at the grid's own points it is exact (1e-12)."""
    w = workload("tiny", with_grid=False)
    coef, kpts, gcart, omega = pw_inputs(w)
    bd = w.bands
    cell = np.eye(3) * bd.crystal.a
    gidx = bd.gvec
    N = _fft_size(int(np.abs(gidx).max()))
    pts = np.concatenate([s.points() for s in w.sites])
    say(f"FFT projection tiny: grid {N}^3, {coef.shape[1]} bands, {len(pts)} points")
    ctx = P.Context(0)
    got = ctx.project_orbitals_fft(kpts, cell, gidx, coef.cuda(), omega, pts, (N, N, N)).cpu().numpy()
    ref = pj.project_fft(coef.numpy()[:, :16], kpts, cell, gidx, pts, omega, (N, N, N))
    e = rel(got[:, :16], ref)
    direct = pj.project(coef.numpy(), kpts, gcart, pts, omega)
    bound = pj.interpolation_bound(coef.numpy()[0], gidx, (N, N, N), omega)
    err_b = np.abs(got[0] - direct[0]).max(1)
    say(f"  vs oracle FFT route {e:.2e}; vs direct max {err_b.max():.2e} "
        f"(bound {bound.max():.2e}); worst ratio {(err_b / bound).max():.2f}")
    assert e < 1e-12 and np.all(err_b <= bound)
    gp = (np.random.default_rng(3).integers(0, N, size=(40, 3)) / N) @ cell
    g_fft = ctx.project_orbitals_fft(kpts, cell, gidx, coef.cuda(), omega, gp, (N, N, N))
    g_dir = pj.project(coef.numpy(), kpts, gcart, gp, omega)
    assert rel(g_fft.cpu().numpy(), g_dir) < 1e-12
    # a different size per axis (each pass prunes to its own axis's support)
    M = int(np.abs(gidx).max())
    nf = (_fft_size(M, 3), _fft_size(M, 4), _fft_size(M, 5))
    got3 = ctx.project_orbitals_fft(kpts, cell, gidx, coef.cuda(), omega, pts, nf).cpu().numpy()
    ref3 = pj.project_fft(coef.numpy()[:, :16], kpts, cell, gidx, pts, omega, nf)
    e3 = rel(got3[:, :16], ref3)
    say(f"  grid {nf}: vs oracle FFT route {e3:.2e}")
    assert e3 < 1e-12
    ctx.close()


def test_fft_projection_long_support_and_set_orbitals_pw(P):
    """Random coefficients on every G with |m| <= 17 (a support of 35 values per axis, beyond
    what the direct-sum axis passes take, so the LDS passes run) in a sheared cell, two k-points,
    on a (36, 40, 45) grid: the library's FFT route against the oracle's element by element
    (1e-12), at random points and at points outside the cell (the grid is periodic); and the
    grid orbitals of lrs_set_orbitals_pw on a short support against the oracle's FFT grid times
    the Bloch phase at every grid point (1e-12)."""
    rng = np.random.default_rng(17)
    cell = np.array([[7.0, 0.0, 0.0], [1.5, 6.5, 0.0], [0.5, -1.0, 8.0]])
    omega = abs(np.linalg.det(cell))
    r = np.arange(-17, 18)
    m = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    gidx = m[(m ** 2).sum(1) <= 17 ** 2].astype(np.int32)
    nk, nb = 2, 3
    coef = torch.complex(torch.randn((nk, nb, len(gidx)), dtype=torch.float64,
                                     generator=torch.Generator().manual_seed(4)),
                         torch.randn((nk, nb, len(gidx)), dtype=torch.float64,
                                     generator=torch.Generator().manual_seed(5)))
    kpts = rng.normal(size=(nk, 3)) * 0.2
    frac = np.concatenate([rng.random((30, 3)), rng.random((10, 3)) * 3.0 - 1.0])
    pts = frac @ cell
    nf = (36, 40, 45)
    say(f"FFT route, long support: {len(gidx)} plane waves, grid {nf}")
    ctx = P.Context(0)
    got = ctx.project_orbitals_fft(kpts, cell, gidx, coef.cuda(), omega, pts, nf).cpu().numpy()
    ref = pj.project_fft(coef.numpy(), kpts, cell, gidx, pts, omega, nf)
    e = rel(got, ref)
    say(f"  vs oracle FFT route {e:.2e}")
    assert e < 1e-12
    ctx.close()
    # grid orbitals on a short support (direct-sum passes), the sheared cell and a non-cubic
    # grid: chi0 on the grid from lrs_set_orbitals_pw against chi0 from the oracle's FFT grid
    # times the Bloch phase, given to lrs_set_orbitals (the same site and site orbitals)
    from workloads import sites as sx
    small = gidx[(np.abs(gidx) <= 4).all(1)]
    cs = coef[:, :, :len(small)].contiguous()
    nfs = (20, 24, 27)
    E = np.array([[-1.0, 0.5, 0.9], [-0.8, 0.6, 1.1]])
    j = np.stack(np.meshgrid(*[np.arange(n) for n in nfs], indexing="ij"), -1).reshape(-1, 3)
    x = (j / np.array(nfs)) @ cell
    ref_grid = np.empty((nk, nb, len(j)), dtype=np.complex128)
    for ik in range(nk):
        ph = np.exp(1j * (x @ kpts[ik])) / np.sqrt(omega)
        for b in range(nb):
            ref_grid[ik, b] = pj.fft_grid(cs.numpy()[ik, b], small, nfs).reshape(-1) * ph
    site = sx.make_site(np.array([2.0, 2.0, 2.0]), 4, 26)
    psi_site = torch.complex(torch.randn((nk, nb, site.npts), dtype=torch.float64,
                                         generator=torch.Generator().manual_seed(6)),
                             torch.randn((nk, nb, site.npts), dtype=torch.float64,
                                         generator=torch.Generator().manual_seed(7)))
    out = []
    for use_pw in (True, False):
        c2 = P.Context(0)
        if use_pw:
            c2.set_orbitals_pw(E, 1, kpts, cell, small, cs.cuda(), omega, nfs)
        else:
            c2.set_orbitals(E, 1, torch.as_tensor(ref_grid), omega / np.prod(nfs))
        c2.set_sites([site], psi_site)
        c2.make_quadrature(P.QUAD_TIME, 16, 0.0)
        out.append(c2.chi0(-1, P.COLS_GRID, P.FP64).cpu().numpy())
        c2.close()
    eg = rel(out[0], out[1])
    say(f"  chi0 from lrs_set_orbitals_pw grid orbitals {nfs} vs the oracle's: {eg:.2e}")
    assert eg < 1e-12


def test_fft_projection_production_within_bound(P):
    """Production workload (2x2x2 k, 576 bands, 2007 plane waves, 2 sites of 800 points): the
    FFT route against the direct sum within each band's derived interpolation bound, and the
    FFT of the grid itself (lrs_set_orbitals_pw) against the workload's grid orbitals (numpy
    FFT) with chi0 on the grid from either equal to rounding."""
    w = workload("production")
    coef, kpts, gcart, omega = pw_inputs(w)
    bd = w.bands
    cell = np.eye(3) * bd.crystal.a
    gidx = bd.gvec
    N = _fft_size(int(np.abs(gidx).max()))
    pts = np.concatenate([s.points() for s in w.sites])
    say(f"FFT projection production: grid {N}^3, {len(pts)} points")
    ctx = P.Context(0)
    got = ctx.project_orbitals_fft(kpts, cell, gidx, coef.cuda(), omega, pts, (N, N, N)).cpu().numpy()
    direct = pj.project(coef.numpy(), kpts, gcart, pts, omega)
    worst = 0.0
    for k in range(coef.shape[0]):
        bound = pj.interpolation_bound(coef.numpy()[k], gidx, (N, N, N), omega)
        err_b = np.abs(got[k] - direct[k]).max(1)
        assert np.all(err_b <= bound)
        worst = max(worst, (err_b / bound).max())
    say(f"  vs direct {rel(got, direct):.2e}; worst error / bound {worst:.2f}")
    # the grid orbitals by FFT in the library, then chi0 on the grid both ways
    n = w.n_terms
    ng = w.ngrid
    ctx.set_orbitals_pw(w.energies, w.nocc, kpts, cell, gidx, coef.cuda(), omega, (ng, ng, ng))
    ctx.set_sites(w.sites, w.psi_site)
    ctx.make_quadrature(P.QUAD_TIME, n, 0.0)
    a = ctx.chi0(-1, P.COLS_GRID, P.FP64).cpu().numpy()
    ctx2 = P.Context(0)
    ctx2.set_orbitals(w.energies, w.nocc, w.psi_grid, w.grid_dV)
    ctx2.set_sites(w.sites, w.psi_site)
    ctx2.make_quadrature(P.QUAD_TIME, n, 0.0)
    b = ctx2.chi0(-1, P.COLS_GRID, P.FP64).cpu().numpy()
    say(f"  chi0 from PW-coefficient grid orbitals vs the workload's: {rel(a, b):.2e}")
    assert rel(a, b) < 1e-12
    ctx.close()
    ctx2.close()
