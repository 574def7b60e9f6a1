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
