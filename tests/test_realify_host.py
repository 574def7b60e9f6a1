"""Host checks of the real-orbital input preparation (workloads/realify.py) that the GPU tests
of lrs_set_orbitals_real rely on: at Gamma the real forms leave no imaginary part, are
orthonormal on the grid like the workload's orbitals, and leave chi0 (the oracle's exact band
sum, Eq. chi1) unchanged; at a zone-boundary k-point of these generators (one plane-wave
sphere for every k) no real form exists, and the check that catches it reports so."""
import numpy as np
import torch

from oracle import chi0 as cz
from tests.conftest import workload
from workloads.realify import realify


def _gram(psi, dV):
    return (psi.conj() @ psi.T) * dV


def test_realify_gamma_keeps_chi0():
    w = workload("tiny")
    (g, s), left = realify(w.energies, [w.psi_grid, w.psi_site])
    assert left < 1e-12
    G0 = _gram(w.psi_grid[0], w.grid_dV)
    G1 = _gram(g[0].to(torch.complex128), w.grid_dV)
    assert float((G1 - G0).abs().max()) < 1e-12
    rng = np.random.default_rng(3)
    rows = rng.integers(0, w.nrows, 24)
    cols = rng.integers(0, w.ngrid ** 3, 24)
    a = cz.chi0_exact_entries(w.psi_site[:, :, rows].numpy(), w.psi_grid[:, :, cols].numpy(),
                              w.energies, w.nocc)
    b = cz.chi0_exact_entries(s[:, :, rows].numpy().astype(complex),
                              g[:, :, cols].numpy().astype(complex), w.energies, w.nocc)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


def test_realify_reports_zone_boundary_orbitals():
    w = workload("production")
    _, left = realify(w.energies, [w.psi_grid, w.psi_site])
    assert left > 1e-3
