"""Real orbitals for the real-orbital path, from a workload's complex ones.

The synthetic potential is real (time-reversal symmetry).  At Gamma the plane-wave sphere
|G|^2 <= cutoff is closed under G -> -G, so each eigenspace of H(Gamma) is closed under complex
conjugation and has a real orthonormal basis.  (At a zone-boundary k the same holds only for a
basis centred on -k, |k + G|^2 <= cutoff; the generators use one sphere for every k, so their
orbitals there have no exact real form.)  This module picks one: a phase per non-degenerate
band (psi e^{-i a/2} with a = arg sum_r psi(r)^2 over the grid), and for a degenerate set
(energies within tol) the real orthonormal vectors spanning [Re psi; Im psi] on the grid,
mapped back onto the set by its Gram matrix.  The change is unitary within each set, so the set's weights, and every
quantity built from band sums with energy-dependent weights, are unchanged.  The first array
(a full grid) fixes the change; the same change is applied to every array (site points).
"""
from __future__ import annotations

import torch


def _groups(E, tol):
    out, b, nb = [], 0, len(E)
    while b < nb:
        e = b + 1
        while e < nb and abs(E[e] - E[b]) <= tol * max(1.0, abs(E[b])):
            e += 1
        out.append((b, e))
        b = e
    return out


def realify(energies, arrays, tol=1e-8):
    """Gamma orbitals only (see above).  energies [nk, nb]; arrays: complex [nk, nb, P_i]
    tensors sampling the same orbitals, the first a full grid.  Returns (list of real float64 tensors of the same shapes, the largest
    imaginary part left relative to the largest value)."""
    nk, nb = energies.shape
    out = [torch.empty(a.shape, dtype=torch.float64, device=a.device) for a in arrays]
    left = 0.0
    for k in range(nk):
        V0 = arrays[0][k]
        # non-degenerate bands: one phase each
        z = (V0 * V0).sum(-1)
        ph = torch.exp(-0.5j * torch.angle(z))
        res = [a[k] * ph[:, None] for a in arrays]
        for b, e in _groups(energies[k], tol):
            if e - b == 1:
                continue
            V = V0[b:e]
            A = torch.cat([V.real, V.imag])
            _, _, Wh = torch.linalg.svd(A, full_matrices=False)
            W = Wh[: e - b].to(V.dtype)
            G = V @ V.conj().T
            C = (W @ V.conj().T) @ torch.linalg.inv(G)
            C = C * torch.sqrt(torch.diagonal(G).real.mean())
            for r, a in zip(res, arrays):
                r[b:e] = C @ a[k][b:e]
        for o, r in zip(out, res):
            left = max(left, float(r.imag.abs().max() / r.abs().max()))
            o[k] = r.real
        del res
    return out, left
