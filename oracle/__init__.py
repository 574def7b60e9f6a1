"""Plain FP64 CPU oracle for the local real-space screening hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_2005_07834_amd``) and never imports it; the two
meet only in the seeded input generators of ``workloads``.

Modules
-------
quadrature  energy-axis quadrature rules (imaginary time; the paper's
            single-grid imaginary-frequency rule, Appendix D.1.b), written as
            separable non-negative terms c_l * alpha_l(n) * beta_l(m).
chi0        the static RPA polarizability chi0(r, r') as a brute-force sum over
            occupied x unoccupied band pairs and k-point pairs (Eq. chi1 with
            the discretised g of Sec. VI.D), with the exact energy denominator
            or with a quadrature kernel in its place.
screen      spherical-basis projection, Coulomb matrix and the dielectric solve
            W = (1 - v chi0)^-1 v of Sec. VI.E, and a test-charge loss.
grads       reference gradients of that loss with respect to band energies and
            site orbitals (exact denominators or quadrature kernel).
project     orbitals at arbitrary points from plane-wave coefficients by the phase
            matrix (Eq. bloch, the direct method of Sec. VI's projection step).
alda        the ALDA vertex: LDA f_xc by a 5-point difference, its contact matrix in the
            site basis, and W for the ALDA polarizability (Eq. chi-alda, Eq. kxc_alda).

Parity status: every function here is pinned by tests in
``tests/test_oracle_*.py`` (closed forms, invariants, brute force, finite
differences); the paper prints no synthetic worked example, so no value is
pinned to a number printed in the paper ("parity unpinned" for that kind of
check only).
"""
