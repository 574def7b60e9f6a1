/*
 * lrs.h -- C ABI of the local real-space screening library for MI355X (gfx950).
 *
 * The library computes the static RPA independent-particle polarizability
 * chi0(r, r') between the points r of one or more sites and a column point set
 * (the cell's real-space grid, or the site's own points), summed over
 * k-points and occupied x unoccupied band pairs (Eq. chi1 with the
 * k-discretised Green's function of Sec. VI.D), and the per-site screened
 * Coulomb interaction W = (1 - v chi0)^-1 v in a radial x real-Y_lm basis
 * (Sec. VI.E, Eqs. reducible and W), plus the adjoints of both.
 *
 * The energy denominator is replaced by a quadrature along the imaginary energy
 * axis (Appendix D.1.b) written as non-negative separable terms
 *     1/(e_m - e_n) ~= sum_l c_l alpha_l(n) beta_l(m),
 * so that, with the weighted Green's functions
 *     G_o^l(r,r') = sum_{k, n occ}   psi_nk*(r) alpha_l(nk) psi_nk(r')
 *     G_u^l(r,r') = sum_{k, m unocc} psi_mk*(r) beta_l(mk)  psi_mk(r'),
 *     chi0(r,r') = -(2 s / N_k^2) sum_l c_l Re[ G_o^l(r,r') conj(G_u^l(r,r')) ].
 * The two Green's functions are dense complex contractions over bands and run
 * on the matrix cores; the Hadamard product is fused into their epilogue.
 *
 * Conventions
 *  - Every pointer named *_host is host memory; every other array pointer is
 *    device memory on the context's device.  Complex arrays are complex128
 *    (interleaved re, im doubles).
 *  - Calls enqueue work on the context's HIP stream and return without
 *    synchronising unless stated; results are valid after the stream is
 *    synchronised.  Inputs may be freed by the caller once the call returned
 *    and the stream has been synchronised (the library keeps packed copies).
 *  - Outputs are overwritten, never accumulated into.
 *  - Errors are return codes; no exception or abort crosses the ABI.  Every
 *    host-checkable input condition is checked before any work is enqueued,
 *    so a call that fails leaves the context and all outputs unchanged.
 *    lrs_last_error() gives a message for the last failed call on a context.
 *  - One context per stream; a context is not re-entrant.
 *  - Site points are ordered radial-major inside a site (p = i * n_ang + a,
 *    position centre + r_i * Omega_a) and sites are concatenated.
 *  - The W basis index of a site is (L, i), L-major: idx = L * n_rad + i,
 *    L = l*l + l + m, with the real spherical harmonics
 *      Y_00 = 1/(2 sqrt(pi)); Y_1,-1 = c1 y, Y_10 = c1 z, Y_11 = c1 x, c1 = sqrt(3/(4 pi));
 *      Y_2,-2 = c2 x y, Y_2,-1 = c2 y z, Y_20 = c20 (3z^2 - 1), Y_21 = c2 x z,
 *      Y_22 = c2/2 (x^2 - y^2), c2 = sqrt(15/(4 pi)), c20 = sqrt(5/(16 pi)).
 */
#ifndef LRS_H
#define LRS_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lrs_ctx lrs_ctx;

typedef enum {
  LRS_OK = 0,
  LRS_EINVAL = 1,        /* bad argument, shape or pointer */
  LRS_ENOMEM = 2,        /* device allocation failed or would exceed LRS_MAX_BYTES */
  LRS_EDEVICE = 3,       /* HIP runtime error, or no gfx950 device */
  LRS_ESTATE = 4,        /* call out of order (e.g. chi0 before orbitals) */
  LRS_ENOGAP = 5,        /* some occupied energy is not below every unoccupied one */
  LRS_ENONFINITE = 6,    /* NaN or Inf in an input */
  LRS_EUNSUPPORTED = 7   /* valid request the library does not implement */
} lrs_status;

typedef enum {
  LRS_FP64 = 0,     /* FP64 matrix-core products, FP64 accumulation */
  LRS_FP32 = 1,     /* FP32 matrix-core products, FP32 accumulation of G */
  LRS_BF16X2 = 2,   /* each operand split into bf16 hi + lo; hi*hi + hi*lo + lo*hi, FP32 accumulation */
  LRS_FP16X2 = 3,   /* the same with fp16 halves (operands prescaled by powers of two) */
  LRS_F16F8 = 4,    /* fp16 hi + lo split: hi*hi on fp16 matrix cores, the cross terms hi*lo +
                       lo*hi on block-scaled fp8 (e4m3) ones, FP32 accumulation; two thirds of
                       the split paths' matrix-core time, relative error of order 1e-6 */
  LRS_FP64_3M = 5   /* FP64 with three real products per complex one (the 3M form:
                       p b_r, q b_i and (p - q)(b_r + b_i) give G_r and G_i) instead of four;
                       forward chi0 only (lrs_compute_chi0) */
} lrs_precision;

typedef enum {
  LRS_COLS_GRID = 0,   /* columns = the cell grid given to lrs_set_orbitals */
  LRS_COLS_SITE = 1    /* columns = the same site's points (site x site blocks) */
} lrs_colset;

typedef enum {
  LRS_QUAD_TIME = 0,   /* imaginary time: Gauss-Legendre on (0,1), tau = C a/(1-a) */
  LRS_QUAD_FREQ = 1    /* the paper's single-grid imaginary-frequency rule, 2 terms per node */
} lrs_quad_kind;

/* Version string of the library build. */
const char* lrs_version(void);

/* Creates a context on HIP device `device`, enqueuing on `hip_stream` (a hipStream_t;
 * NULL = the legacy default stream).  Fails with LRS_EDEVICE if the device is not
 * gfx950 or cannot be initialised.  *ctx is set to NULL on failure.  If the environment
 * variable LRS_MAX_BYTES holds a byte count when the context is created, the context's own
 * device allocations are kept at or below it: a call that would pass it fails with
 * LRS_ENOMEM and leaves the context usable (caller-owned buffers do not count). */
lrs_status lrs_create(lrs_ctx** ctx, int device, void* hip_stream);

/* Synchronises the context's stream and frees every device buffer the context owns. */
void lrs_destroy(lrs_ctx* ctx);

/* Message of the last failed call on ctx ("" if none).  Valid until the next call. */
const char* lrs_last_error(const lrs_ctx* ctx);

/* Host-only validation of a band set, usable without a device: nk >= 1,
 * 1 <= nocc < nb, finite energies, and a global gap:
 * min over k of e[k][nocc] > max over k of e[k][nocc-1], with mu (if given) inside it.
 * The side of mu decides occupation (Sec. VI.D) and the lowest nocc bands are the occupied
 * ones at every k, so a set without such a gap is LRS_ENOGAP with delta == 0 and
 * LRS_EUNSUPPORTED with delta > 0 (a metal whose occupied count changes with k).  Returns
 * the status lrs_set_orbitals would return for these energies. */
lrs_status lrs_check_bands(int nk, int nb, int nocc, const double* energies_host, double mu,
                           double delta);

/* Band energies and the grid orbitals (Sec. VI.A-D).
 *   energies_host  [nk][nb] float64, Ha; the lowest nocc bands at every k are occupied.
 *   mu             chemical potential; NaN = middle of the global gap (Sec. VI.D).
 *                  It must lie strictly inside the gap.
 *   delta          metallic regularisation of Sec. VI.D: every offset mu - e keeps its sign and
 *                  takes delta in quadrature, mu - e -> +-sqrt((mu - e)^2 + delta^2) (0 = off).
 *                  Every occupied band must still lie below mu and every other band above it
 *                  (lrs_check_bands).
 *   spin_factor    s in the prefactor -2 s / N_k^2 (2 for a closed shell, 1 per spin channel).
 *   psi_grid       complex128 [nk][nb][ngrid] on the device, or NULL with ngrid = 0.
 *   grid_dV        volume element of the grid (kept for the caller; not used by chi0).
 * Packs psi_grid into the library's operand layouts (FP64 copy kept; reduced-precision
 * copies are made on first use).  Synchronises the stream to check finiteness
 * (LRS_ENONFINITE).  Invalidates sites, quadrature and cached plans. */
lrs_status lrs_set_orbitals(lrs_ctx* ctx, int nk, int nb, int nocc, int spin_factor,
                            const double* energies_host, double mu, double delta,
                            const void* psi_grid, int ngrid, double grid_dV);

/* lrs_set_orbitals for real orbitals (Sec. VI.F, the Gamma point): with a real potential
 * (time-reversal symmetry, no spin-orbit coupling) the Gamma orbitals can be chosen real (a
 * phase per band, a real basis of each degenerate set); so can those at the other k-points
 * equal to their own negatives modulo the reciprocal lattice (the zone-boundary points of a
 * Gamma-centred 2 x 2 x 2 grid, Bloch factors +-1) when their plane-wave basis is centred on
 * -k.  Any nk is accepted: chi0 is computed for the real orbitals given.  Each Green's
 * function is then a real contraction, G = sum_K w_K psi_K(r) psi_K(r'), one real product
 * where the complex form takes four.  Arguments as lrs_set_orbitals; psi_grid complex128 [nk][nb][ngrid] whose imaginary
 * parts vanish (at most 1e-12 of the largest real part, else LRS_EINVAL; only the real parts
 * are read).  The operands hold two real orbitals per slot, so they take half the memory.
 * lrs_set_sites then requires real psi_site the same way.  lrs_compute_chi0 supports LRS_FP64
 * and LRS_F16F8 on real orbitals (others: LRS_EUNSUPPORTED), every column set and both rules;
 * the W solves are unchanged.  lrs_compute_chi0_backward runs in LRS_F16F8 only, from the
 * Green's functions an LRS_F16F8 lrs_compute_chi0 over every site block kept (else
 * LRS_EUNSUPPORTED); the real parts of dL_dpsi_site are then the gradient with respect to the
 * real orbitals (the imaginary parts, zero for the static terms, are the derivatives with
 * respect to imaginary parts of the orbitals).  A later lrs_set_orbitals returns the context to
 * complex orbitals. */
lrs_status lrs_set_orbitals_real(lrs_ctx* ctx, int nk, int nb, int nocc, int spin_factor,
                                 const double* energies_host, double mu, double delta,
                                 const void* psi_grid, int ngrid, double grid_dV);

/* Site geometry and the orbitals at the site points.
 *   nrad_host, nang_host  [nsites] shell and angular-point counts; npts_s = nrad * nang.
 *   radii_host, rad_w_host [sum nrad]  radii r_i and radial weights u_i (~ r_i^2 dr).
 *   ang_xyz_host  [sum nang][3] unit vectors; ang_w_host [sum nang] weights (sum 4 pi).
 *   psi_site      complex128 [nk][nb][sum npts_s] on the device (same nk, nb as the orbitals).
 *   lmax          angular cut-off of the W basis, 0 <= lmax <= 2.
 * Requires lrs_set_orbitals first (LRS_ESTATE).  Synchronises the stream. */
lrs_status lrs_set_sites(lrs_ctx* ctx, int nsites, const int* nrad_host, const int* nang_host,
                         const double* radii_host, const double* rad_w_host,
                         const double* ang_xyz_host, const double* ang_w_host,
                         const void* psi_site, int lmax);

/* Generic quadrature terms: c_host [nterms] > 0, alpha_host [nterms][nk][nocc] >= 0,
 * beta_host [nterms][nk][nb-nocc] >= 0, 1 <= nterms <= 128.  The backward pass
 * is unavailable with generic terms (no derivative is known). */
lrs_status lrs_set_quadrature(lrs_ctx* ctx, int nterms, const double* c_host,
                              const double* alpha_host, const double* beta_host);

/* Builds terms from the current energies (Appendix D.1.b):
 *   LRS_QUAD_TIME: nnodes Gauss-Legendre nodes a_j, w_j on (0,1);
 *     tau_j = C a_j/(1-a_j), c_j = C w_j/(1-a_j)^2, alpha = exp(-x tau), beta = exp(-y tau),
 *     x = mu - e_occ, y = e_unocc - mu.  scale > 0 sets C; scale <= 0 picks
 *     C = kappa / sqrt(Dmin Dmax), kappa = 10^(j/40) (j = -80..100) minimising the worst
 *     relative error of sum_j c_j exp(-D tau_j) against 1/D over 512 log-spaced D in
 *     [Dmin, Dmax] (the smallest kappa on ties).
 *   LRS_QUAD_FREQ: t_j = zeta a_j/(1-a_j), c_j = zeta w_j/(pi (1-a_j)^2); the integrand is
 *     folded to t > 0 (its value at -t is the conjugate of that at +t), giving two terms per
 *     node with alpha, beta = x/(x^2+t^2) and t/(x^2+t^2).  scale > 0 sets zeta, else zeta is
 *     the geometric mean of the smallest and largest |mu - e| (0.5 eV added in quadrature
 *     to the smallest when delta > 0).
 * 1 <= nnodes <= 64.  Node positions and mu are constants under differentiation. */
lrs_status lrs_make_quadrature(lrs_ctx* ctx, int kind, int nnodes, double scale);

/* The imaginary-time rule for chi0 at imaginary frequency i omega (omega >= 0, Ha; the
 * dynamic extension of Eq. chi1 on the same contour).  Each occupied x unoccupied pair then
 * needs (Delta + i omega) / (Delta^2 + omega^2) = int_0^inf e^{i omega tau} e^{-Delta tau} dtau,
 * so the terms of lrs_make_quadrature(LRS_QUAD_TIME) take complex coefficients
 * c e^{i omega tau} and lrs_compute_chi0 accumulates Re[c e^{i omega tau} G_o o conj(G_u)]:
 *   chi0(i omega) = -(2s/N_k^2) sum [Delta Re P - omega Im P] / (Delta^2 + omega^2).
 * The scale (scale <= 0: automatic) minimises the rule's worst relative error on
 * Delta / (Delta^2 + omega^2) over the gap range; the rule loses accuracy once omega tau
 * oscillates within the decay of e^{-Delta tau} (omega well above the smallest gap).
 * Site x site blocks of chi0(i omega) are not symmetric (the odd part); they are computed
 * tile by tile over the whole block, and lrs_compute_chi0_backward differentiates them (mu,
 * omega and the nodes held fixed).  omega = 0 gives exactly
 * lrs_make_quadrature(LRS_QUAD_TIME, ...). */
lrs_status lrs_make_quadrature_iw(lrs_ctx* ctx, int nnodes, double scale, double omega);

/* The imaginary-time rule of lrs_make_quadrature(LRS_QUAD_TIME) with the node count picked from
 * the band-energy range: the smallest n in [nmin, nmax] (1 <= nmin <= nmax <= 64) whose rule,
 * at its automatic scale, keeps the worst relative error of sum_j c_j exp(-D tau_j) against 1/D
 * at or below tol over 512 log-spaced D in [Dmin, Dmax] (every band pair's denominator lies in
 * that range); nmax when none does.  One node set serves every k (cross-k pairs need a common
 * tau).  Writes the chosen n and its error to *nnodes_host and *err_host (either may be NULL).
 * LRS_EINVAL for tol <= 0 or a bad range. */
lrs_status lrs_make_quadrature_tol(lrs_ctx* ctx, double tol, int nmin, int nmax, int* nnodes_host,
                                   double* err_host);

/* Reads back the terms in use: c_host [nterms], tau_host [nterms] (tau for LRS_QUAD_TIME,
 * t for LRS_QUAD_FREQ, 0 for generic), mu and the time scale C / zeta (may be NULL). */
lrs_status lrs_get_quadrature(const lrs_ctx* ctx, int* nterms, double* c_host, double* tau_host,
                              double* mu_host, double* scale_host);

/* Orbitals at arbitrary points from plane-wave coefficients (Sec. VI, projecting the wave
 * functions; Eq. bloch): psi_bk(r) = Omega^-1/2 sum_G C_bk(G) exp(i (k+G).r), by the direct
 * method: per k the phase matrix P_k(r, G) = exp(i (k+G).r), then psi_k = C_k P_k^T as a
 * complex FP64 GEMM on the matrix cores.
 *   kpts_host    float64 [nk][3], Cartesian k (bohr^-1)
 *   gvec_host    float64 [npw][3], Cartesian G (bohr^-1)
 *   coef         complex128 [nk][nb][npw] on the device: C_bk(G), unit norm over the cell
 *   omega        cell volume (bohr^3)
 *   points_host  float64 [npts][3], Cartesian (bohr)
 *   psi_out      complex128 [nk][nb][npts] on the device, the layout lrs_set_sites takes.
 * Uses only the context's device and stream (no orbitals, sites or terms need be set).
 * Its workspace stays with the context (allocated or grown only when a call needs more); it
 * copies its host tables once and synchronises at the end: LRS_ESTATE under stream capture.
 * LRS_EINVAL for non-positive sizes or omega, LRS_ENONFINITE for non-finite k, G or points,
 * LRS_ENOMEM if the workspace (16 B x (nb + npts) x npw, padded) does not fit. */
lrs_status lrs_project_orbitals(lrs_ctx* ctx, int nk, int nb, int npw, const double* kpts_host,
                                const double* gvec_host, const void* coef, double omega,
                                int npts, const double* points_host, void* psi_out);

/* The same orbitals by the FFT route of that section: per band, C_bk(G) placed at its Miller
 * indices m mod N in a zeroed N0 x N1 x N2 box and inverse-transformed (unnormalised, a
 * hand-written mixed-radix FFT), u_bk(x_j) = sum_G C exp(i G.x_j) on the grid
 * x_j = sum_d (j_d / N_d) a_d; then cubic Lagrange interpolation at each point over the 4 x 4 x 4
 * grid nodes around it (the interpolants computed once per point, reused for every band and k)
 * and the Bloch phase: psi_bk(r) = exp(i k.r) u_bk(r) / sqrt(Omega).  The interpolation error of
 * a plane wave with phase step theta per grid spacing is of order theta^4 / 40 per dimension, so
 * the grid should oversample the plane-wave sphere (N_d of about 4 (2 max|m_d| + 1) for 10^-3 on
 * the largest G).
 *   cell_host   float64 [3][3], lattice vectors a_d as rows (bohr); |det| must equal omega
 *   gidx_host   int32 [npw][3], Miller indices m of the plane waves (G = sum_d m_d b_d)
 *   nfft_host   int32 [3], the FFT grid N_d: 2^a 3^b 5^c, at most 128, N_d > 2 max |m_d|
 *   the other arguments as lrs_project_orbitals.
 * LRS_EUNSUPPORTED for a grid size outside those; synchronises (host tables); LRS_ESTATE under
 * stream capture. */
lrs_status lrs_project_orbitals_fft(lrs_ctx* ctx, int nk, int nb, int npw, const double* kpts_host,
                                   const double* cell_host, const int* gidx_host, const void* coef,
                                   double omega, const int* nfft_host, int npts,
                                   const double* points_host, void* psi_out);

/* lrs_set_orbitals from plane-wave coefficients: the grid orbitals are made on the device by
 * the FFT of lrs_project_orbitals_fft on the ngrid_host[0] x [1] x [2] grid (C order, j2
 * fastest; x_j = sum_d (j_d / N_d) a_d) with the Bloch phase, then packed as by
 * lrs_set_orbitals with grid_dV = omega / (N0 N1 N2).  coef complex128 [nk][nb][npw] on the
 * device; the other arguments as lrs_set_orbitals and lrs_project_orbitals_fft.  Allocates the
 * grid orbitals for the call (nk nb N0 N1 N2 x 16 bytes) and synchronises. */
lrs_status lrs_set_orbitals_pw(lrs_ctx* ctx, int nk, int nb, int nocc, int spin_factor,
                               const double* energies_host, double mu, double delta,
                               const double* kpts_host, const double* cell_host,
                               const int* gidx_host, const void* coef, int npw, double omega,
                               const int* ngrid_host);

/* chi0 for one site (site >= 0) or all sites concatenated (site = -1), in precision prec.
 *   LRS_COLS_GRID: chi0_out float64 [rows][ngrid], rows = npts of the site (or all sites).
 *   LRS_COLS_SITE: chi0_out float64 site blocks [npts_s][npts_s], concatenated over sites.
 * chi0 is real for the static case, so float64 is returned.  Asynchronous.
 * All sites and terms go into one persistent launch per operand batch (a batch holds as many
 * sites' weighted operands as fit LRS_SITE_OPERAND_BYTES, default 24 GiB).  The workgroups of
 * each XCD wait for each other at every term start (a bounded wait of at most about 0.5 ms),
 * so that they share operand panels in that XCD's L2; LRS_XCD_SYNC=0 turns this off, which
 * suits launches that share the GPU with other kernels.
 * Graph capture: once a call has run on a problem (same site, column set and precision), the
 * same call may be captured on the context's stream (e.g. into a HIP graph); under capture it
 * records kernels only (the weighted site operand's preparation included, so a replay does not
 * depend on what the operand buffer holds), records no timing event, and returns LRS_ESTATE
 * instead of allocating or building a plan.  A successful capture pins the context: the graph
 * holds the addresses of its buffers (orbital operands, weights, term coefficients, tile
 * lists, the site operand and the per-workgroup scratch), so until lrs_release_graphs
 * lrs_set_orbitals, lrs_set_sites, lrs_set_quadrature, lrs_make_quadrature(_iw, _tol) and any
 * call that would have to replace one of those buffers with a larger one (chi0 in another
 * precision or column set, the backward pass, lrs_tune) return LRS_ESTATE; eager calls that
 * fit the existing buffers, the solves of lrs_screen_W and friends, and replays stay valid.
 * lrs_destroy frees the buffers regardless: destroy the graphs first. */
lrs_status lrs_compute_chi0(lrs_ctx* ctx, int site, int cols, int prec, double* chi0_out);

/* Unpins the context (see lrs_compute_chi0): the caller declares that no graph captured from
 * this context's calls will be replayed again. */
lrs_status lrs_release_graphs(lrs_ctx* ctx);

/* Per-site dielectric solve from site x site chi0 blocks (layout of LRS_COLS_SITE, all sites):
 *   X = P chi0 P^T (P_{(L,i),(i',a)} = delta_ii' w_a Y_L(a)), V_L = 4 pi/(2l+1) r_<^l / r_>^(l+1),
 *   D = diag(u_i), eps = I - V D X D, W = eps^-1 V (LU with partial pivoting, FP64).
 *   W_out      float64 [nsites][n][n] with n = (lmax+1)^2 * n_rad of each site, concatenated.
 *   rho_test   optional float64 [sum npts] test charge at the site points (NULL = none).
 *   loss_out   optional float64 [nsites]: rho_L^T D W D rho_L, rho_L = P rho (needs rho_test).
 * Keeps W (and rho_test) for lrs_screen_W_backward.  Asynchronous.  LRS_EUNSUPPORTED when a
 * site has more than 448 basis functions (n_rad > 49 at lmax 2) or 256 directions. */
lrs_status lrs_screen_W(lrs_ctx* ctx, const double* chi0_sitesite, double* W_out,
                        const double* rho_test, double* loss_out);

/* lrs_screen_W for callers that cannot allocate device memory (code under graph capture
 * elsewhere in the process, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results (W_out, and loss_out when rho_test is given), with the solve's tables and
 * workspace in a fixed device array of 64 MiB that each GPU holds until the process ends, so the
 * call allocates and frees nothing.  The caller passes inputs and outputs as for lrs_screen_W.
 * LRS_ENOMEM when the sites need more scratch than the array holds (3 n^2 + n doubles per site
 * plus the tables, so up to about 100 sites of 288 basis functions or 40 of 448),
 * LRS_EUNSUPPORTED beyond
 * the solve's limits as lrs_screen_W.  It keeps no state for lrs_screen_W_backward.  It copies
 * host tables into the array and synchronises the stream: LRS_ESTATE under stream capture.
 * Every call on one GPU shares that GPU's array, which keeps the last call's contents: calls
 * that overlap on one GPU (other streams, other contexts, other threads) race. */
lrs_status lrs_screen_W_noalloc(lrs_ctx* ctx, const double* chi0_sitesite, double* W_out,
                                const double* rho_test, double* loss_out);

/* Induced density and potential of a spherical perturbation at every site (Sec. VI,
 * construction of chi and W; the perturbation is the short-range part of a potential split by
 * a shell of charge, Eq. partition).  With X, V, D of lrs_screen_W and v1 in the L = 00
 * channel (its Y_00 coefficient sqrt(4 pi) v1(r_i)):
 *   rho = (I - X D V D)^-1 X D v1 (= chi v1),   v_ind = V D rho,
 * computed per site as y = (I - V D X D)^-1 v1 (Gauss-Jordan, FP64), rho = X D y,
 * v_ind = y - v1.  l0_only != 0 keeps the 00;00 block alone (the paper's default l = 0
 * response); rho and v_ind are then zero outside L = 00.
 *   chi0_sitesite  site blocks (layout of LRS_COLS_SITE, all sites), device
 *   v1_host        float64 [sum n_rad], each site's radial values in site order; or NULL for
 *                  the short-range part of q/|r - centre| split at the shell radius r_shell:
 *                  q (1/r - 1/r_shell) for r < r_shell, 0 beyond
 *   rho_out, v_out float64 [sum n], n = (lmax+1)^2 n_rad per site, L-major, device.
 * Requires lrs_set_sites.  Synchronous in its host part; LRS_ESTATE under stream capture,
 * LRS_EUNSUPPORTED when a site has more than 448 basis functions or 256 directions. */
lrs_status lrs_induced_potential(lrs_ctx* ctx, const double* chi0_sitesite, const double* v1_host,
                                 double q, double r_shell, int l0_only, double* rho_out,
                                 double* v_out);

/* Valence screened interaction W(x, x') within r_m (Sec. V.A, Eq. rpa-val): the sites are grid
 * points x (centres_host [nsites][3], bohr), each screening a unit charge spread uniformly over
 * a sphere of the grid's discretisation volume vx = Omega / N_x (radius R_x = (3 vx/4 pi)^(1/3)),
 * potential v_ext = (3 - r^2/R_x^2)/(2 R_x) inside, 1/r outside.  The shell of charge at r_shell
 * splits it (Eq. partition) into v1 = v_ext - v2 and v2 = 1/r_shell inside, 1/r outside; v1 is
 * screened by the local RPA response of the site (the solve of lrs_induced_potential, l <= lmax
 * response to v1 in the L = 00 channel), v2 by the long-wavelength limit of the model, 1/eps_inf
 * (eps_inf = 1: bare).  With v_ind,L the induced potential's radial functions on the site's
 * shells, read at |d| by cubic Lagrange interpolation over the four nearest shells:
 *   W^[x](x + d) = v_ext(|d|) + sum_L v_ind,L(|d|) Y_L(d/|d|) - (1 - 1/eps_inf) v2(|d|)
 *   W_out[x][x'] = (W^[x](x') + W^[x'](x)) / 2   for 0 < |d| <= r_m (d = x' - x, nearest image)
 *   W_out[x][x]  = (3/R_x^3) int_0^R_x W^[x]_00(r) r^2 dr  (the l = 0 part over the
 *                  discretisation sphere: 6/(5 R_x) for the bare sphere, the induced part by
 *                  8-point Gauss-Legendre on [0, R_x])
 *   W_out[x][x'] = 0 beyond r_m (the paper's HLL model there is outside this library).
 *   chi0_sitesite  site blocks (layout of LRS_COLS_SITE, all sites), device
 *   cell_host      lattice vectors [3][3] (rows, bohr) for the nearest periodic image (by
 *                  rounding fractional coordinates: exact while r_m is below half the smallest
 *                  cell height), or NULL for plain differences
 *   W_out          float64 [nsites][nsites], device; exactly symmetric.
 * LRS_EINVAL unless vx > 0, r_shell > R_x, eps_inf >= 1, 0 < r_m <= every site's largest shell
 * radius; LRS_EUNSUPPORTED for a site with fewer than 4 shells or beyond the solve's limits.
 * Synchronous in its host part; LRS_ESTATE under stream capture. */
lrs_status lrs_valence_W(lrs_ctx* ctx, const double* chi0_sitesite, const double* centres_host,
                         const double* cell_host, double vx, double r_shell, double eps_inf,
                         double r_m, double* W_out);

/* W for the ALDA polarizability (App. ALDA, Eq. chi-alda: chi~ = (1 - chi0 (v + f_xc))^-1 chi0,
 * with the contact kernel of Eq. kxc_alda, f_xc(r, r') = delta(r - r') dv_xc/dn at n(r)).
 * f_xc is the second derivative of the LDA exchange-correlation energy (Slater exchange,
 * Vosko-Wilk-Nusair correlation) by a 5-point difference with density steps of 0.01
 * (n/4 where n < 0.04).  In the basis of lrs_screen_W, with
 * F_{(L,i),(L',i)} = sum_a w_a Y_L(a) f_xc(r_i a) Y_L'(a):
 *   W~ = V + V D chi~ D V = V + V D X D Y,   Y = (I - V D X D - F X D)^-1 V   (FP64).
 *   chi0_sitesite  site blocks (layout of LRS_COLS_SITE, all sites), device
 *   density        float64 [sum npts] electron density at the site points (e/bohr^3), device
 *   W_out          float64 [nsites][n][n] as lrs_screen_W.
 * Does not change the W kept for lrs_screen_W_backward.  LRS_ESTATE under stream capture. */
lrs_status lrs_screen_W_alda(lrs_ctx* ctx, const double* chi0_sitesite, const double* density,
                             double* W_out);

/* Adjoint of lrs_screen_W.  dL_dW float64 [nsites][n][n], or NULL to differentiate
 * sum(loss_out) of the last lrs_screen_W call with rho_test.  Writes
 * dL_dchi0_sitesite (site-block layout) = P^T (D W^T Gbar W^T D) P per site.  Asynchronous. */
lrs_status lrs_screen_W_backward(lrs_ctx* ctx, const double* dL_dW, double* dL_dchi0_sitesite);

/* Adjoint of lrs_compute_chi0 for site x site blocks (cols must be LRS_COLS_SITE, all sites):
 * given dL/dchi0 (site-block layout) writes dL_dE float64 [nk][nb] and
 * dL_dpsi_site complex128 [nk][nb][sum npts] (complex gradients as dL/dRe + i dL/dIm).
 * Each term's G_o, G_u are recomputed rather than stored.  prec LRS_FP64 runs every product
 * in FP64; LRS_BF16X2 recomputes G and forms the products with psi in split bfloat16 (hi + lo,
 * FP32 accumulation; relative error of order 1e-5), with the gradient accumulation in FP64;
 * LRS_F16F8 recomputes G as the forward F16F8 path does (and so reads the site operand a
 * forward F16F8 call prepared) and forms the products with psi as LRS_BF16X2 does.  An
 * LRS_F16F8, LRS_BF16X2 or LRS_FP64 lrs_compute_chi0 over every site block (site -1,
 * LRS_COLS_SITE; BF16X2: a tuned variant without rotating B fragments) keeps each term's G_o
 * and G_u instead (FP32 complex, FP64 for LRS_FP64: 16 or 32 * nterms * sum n^2 bytes, when
 * that is at most 16 GiB and within LRS_MAX_BYTES; not under stream capture); backward calls
 * in the same precision then form H from them, bit for bit as from recomputed ones, until new
 * orbitals, sites or terms drop them.
 * Other precisions: LRS_EUNSUPPORTED.  Requires terms from lrs_make_quadrature or
 * lrs_make_quadrature_iw (generic terms carry no energy derivative: LRS_EUNSUPPORTED).  With
 * the imaginary-frequency terms dL/dchi0 may be any real matrix per block; with the static
 * terms only its symmetric part matters (chi0 is symmetric there).
 * dL_dpsi_grid must be NULL (site blocks do not use grid orbitals).  Synchronous; under stream
 * capture it returns LRS_ESTATE. */
lrs_status lrs_compute_chi0_backward(lrs_ctx* ctx, int cols, int prec, const double* dL_dchi0,
                                     double* dL_dE, void* dL_dpsi_site, void* dL_dpsi_grid);

/* Autotuner: times every compiled chi0 variant (workgroup tile shape, LDS ring depth, operand
 * scheduling) of precision prec on each column set of the current problem (the cell grid if
 * it was given, and the site blocks), sampled on the site with the most points: the site x grid
 * launch over its first two rounds of tiles of the real plan, the site block whole, scored by
 * milliseconds per output entry covered.  The fastest is kept per (precision, column set) for
 * later lrs_compute_chi0 calls (the environment variable LRS_VARIANT overrides it).  If
 * LRS_TUNE_CACHE names a file, choices are read from it (keyed by precision, column set, the
 * site's rows, columns, K and terms) instead of timed, and new ones appended.  Synchronous;
 * LRS_ESTATE without orbitals, sites and terms. */
lrs_status lrs_tune(lrs_ctx* ctx, int prec);

/* The chi0 variant that lrs_compute_chi0 uses for (prec, cols) (tuned, or the default) and its
 * workgroup tile shape: *variant_host, and *tile_rows_host x *tile_cols_host (may be NULL). */
lrs_status lrs_tuned_variant(const lrs_ctx* ctx, int prec, int cols, int* variant_host,
                             int* tile_rows_host, int* tile_cols_host);

/* Duration in milliseconds of the main kernel of the last lrs_compute_chi0 call, measured
 * with HIP events on the context's stream (synchronises).  -1 if none. */
double lrs_last_kernel_ms(lrs_ctx* ctx);

/* Sustained matrix-core rate of the instruction mix the chi0 kernel of precision `prec`
 * issues (FP64 and FP32: 16x16x4 instructions; BF16X2 and FP16X2: 32x32x16; F16F8: two
 * 32x32x16 fp16 instructions per scaled 32x32x64 fp8 instruction), measured by one launch of
 * one 256-thread workgroup per CU (one wave per SIMD, as the chi0 kernel runs) that issues
 * `iters` rounds of independent instructions and touches memory only to store one value per
 * thread.  *tflops_host: flops per second / 1e12 at the instruction's own rate, an fp8
 * instruction counted as the two fp16 instructions of equal matrix-core time (the unit of
 * the 2.5 PFLOP/s dense 16-bit peak); *ms_host (may be NULL): the launch's duration.  This
 * is the measured denominator for the chi0 kernel's executed rate; it is not part of the
 * method.  Synchronises the stream; LRS_ESTATE under capture; LRS_EINVAL for iters <= 0 or
 * a bad precision. */
lrs_status lrs_mfma_rate(lrs_ctx* ctx, int prec, long long iters, double* tflops_host,
                         double* ms_host);

#ifdef __cplusplus
}
#endif
#endif /* LRS_H */
