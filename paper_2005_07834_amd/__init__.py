"""Local real-space RPA screening on MI355X: Python binding of the liblrs C ABI.

Argument marshalling only: every step of the computation runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  The binding refuses to
work without the built library (no CPU fallback).

Low-level: ``lib`` is the ctypes handle with the C names (``lib.lrs_create`` ...).
High-level: :class:`Context` wraps one library context on the current torch stream.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblrs.so")

LRS_OK, LRS_EINVAL, LRS_ENOMEM, LRS_EDEVICE, LRS_ESTATE, LRS_ENOGAP, LRS_ENONFINITE, \
    LRS_EUNSUPPORTED = range(8)
FP64, FP32, BF16X2, FP16X2, F16F8, FP64_3M = range(6)
COLS_GRID, COLS_SITE = 0, 1
QUAD_TIME, QUAD_FREQ = 0, 1
PREC_NAMES = {"fp64": FP64, "fp32": FP32, "bf16x2": BF16X2, "fp16x2": FP16X2, "f16f8": F16F8,
              "fp64m3": FP64_3M}
STATUS_NAMES = {0: "LRS_OK", 1: "LRS_EINVAL", 2: "LRS_ENOMEM", 3: "LRS_EDEVICE", 4: "LRS_ESTATE",
                5: "LRS_ENOGAP", 6: "LRS_ENONFINITE", 7: "LRS_EUNSUPPORTED"}

# (name, restype, argtypes) for every entry point of include/lrs.h
_P, _I, _D, _CS = C.c_void_p, C.c_int, C.c_double, C.c_char_p
SIGNATURES = [
    ("lrs_version", _CS, []),
    ("lrs_create", _I, [C.POINTER(_P), _I, _P]),
    ("lrs_destroy", None, [_P]),
    ("lrs_last_error", _CS, [_P]),
    ("lrs_check_bands", _I, [_I, _I, _I, _P, _D, _D]),
    ("lrs_set_orbitals", _I, [_P, _I, _I, _I, _I, _P, _D, _D, _P, _I, _D]),
    ("lrs_set_orbitals_real", _I, [_P, _I, _I, _I, _I, _P, _D, _D, _P, _I, _D]),
    ("lrs_set_sites", _I, [_P, _I, _P, _P, _P, _P, _P, _P, _P, _I]),
    ("lrs_set_quadrature", _I, [_P, _I, _P, _P, _P]),
    ("lrs_make_quadrature", _I, [_P, _I, _I, _D]),
    ("lrs_get_quadrature", _I, [_P, C.POINTER(_I), _P, _P, _P, _P]),
    ("lrs_compute_chi0", _I, [_P, _I, _I, _I, _P]),
    ("lrs_screen_W", _I, [_P, _P, _P, _P, _P]),
    ("lrs_screen_W_backward", _I, [_P, _P, _P]),
    ("lrs_screen_W_noalloc", _I, [_P, _P, _P, _P, _P]),
    ("lrs_compute_chi0_backward", _I, [_P, _I, _I, _P, _P, _P, _P]),
    ("lrs_tune", _I, [_P, _I]),
    ("lrs_tuned_variant", _I, [_P, _I, _I, _P, _P, _P]),
    ("lrs_project_orbitals", _I, [_P, _I, _I, _I, _P, _P, _P, _D, _I, _P, _P]),
    ("lrs_induced_potential", _I, [_P, _P, _P, _D, _D, _I, _P, _P]),
    ("lrs_screen_W_alda", _I, [_P, _P, _P, _P]),
    ("lrs_valence_W", _I, [_P, _P, _P, _P, _D, _D, _D, _D, _P]),
    ("lrs_make_quadrature_iw", _I, [_P, _I, _D, _D]),
    ("lrs_make_quadrature_tol", _I, [_P, _D, _I, _I, _P, _P]),
    ("lrs_project_orbitals_fft", _I, [_P, _I, _I, _I, _P, _P, _P, _P, _D, _P, _I, _P, _P]),
    ("lrs_set_orbitals_pw", _I, [_P, _I, _I, _I, _I, _P, _D, _D, _P, _P, _P, _P, _I, _D, _P]),
    ("lrs_last_kernel_ms", _D, [_P]),
    ("lrs_release_graphs", _I, [_P]),
    ("lrs_mfma_rate", _I, [_P, _I, C.c_longlong, _P, _P]),
]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python paper_2005_07834_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


class LrsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return C.c_void_p(x.data_ptr())
    if isinstance(x, np.ndarray):
        return x.ctypes.data_as(C.c_void_p)
    raise TypeError(type(x))


def _host(a, dtype):
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _dev(t, dtype, device):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t))
    return t.to(device=device, dtype=dtype).contiguous()


class Context:
    """One library context on a CUDA (HIP) device, enqueuing on the current torch stream."""

    def __init__(self, device=0):
        if not torch.cuda.is_available():
            raise LrsError(LRS_EDEVICE, "no GPU visible to torch")
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = lib.lrs_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if st != LRS_OK:
            raise LrsError(st, "lrs_create failed")
        self.h = h
        self._keep = []
        self.nsites = 0
        # bumped by every call that changes the state a backward pass reads: orbitals, sites
        # and quadrature (chi0 adjoint), and the last W solve (W adjoint)
        self.orb_version = 0
        self.screen_version = 0

    def close(self):
        if getattr(self, "h", None):
            lib.lrs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != LRS_OK:
            raise LrsError(st, lib.lrs_last_error(self.h).decode())

    # ------------------------------------------------------------------ inputs
    def set_orbitals(self, energies, nocc, psi_grid=None, grid_dV=0.0, spin=2, mu=float("nan"),
                     delta=0.0):
        E = _host(energies, np.float64)
        nk, nb = E.shape
        g = None
        ngrid = 0
        if psi_grid is not None:
            g = _dev(psi_grid, torch.complex128, self.device)
            assert g.shape[:2] == (nk, nb)
            ngrid = g.shape[2]
        self.orb_version += 1
        self._check(lib.lrs_set_orbitals(self.h, nk, nb, nocc, spin, _ptr(E), mu, delta, _ptr(g),
                                         ngrid, grid_dV))
        self.nk, self.nb, self.nocc, self.ngrid = nk, nb, nocc, ngrid

    def set_orbitals_real(self, energies, nocc, psi_grid=None, grid_dV=0.0, spin=2,
                          mu=float("nan"), delta=0.0):
        """Real orbitals (Gamma, or k-points equal to their negatives modulo the reciprocal
        lattice): energies [nk, nb] (or [nb] at one k), psi_grid [nk, nb, ngrid] (or
        [nb, ngrid]) real, or complex with vanishing imaginary parts."""
        E = _host(energies, np.float64)
        if E.ndim == 1:
            E = E[None]
        nk, nb = E.shape
        g = None
        ngrid = 0
        if psi_grid is not None:
            g = _dev(psi_grid, torch.complex128, self.device).reshape(nk, nb, -1).contiguous()
            ngrid = g.shape[2]
        self.orb_version += 1
        self._check(lib.lrs_set_orbitals_real(self.h, nk, nb, nocc, spin, _ptr(E), mu, delta,
                                              _ptr(g), ngrid, grid_dV))
        self.nk, self.nb, self.nocc, self.ngrid = nk, nb, nocc, ngrid

    def set_sites(self, sites, psi_site, lmax=2):
        nrad = _host([s.n_rad for s in sites], np.int32)
        nang = _host([s.n_ang for s in sites], np.int32)
        radii = _host(np.concatenate([s.radii for s in sites]), np.float64)
        radw = _host(np.concatenate([s.rad_w for s in sites]), np.float64)
        axyz = _host(np.concatenate([s.ang_xyz for s in sites]), np.float64)
        angw = _host(np.concatenate([s.ang_w for s in sites]), np.float64)
        p = _dev(psi_site, torch.complex128, self.device)
        self.orb_version += 1
        self._check(lib.lrs_set_sites(self.h, len(sites), _ptr(nrad), _ptr(nang), _ptr(radii),
                                      _ptr(radw), _ptr(axyz), _ptr(angw), _ptr(p), lmax))
        self.nsites = len(sites)
        self.npts = [s.npts for s in sites]
        self.nbasis = [(lmax + 1) ** 2 * s.n_rad for s in sites]

    def make_quadrature(self, kind=QUAD_TIME, nnodes=16, scale=0.0):
        self.orb_version += 1
        self._check(lib.lrs_make_quadrature(self.h, kind, nnodes, scale))

    def make_quadrature_iw(self, nnodes=32, scale=0.0, omega=0.0):
        """Imaginary-time terms for chi0 at imaginary frequency i omega (Ha)."""
        self.orb_version += 1
        self._check(lib.lrs_make_quadrature_iw(self.h, nnodes, scale, omega))

    def make_quadrature_tol(self, tol, nmin=24, nmax=32):
        """Imaginary-time terms with the node count picked from the band-energy range: the
        smallest n in [nmin, nmax] meeting the per-pair bound tol.  Returns (n, error)."""
        n = np.zeros(1, dtype=np.int32)
        e = np.zeros(1)
        self.orb_version += 1
        self._check(lib.lrs_make_quadrature_tol(self.h, float(tol), int(nmin), int(nmax), _ptr(n),
                                                _ptr(e)))
        return int(n[0]), float(e[0])

    def set_quadrature(self, c, alpha, beta):
        c = _host(c, np.float64)
        a = _host(alpha, np.float64)
        b = _host(beta, np.float64)
        self.orb_version += 1
        self._check(lib.lrs_set_quadrature(self.h, c.shape[0], _ptr(c), _ptr(a), _ptr(b)))

    def get_quadrature(self):
        n = C.c_int()
        c = np.zeros(128)
        tau = np.zeros(128)
        mu = np.zeros(1)
        sc = np.zeros(1)
        self._check(lib.lrs_get_quadrature(self.h, C.byref(n), _ptr(c), _ptr(tau), _ptr(mu),
                                           _ptr(sc)))
        return dict(c=c[:n.value].copy(), tau=tau[:n.value].copy(), mu=float(mu[0]),
                    scale=float(sc[0]))

    # ------------------------------------------------------------------ compute
    def chi0(self, site=-1, cols=COLS_GRID, prec=FP64, out=None):
        if isinstance(prec, str):
            prec = PREC_NAMES[prec]
        if cols == COLS_GRID:
            rows = sum(self.npts) if site < 0 else self.npts[site]
            shape = (rows, self.ngrid)
        else:
            sel = self.npts if site < 0 else [self.npts[site]]
            shape = (sum(n * n for n in sel),)
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=self.device)
        self._check(lib.lrs_compute_chi0(self.h, site, cols, prec, _ptr(out)))
        return out

    def site_blocks(self, flat):
        """Splits the site-block layout into per-site [n, n] views."""
        out, o = [], 0
        for n in self.npts:
            out.append(flat[o:o + n * n].view(n, n))
            o += n * n
        return out

    def screen_W(self, chi0_ss, rho=None, want_loss=False):
        W = torch.empty(sum(n * n for n in self.nbasis), dtype=torch.float64, device=self.device)
        r = None if rho is None else _dev(rho, torch.float64, self.device)
        loss = torch.empty(self.nsites, dtype=torch.float64, device=self.device) if want_loss else None
        self._keep = [r]
        self.screen_version += 1
        self._check(lib.lrs_screen_W(self.h, _ptr(chi0_ss.contiguous()), _ptr(W), _ptr(r),
                                     _ptr(loss)))
        return W, loss

    def screen_W_noalloc(self, chi0_ss, rho=None, want_loss=False, out=None):
        """lrs_screen_W_noalloc: W (and the loss) with the library's fixed scratch array; `out`
        (float64 [sum n^2] on this device) may be given so that nothing is allocated here."""
        W = out if out is not None else torch.empty(sum(n * n for n in self.nbasis),
                                                    dtype=torch.float64, device=self.device)
        r = None if rho is None else _dev(rho, torch.float64, self.device)
        loss = torch.empty(self.nsites, dtype=torch.float64, device=self.device) if want_loss else None
        self._check(lib.lrs_screen_W_noalloc(self.h, _ptr(chi0_ss.contiguous()), _ptr(W), _ptr(r),
                                             _ptr(loss)))
        return W, loss

    def W_blocks(self, flat):
        out, o = [], 0
        for n in self.nbasis:
            out.append(flat[o:o + n * n].view(n, n))
            o += n * n
        return out

    def screen_W_backward(self, dL_dW=None):
        g = torch.empty(sum(n * n for n in self.npts), dtype=torch.float64, device=self.device)
        d = None if dL_dW is None else dL_dW.contiguous()
        self._check(lib.lrs_screen_W_backward(self.h, _ptr(d), _ptr(g)))
        return g

    def chi0_backward(self, dL_dchi0_ss, prec=FP64):
        """dL/dE [nk, nb] and dL/dpsi_site (complex) from dL/dchi0 on the site blocks; prec
        FP64, BF16X2 (split products, relative error of order 1e-5) or F16F8 (Green's
        functions as the forward F16F8 path, split products)."""
        if isinstance(prec, str):
            prec = PREC_NAMES[prec]
        dE = torch.empty((self.nk, self.nb), dtype=torch.float64, device=self.device)
        dpsi = torch.empty((self.nk, self.nb, sum(self.npts)), dtype=torch.complex128,
                           device=self.device)
        self._check(lib.lrs_compute_chi0_backward(self.h, COLS_SITE, prec,
                                                  _ptr(dL_dchi0_ss.contiguous()), _ptr(dE),
                                                  _ptr(dpsi), None))
        return dE, dpsi

    def screen_W_alda(self, chi0_ss, density):
        """W [sum n^2] for the ALDA polarizability, from the site-block chi0 and the electron
        density at the site points [sum npts] (App. ALDA)."""
        W = torch.empty(sum(n * n for n in self.nbasis), dtype=torch.float64, device=self.device)
        d = _dev(density, torch.float64, self.device)
        self._check(lib.lrs_screen_W_alda(self.h, _ptr(chi0_ss.contiguous()), _ptr(d), _ptr(W)))
        return W

    def induced_potential(self, chi0_ss, v1=None, q=1.0, r_shell=1.0, l0_only=False):
        """(rho_ind, v_ind) [sum n] of a spherical perturbation: `v1` [sum n_rad] radial
        values, or the short-range part of q/r split at `r_shell` (Eq. partition)."""
        n = sum(self.nbasis)
        rho = torch.empty(n, dtype=torch.float64, device=self.device)
        v = torch.empty(n, dtype=torch.float64, device=self.device)
        v1h = None if v1 is None else _host(v1, np.float64).reshape(-1)
        self._check(lib.lrs_induced_potential(self.h, _ptr(chi0_ss.contiguous()), _ptr(v1h),
                                              float(q), float(r_shell), int(bool(l0_only)),
                                              _ptr(rho), _ptr(v)))
        return rho, v

    def valence_W(self, chi0_ss, centres, vx, r_shell, eps_inf=1.0, r_m=2.0, cell=None):
        """Valence W(x, x') [nsites, nsites] within r_m for sites centred at grid points
        `centres` [nsites, 3] (Sec. V.A, Eq. rpa-val): the sphere of the discretisation volume
        vx, the shell radius r_shell, eps_inf for the shell's potential, lattice `cell` [3, 3]
        (rows) for the nearest image or None."""
        c = _host(centres, np.float64).reshape(-1, 3)
        if c.shape[0] != self.nsites:
            raise ValueError("one centre per site")
        cl = None if cell is None else _host(cell, np.float64).reshape(3, 3)
        W = torch.empty((self.nsites, self.nsites), dtype=torch.float64, device=self.device)
        self._check(lib.lrs_valence_W(self.h, _ptr(chi0_ss.contiguous()), _ptr(c), _ptr(cl),
                                      float(vx), float(r_shell), float(eps_inf), float(r_m),
                                      _ptr(W)))
        return W

    def project_orbitals(self, kpts, gvec, coef, omega, points):
        """Orbitals at `points` (float64 [npts, 3], bohr) from plane-wave coefficients `coef`
        (complex128 [nk, nb, npw] on this device) with k-points `kpts` [nk, 3] and G vectors
        `gvec` [npw, 3] (Cartesian, bohr^-1): complex128 [nk, nb, npts] (Eq. bloch)."""
        kp = _host(kpts, np.float64).reshape(-1, 3)
        gv = _host(gvec, np.float64).reshape(-1, 3)
        pt = _host(points, np.float64).reshape(-1, 3)
        c = _dev(coef, torch.complex128, self.device)
        nk, nb, npw = c.shape
        if kp.shape[0] != nk or gv.shape[0] != npw:
            raise ValueError("kpts and gvec must match coef's [nk, nb, npw]")
        out = torch.empty((nk, nb, pt.shape[0]), dtype=torch.complex128, device=self.device)
        self._check(lib.lrs_project_orbitals(self.h, nk, nb, npw, _ptr(kp), _ptr(gv), _ptr(c),
                                             float(omega), pt.shape[0], _ptr(pt), _ptr(out)))
        return out

    def release_graphs(self):
        """Unpins the context after the graphs that captured its calls are gone."""
        self._check(lib.lrs_release_graphs(self.h))

    def project_orbitals_fft(self, kpts, cell, gidx, coef, omega, points, nfft):
        """Orbitals at `points` by the FFT route: `cell` [3, 3] lattice vectors (rows), `gidx`
        [npw, 3] Miller indices, `coef` complex128 [nk, nb, npw], FFT grid `nfft` (3 sizes);
        complex128 [nk, nb, npts]."""
        kp = _host(kpts, np.float64).reshape(-1, 3)
        cl = _host(cell, np.float64).reshape(3, 3)
        gi = _host(gidx, np.int32).reshape(-1, 3)
        pt = _host(points, np.float64).reshape(-1, 3)
        nf = _host(nfft, np.int32).reshape(3)
        c = _dev(coef, torch.complex128, self.device)
        nk, nb, npw = c.shape
        out = torch.empty((nk, nb, pt.shape[0]), dtype=torch.complex128, device=self.device)
        self._check(lib.lrs_project_orbitals_fft(self.h, nk, nb, npw, _ptr(kp), _ptr(cl), _ptr(gi),
                                                 _ptr(c), float(omega), _ptr(nf), pt.shape[0],
                                                 _ptr(pt), _ptr(out)))
        return out

    def set_orbitals_pw(self, energies, nocc, kpts, cell, gidx, coef, omega, ngrid, spin=2,
                        mu=float("nan"), delta=0.0):
        """set_orbitals with the grid orbitals made by FFT from plane-wave coefficients `coef`
        complex128 [nk, nb, npw] on the ngrid[0] x ngrid[1] x ngrid[2] grid."""
        E = _host(energies, np.float64)
        kp = _host(kpts, np.float64).reshape(-1, 3)
        cl = _host(cell, np.float64).reshape(3, 3)
        gi = _host(gidx, np.int32).reshape(-1, 3)
        ng = _host(ngrid, np.int32).reshape(3)
        c = _dev(coef, torch.complex128, self.device)
        nk, nb, npw = c.shape
        self.orb_version += 1
        self._check(lib.lrs_set_orbitals_pw(self.h, nk, nb, nocc, spin, _ptr(E), mu, delta, _ptr(kp),
                                            _ptr(cl), _ptr(gi), _ptr(c), npw, float(omega), _ptr(ng)))
        self.nk, self.nb, self.nocc, self.ngrid = nk, nb, nocc, int(np.prod(ng))

    def tune(self, prec):
        if isinstance(prec, str):
            prec = PREC_NAMES[prec]
        self._check(lib.lrs_tune(self.h, prec))

    def tuned_variant(self, prec, cols=COLS_GRID):
        """(variant, tile rows, tile cols) that chi0 uses for this precision and column set."""
        if isinstance(prec, str):
            prec = PREC_NAMES[prec]
        v = np.zeros(3, dtype=np.int32)
        self._check(lib.lrs_tuned_variant(self.h, prec, cols, _ptr(v[0:1]), _ptr(v[1:2]),
                                          _ptr(v[2:3])))
        return int(v[0]), int(v[1]), int(v[2])

    def last_kernel_ms(self):
        return float(lib.lrs_last_kernel_ms(self.h))

    def mfma_rate(self, prec, iters):
        """Sustained matrix-core rate of prec's chi0 instruction mix: (TFLOP/s, ms)."""
        p = PREC_NAMES[prec] if isinstance(prec, str) else prec
        t = np.zeros(1)
        ms = np.zeros(1)
        self._check(lib.lrs_mfma_rate(self.h, p, int(iters), _ptr(t), _ptr(ms)))
        return float(t[0]), float(ms[0])


class Chi0Fn(torch.autograd.Function):
    """chi0 on the site x site blocks as a differentiable function of the band energies and
    the site orbitals: Eq. chi1 with the imaginary-time quadrature.

    ``Chi0Fn.apply(energies, psi_site, ctx, nocc, sites, nnodes, scale[, prec[, omega]])`` sets
    the context's orbitals (no grid), sites and quadrature, and returns the flat site-block
    layout computed in ``prec`` (FP64 by default); ``omega`` > 0 gives chi0 at imaginary
    frequency i omega (the imaginary-time terms with complex coefficients).  The backward pass
    runs the library's adjoint
    (Green's functions recomputed per term, in ``prec`` when it is BF16X2 or F16F8 with split
    products, FP64 otherwise) and returns dL/de [nk, nb] and dL/dpsi_site (complex, dL/dRe + i dL/dIm); dL/de
    is None when the energies were not a tensor or do not require a gradient.  The nodes are held
    fixed: pass ``scale > 0`` so the node set does not depend on the energies.  mu is the
    mid-gap value of the energies given to each forward pass; it cancels in the imaginary-time
    rule (and its frequency-rule counterpart), so no gradient flows through it.  If the context
    was given other inputs since the forward pass, the backward pass sets the forward's inputs
    again first.
    """

    @staticmethod
    def _setup(lctx, energies, psi_site, nocc, sites, nnodes, scale, omega):
        lctx.set_orbitals(energies, nocc)
        lctx.set_sites(sites, psi_site)
        if omega:
            lctx.make_quadrature_iw(nnodes, scale, omega)
        else:
            lctx.make_quadrature(QUAD_TIME, nnodes, scale)

    @staticmethod
    def forward(fctx, energies, psi_site, lctx, nocc, sites, nnodes, scale, *opt):
        p = opt[0] if opt else FP64
        p = PREC_NAMES[p] if isinstance(p, str) else p
        omega = float(opt[1]) if len(opt) > 1 else 0.0
        args = (energies.detach() if isinstance(energies, torch.Tensor) else energies,
                psi_site.detach(), nocc, sites, nnodes, scale, omega)
        Chi0Fn._setup(lctx, *args)
        out = lctx.chi0(-1, COLS_SITE, p)
        fctx.lctx = lctx
        fctx.args = args
        fctx.prec = p if p in (BF16X2, F16F8) else FP64
        fctx.nextra = len(opt)
        fctx.version = lctx.orb_version
        fctx.e_like = (energies.device, energies.dtype) \
            if isinstance(energies, torch.Tensor) else None
        return out

    @staticmethod
    def backward(fctx, g):
        lctx = fctx.lctx
        if lctx.orb_version != fctx.version:
            Chi0Fn._setup(lctx, *fctx.args)
            fctx.version = lctx.orb_version
        dE, dpsi = lctx.chi0_backward(g, fctx.prec)
        if fctx.e_like is None or not fctx.needs_input_grad[0]:
            dE = None
        else:
            dE = dE.to(device=fctx.e_like[0], dtype=fctx.e_like[1])
        if not fctx.needs_input_grad[1]:
            dpsi = None
        return (dE, dpsi,
                None, None, None, None, None) + (None,) * fctx.nextra


class ScreenWFn(torch.autograd.Function):
    """The per-site solve W = (1 - v chi0)^-1 v of Sec. VI.E as a differentiable function of
    the site-block chi0, with the test-charge loss L_s = rho^T D W D rho per site.

    ``W, loss = ScreenWFn.apply(chi0_ss, ctx, rho)`` (rho may be None: loss is then zero and
    not differentiable).  The backward pass combines dL/dW and dL/dloss through the library's
    adjoint; if the context solved another problem since the forward pass, the forward's solve
    is run again first (with the context's sites, which must be the forward's).
    """

    @staticmethod
    def forward(fctx, chi0_ss, lctx, rho):
        chi = chi0_ss.detach()
        W, loss = lctx.screen_W(chi, rho=rho, want_loss=rho is not None)
        fctx.lctx = lctx
        fctx.saved = (chi, rho)
        # new sites drop the kept W too, so both counters are watched
        fctx.version = (lctx.orb_version, lctx.screen_version)
        fctx.has_loss = rho is not None
        if loss is None:
            loss = torch.zeros(lctx.nsites, dtype=torch.float64, device=lctx.device)
        if rho is None:
            fctx.mark_non_differentiable(loss)
        return W, loss

    @staticmethod
    def backward(fctx, gW, gloss):
        lctx = fctx.lctx
        if (lctx.orb_version, lctx.screen_version) != fctx.version:
            chi, rho = fctx.saved
            lctx.screen_W(chi, rho=rho, want_loss=rho is not None)
            fctx.version = (lctx.orb_version, lctx.screen_version)
        total = None
        if fctx.has_loss and gloss is not None and bool((gloss != 0).any()):
            # each site's loss depends on its own block only: scale the blocks of d(sum L)/dchi0
            total = lctx.screen_W_backward(None)
            for s, b in enumerate(lctx.site_blocks(total)):
                b.mul_(gloss[s])
        if gW is not None and bool((gW != 0).any()):
            g2 = lctx.screen_W_backward(gW)
            total = g2 if total is None else total + g2
        if total is None:
            total = torch.zeros(sum(n * n for n in lctx.npts), dtype=torch.float64,
                                device=lctx.device)
        return total, None, None


def check_bands(energies, nocc, mu=float("nan"), delta=0.0):
    """Host-only validation of a band set; returns the status code."""
    E = _host(energies, np.float64)
    return lib.lrs_check_bands(E.shape[0], E.shape[1], nocc, _ptr(E), mu, delta)


__all__ = ["lib", "Context", "LrsError", "check_bands", "Chi0Fn", "ScreenWFn", "FP64", "FP32", "BF16X2", "FP16X2", "F16F8", "FP64_3M",
           "COLS_GRID", "COLS_SITE", "QUAD_TIME", "QUAD_FREQ", "SIGNATURES"]
