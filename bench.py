"""Benchmark of the screening hot path on one MI355X.

One step = one pass of the hot path over one synthetic input (the precision workload, 2x2x2 k):
  quadrature terms (host) -> chi0 site x grid (the headline) -> chi0 site x site ->
  W solve with a test-charge loss -> adjoint of the solve -> adjoint of chi0 (split
  products when chi0 runs split, else FP64).
Inputs (orbitals on the grid and at the site points, packed into the library's layouts)
are resident in HBM before the timed region.  The autotuner picks the chi0 variant first.

Prints one JSON line.  `value` = chi0 (site x grid) entries per second of step time in the
bench precision (default F16F8: fp16 hi products with fp8 cross terms; --prec bf16x2 for the
split-BF16 path).  After the steps, once each: the same launch in every other precision (FP64
for the speedup; the split BF16 and FP16 paths; FP32), W from the step's site blocks against W
from the FP64 ones, the FP64 adjoint against the split one, the per-site solves beside W (ALDA
W, induced potential), chi0 at imaginary frequency, the projection of the plane-wave orbitals
onto the site points, and the batching workload's site x grid call (64 uneven sites).  Sampled
entries of every path are compared with the CPU oracle; the oracle's exact pair sum is timed on
the host (cpu_baseline), beside the same factorised algorithm in NumPy (cpu_factorised).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS_TFLOPS = {"bf16x2": 2500.0, "fp16x2": 2500.0, "f16f8": 2500.0, "fp32": 157.3, "fp64": 78.6,
                "fp64m3": 78.6}
DTYPE = {"bf16x2": "bf16", "fp16x2": "f16", "f16f8": "f16+f8", "fp32": "f32", "fp64": "f64",
         "fp64m3": "f64"}
# matrix-core time per algorithmic product, in units of one product at the 2.5 PF/s dense
# 16-bit rate: the split paths run hi*hi + hi*lo + lo*hi (3); F16F8 runs hi*hi on fp16 (1) and
# both cross terms on one fp8 instruction of twice the K at twice the rate (1); the FP64 3M form
# three real products for four
EXEC_FACTOR = {"bf16x2": 3.0, "fp16x2": 3.0, "f16f8": 2.0, "fp32": 1.0, "fp64": 1.0,
               "fp64m3": 0.75}
SPLIT = ("bf16x2", "fp16x2", "f16f8")


def host_info():
    """CPU model, logical CPUs and the BLAS NumPy calls (after a BLAS call has loaded it)."""
    import platform
    model = platform.processor()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        import threadpoolctl
        info = [i for i in threadpoolctl.threadpool_info() if i.get("user_api") == "blas"]
        if info:
            blas = {"library": info[0].get("internal_api"), "version": info[0].get("version"),
                    "threads": info[0].get("num_threads")}
    except Exception:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "blas": blas}


def cpu_factorised(ps_rows, pg_cols, nocc, c, alpha, beta, spin=2):
    """chi0 on a block of rows x columns by the same factorised imaginary-time algorithm as the
    GPU path, in NumPy (one complex GEMM per Green's function and term): G_o^l = sum over
    occupied (k, n) of conj(psi(r)) alpha_l psi(r'), G_u^l likewise, and
    chi0 = -(2 s / N_k^2) sum_l c_l Re[G_o^l conj(G_u^l)].  A CPU baseline, not the oracle."""
    nk = ps_rows.shape[0]
    a_o = np.conj(ps_rows[:, :nocc]).reshape(-1, ps_rows.shape[2])     # [K_o, rows]
    a_u = np.conj(ps_rows[:, nocc:]).reshape(-1, ps_rows.shape[2])
    b_o = pg_cols[:, :nocc].reshape(-1, pg_cols.shape[2])               # [K_o, cols]
    b_u = pg_cols[:, nocc:].reshape(-1, pg_cols.shape[2])
    out = np.zeros((ps_rows.shape[2], pg_cols.shape[2]))
    for l in range(len(c)):
        go = (a_o * alpha[l].reshape(-1, 1)).T @ b_o
        gu = (a_u * beta[l].reshape(-1, 1)).T @ b_u
        out += c[l] * (go.real * gu.real + go.imag * gu.imag)
    return -2.0 * spin / nk ** 2 * out


def fft_grid_size(m, over=4):
    """Smallest 2^a 3^b 5^c >= over * (2 m + 1): the oversampled grid of the FFT route."""
    n = over * (2 * m + 1)
    while True:
        k = n
        for f in (2, 3, 5):
            while k % f == 0:
                k //= f
        if k == 1:
            return n
        n += 1


def fft_projection(ctx, bd, coef, pts, psi_direct):
    """The FFT route of the projection (the same orbitals from an oversampled FFT grid and
    cubic interpolation) timed once after a warm-up, beside the direct method's result."""
    import torch
    cell = np.eye(3) * bd.crystal.a
    n = fft_grid_size(int(np.abs(bd.gvec).max()))
    args = (bd.kpts, cell, bd.gvec, coef, bd.crystal.omega, pts, (n, n, n))
    ctx.project_orbitals_fft(*args)
    torch.cuda.synchronize()
    t = time.time()
    psi = ctx.project_orbitals_fft(*args)
    torch.cuda.synchronize()
    ms = (time.time() - t) * 1e3
    nk_, nb_, npw_ = coef.shape
    # least traffic of the pruned route per band (16 bytes per value): the coefficient
    # sub-box c^3 cleared, read and the coefficients scattered; axis 2 on c^2 lines (writes
    # c^2 n), axis 1 on c slabs (reads c^2 n, writes c n^2), axis 0 everywhere (reads c n^2,
    # writes n^3); the interpolation reads at most every grid value once and writes the points
    c = 2 * int(np.abs(bd.gvec).max()) + 1
    per_band = (2 * c ** 3 + npw_ + 2 * c * c * n + 2 * c * n * n + n ** 3
                + min(64 * len(pts), n ** 3) + len(pts))
    moved = 16.0 * per_band * nk_ * nb_
    return {"call_ms": ms, "grid": [n, n, n], "interpolation": "cubic Lagrange, 4x4x4 nodes",
            "pruned_route_bytes": moved, "pruned_route_gb_per_s": moved / (ms / 1e3) / 1e9,
            "frac_of_hbm": moved / (ms / 1e3) / 8e12,
            "max_rel_diff_vs_direct": float((psi - psi_direct).abs().max()
                                            / psi_direct.abs().max())}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_sha():
    """Hash of the sources that fix the chi0 launch's memory traffic (kernel, operand layout,
    tile order)."""
    h = hashlib.sha256()
    for f in ("chi0.hip", "ring.h", "pack.hip", "lrs_api.cpp", "lrs_internal.h"):
        with open(os.path.join(ROOT, "paper_2005_07834_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counters_for(workload, prec):
    """HBM bytes per launch and MFMA busy fraction from the committed counter runs
    (profiles/chi0_<prec>_<workload>_traffic.json), only if they were taken on the current
    kernel, layout and planner sources."""
    path = os.path.join(ROOT, "profiles", f"chi0_{prec}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_sha") != kernel_source_sha():
        return None
    return d


def copy_calibration(mib):
    """A plain streaming kernel of known traffic: reads and writes `mib` MiB, three launches.
    Hardware byte counters read on it give the scale between counter units and bytes."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_kernel": "neg (float32)", "bytes_read": n * 4, "bytes_written": n * 4,
                      "launches": 3}), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="precision", choices=["precision", "production", "tiny"])
    ap.add_argument("--gamma", action="store_true", help="Gamma-only k-set (precision workload)")
    ap.add_argument("--prec", default="f16f8", choices=list(PEAKS_TFLOPS))
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-fp16", action="store_true",
                    help="skip the one FP16X2 launch run beside a BF16X2 bench")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-projection", action="store_true",
                    help="skip the plane-wave -> site-point projection timed after the steps")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the batching workload's site x grid launch timed at the end")
    ap.add_argument("--no-tune", action="store_true", help="use the default chi0 variant")
    ap.add_argument("--no-gamma-real", action="store_true",
                    help="skip the real-orbital launches at Gamma timed at the end")
    ap.add_argument("--adjoint-prec", default="auto", choices=["auto", "fp64", "bf16x2", "f16f8"],
                    help="precision of the adjoint's products (auto: bf16x2 with a split "
                         "--prec, else fp64)")
    ap.add_argument("--omega", type=float, default=0.1,
                    help="imaginary frequency (Ha) of the chi0(i omega) launch run after the steps")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--steps-only", action="store_true",
                    help="only the warm-up and timed steps and the JSON line: no CPU legs, other "
                         "precisions, checks or side workloads (for profiler runs)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the path is "
              "built and measured for a single device; sharding over sites or grid columns "
              "is not implemented", file=sys.stderr)
        return 2
    if args.copy_mib:
        return copy_calibration(args.copy_mib)
    if args.steps_only:
        args.no_cpu = args.no_fp64 = args.no_fp16 = True
        args.no_projection = args.no_batching = args.no_gamma_real = True

    import torch
    import paper_2005_07834_amd as P
    from workloads import configs
    from workloads.crystal import valence_density

    dev = "cuda"
    t0 = time.time()
    if args.workload == "precision":
        w = configs.precision(device=dev, gamma_only=args.gamma)
    else:
        w = configs.BUILDERS[args.workload](device=dev)
    torch.cuda.synchronize()
    nk, nb = w.energies.shape
    nrows, ncols = w.nrows, w.ngrid ** 3
    log(f"workload {w.name} nk={nk} nb={nb} nocc={w.nocc} rows={nrows} cols={ncols} "
        f"terms={w.n_terms} npw={w.meta['npw']} gen {time.time() - t0:.1f}s")

    # sampled entries for the error check and the CPU oracle (host copies of the orbitals)
    rng = np.random.default_rng(1234)
    ns = 384
    rows = rng.integers(0, nrows, size=ns)
    cols = rng.integers(0, ncols, size=ns)
    ps_s = w.psi_site[:, :, torch.as_tensor(rows, device=dev)].cpu().numpy()
    pg_s = w.psi_grid[:, :, torch.as_tensor(cols, device=dev)].cpu().numpy()

    # CPU baseline block: calibrate the oracle's per-entry cost on the error sample, then take
    # a block of rows x grid columns sized for about --cpu-seconds of oracle work
    from oracle import chi0 as cz
    cpu_block = None
    if not args.no_cpu:
        tc = time.time()
        cz.chi0_exact_entries(ps_s[:, :, :8], pg_s[:, :, :8], w.energies, w.nocc)
        per = (time.time() - tc) / 8
        m = int(max(16, min(200000, args.cpu_seconds / max(per, 1e-7))))
        br = min(16, nrows)
        bc = max(1, m // br)
        brow = rng.integers(0, nrows, size=br)
        bcol = rng.integers(0, ncols, size=bc)
        cpu_block = (w.psi_site[:, :, torch.as_tensor(brow, device=dev)].cpu().numpy(),
                     w.psi_grid[:, :, torch.as_tensor(bcol, device=dev)].cpu().numpy())
        fcol = rng.integers(0, ncols, size=min(ncols, 4096))
        fact_cols = w.psi_grid[:, :, torch.as_tensor(fcol, device=dev)].cpu().numpy()
        frow = rng.integers(0, nrows, size=min(nrows, 128))
        fact_rows = w.psi_site[:, :, torch.as_tensor(frow, device=dev)].cpu().numpy()
        log(f"oracle ~{per * 1e3:.3f} ms/entry; baseline block {br} x {bc}")

    ctx = P.Context(0)
    t1 = time.time()
    ctx.set_orbitals(w.energies, w.nocc, w.psi_grid, w.grid_dV)
    ctx.set_sites(w.sites, w.psi_site)
    torch.cuda.synchronize()
    pack_ms = (time.time() - t1) * 1e3
    w.psi_grid = None
    torch.cuda.empty_cache()
    rho = torch.as_tensor(w.rho_test, device=dev)
    out_grid = torch.empty((nrows, ncols), dtype=torch.float64, device=dev)
    prec = args.prec
    adj_prec = args.adjoint_prec
    if adj_prec == "auto":
        adj_prec = prec if prec in ("bf16x2", "f16f8") else ("bf16x2" if prec in SPLIT else "fp64")
    # the autotuner's choice for this problem (both column sets), before the timed steps
    ctx.make_quadrature(P.QUAD_TIME, w.n_terms, 0.0)
    tq = time.time()
    if not args.no_tune:
        ctx.tune(prec)
    tuned = {"tune_s": time.time() - tq}
    for name, cset in (("grid", P.COLS_GRID), ("site", P.COLS_SITE)):
        v, bm, bn = ctx.tuned_variant(prec, cset)
        tuned[name] = {"variant": v, "tile": [bm, bn]}
    log("tuned", tuned)

    comp = {}
    W_step = {}

    def step(record):
        tq = time.time()
        ctx.make_quadrature(P.QUAD_TIME, w.n_terms, 0.0)
        ctx.chi0(-1, P.COLS_GRID, prec, out=out_grid)
        kms = ctx.last_kernel_ms()
        chi_ss = ctx.chi0(-1, P.COLS_SITE, prec)
        W, loss = ctx.screen_W(chi_ss, rho=rho, want_loss=True)
        lam = ctx.screen_W_backward()
        dE, dpsi = ctx.chi0_backward(lam, adj_prec)
        torch.cuda.synchronize()
        if record:
            comp.setdefault("kernel_ms", []).append(kms)
            comp.setdefault("step_ms", []).append((time.time() - tq) * 1e3)
            comp["adjoint"] = (lam, dE, dpsi)
            W_step["W"] = W
        return loss

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t_start = time.time()
    for _ in range(args.steps):
        loss = step(True)
    torch.cuda.synchronize()
    elapsed = time.time() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    entries = nrows * ncols
    value = entries / (ms_per_step / 1e3)
    kern_ms = float(np.mean(comp["kernel_ms"]))
    got_low = out_grid[torch.as_tensor(rows, device=dev), torch.as_tensor(cols, device=dev)].cpu().numpy()
    log(f"step {ms_per_step:.1f} ms; chi0 kernel ({prec}) {kern_ms:.1f} ms")
    qd = ctx.get_quadrature()      # the static rule of the timed steps

    # every other precision once on the same launch: FP64 (the speedup and the error
    # statement), the split BF16 and FP16 paths, FP32
    paths, got_p = {}, {}
    others = [x for x in ("fp64", "fp64m3", "bf16x2", "fp16x2", "f16f8", "fp32") if x != prec]
    if args.no_fp64:
        others = [x for x in others if x not in ("fp64", "fp64m3")]
    if args.no_fp16 and "fp16x2" in others:
        others.remove("fp16x2")
    if args.steps_only:
        others = []
    for p in others:
        ctx.make_quadrature(P.QUAD_TIME, w.n_terms, 0.0)
        ctx.chi0(-1, P.COLS_GRID, p, out=out_grid)
        ms = ctx.last_kernel_ms()
        got_p[p] = out_grid[torch.as_tensor(rows, device=dev),
                            torch.as_tensor(cols, device=dev)].cpu().numpy()
        paths[p] = dict(kernel_ms=ms, entries_per_s=entries / (ms / 1e3),
                        vs_headline=ms / kern_ms)
        log(f"{p} chi0 kernel {ms:.1f} ms")
    got64 = got_low if prec == "fp64" else got_p.get("fp64")
    # W from this precision's site blocks (the last step's) against W from the FP64 blocks:
    # transitive parity, the FP64 path being pinned to the oracle at the smaller workloads
    w_err = None
    if prec != "fp64" and not args.no_fp64:
        ctx.make_quadrature(P.QUAD_TIME, w.n_terms, 0.0)
        W64, _ = ctx.screen_W(ctx.chi0(-1, P.COLS_SITE, "fp64"))
        Wp = W_step["W"]
        w_err = {"precision": prec, "vs": "W from the FP64 GPU site blocks (transitive)",
                 "max_rel": float((Wp - W64).abs().max() / W64.abs().max()),
                 "frobenius_rel": float(torch.linalg.norm(Wp - W64) / torch.linalg.norm(W64))}
        log("W", w_err)
        del W64
    # the split adjoint against the FP64 adjoint on the last step's dL/dchi0
    adjoint = {"precision": adj_prec}
    if adj_prec != "fp64" and not args.no_fp64:
        lam, dE, dpsi = comp.pop("adjoint")
        ctx.make_quadrature(P.QUAD_TIME, w.n_terms, 0.0)
        ctx.chi0(-1, P.COLS_SITE, prec)      # (the operand the adjoint reads, as in a step)
        torch.cuda.synchronize()
        ta = time.time()
        dEs2, dpsis2 = ctx.chi0_backward(lam, adj_prec)
        torch.cuda.synchronize()
        adjoint["call_ms"] = (time.time() - ta) * 1e3
        del dEs2, dpsis2
        ta = time.time()
        dE64, dpsi64 = ctx.chi0_backward(lam, "fp64")
        torch.cuda.synchronize()
        adjoint["fp64_call_ms"] = (time.time() - ta) * 1e3
        # the FP64 adjoint again after an FP64 site-block call, from the Green's functions it
        # kept (bit for bit the same gradients)
        ctx.chi0(-1, P.COLS_SITE, "fp64")
        torch.cuda.synchronize()
        ta = time.time()
        dE64k, dpsi64k = ctx.chi0_backward(lam, "fp64")
        torch.cuda.synchronize()
        adjoint["fp64_kept_call_ms"] = (time.time() - ta) * 1e3
        adjoint["fp64_kept_bitwise_equal"] = bool(torch.equal(dE64k, dE64) and
                                                  torch.equal(dpsi64k, dpsi64))
        del dE64k, dpsi64k
        adjoint["dE_rel_vs_fp64"] = float((dE - dE64).abs().max() / dE64.abs().max())
        adjoint["dpsi_rel_vs_fp64"] = float((dpsi - dpsi64).abs().max() / dpsi64.abs().max())
        del dE64, dpsi64
        log("adjoint", adjoint)
    comp.pop("adjoint", None)
    solves, iw, got_iw = None, None, None
    if not args.steps_only:
        # the per-site solves beside W (ALDA W, induced potential of a spherical perturbation) on
        # this workload's site block, per call on the library stream
        ctx.make_quadrature(P.QUAD_TIME, w.n_terms, 0.0)
        chi_ss = ctx.chi0(-1, P.COLS_SITE, prec)
        dens = valence_density(w.psi_site, w.nocc)

        def per_call_ms(fn, reps=10):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        def induced(l0):
            return ctx.induced_potential(chi_ss, q=1.0, r_shell=1.5, l0_only=l0)
        solves = {"sites": len(w.sites), "basis": [9 * st.n_rad for st in w.sites],
                  "screen_W_ms": per_call_ms(lambda: ctx.screen_W(chi_ss)),
                  "screen_W_alda_ms": per_call_ms(lambda: ctx.screen_W_alda(chi_ss, dens)),
                  "induced_ms": per_call_ms(lambda: induced(False)),
                  "induced_l0_ms": per_call_ms(lambda: induced(True))}
        del chi_ss
        log("site solves", solves)
        # chi0 at imaginary frequency i omega: the same site x grid launch with complex term
        # coefficients, once
        ctx.make_quadrature_iw(w.n_terms, 0.0, args.omega)
        ctx.chi0(-1, P.COLS_GRID, prec, out=out_grid)
        iw = {"omega": args.omega, "terms": w.n_terms, "precision": prec,
              "kernel_ms": ctx.last_kernel_ms(), "scale": ctx.get_quadrature()["scale"]}
        iw["vs_static_kernel"] = iw["kernel_ms"] / kern_ms
        got_iw = out_grid[torch.as_tensor(rows, device=dev),
                          torch.as_tensor(cols, device=dev)].cpu().numpy()
        log(f"chi0(i omega) kernel {iw['kernel_ms']:.1f} ms")
    # the projection of the plane-wave orbitals onto the site points (the step before the
    # packing), once, outside the timed steps
    proj = None
    if not args.no_projection:
        bd = w.bands
        coef = torch.stack([c.T for c in bd.coef]).contiguous()
        gcart = bd.gvec * (2.0 * np.pi / bd.crystal.a)
        pts = np.concatenate([st.points() for st in w.sites])
        ctx.project_orbitals(bd.kpts, gcart, coef, bd.crystal.omega, pts)   # warm-up
        torch.cuda.synchronize()
        tp = time.time()
        psi_p = ctx.project_orbitals(bd.kpts, gcart, coef, bd.crystal.omega, pts)
        torch.cuda.synchronize()
        pms = (time.time() - tp) * 1e3
        nk_, nb_, npw_ = coef.shape
        fl = 8.0 * nk_ * nb_ * npw_ * len(pts)
        proj = {"call_ms": pms, "nk": nk_, "bands": nb_, "plane_waves": npw_, "points": len(pts),
                "algorithmic_tflops": fl / (pms / 1e3) / 1e12,
                "frac_of_fp64_peak": fl / (pms / 1e3) / 1e12 / PEAKS_TFLOPS["fp64"],
                "rel_err_vs_workload_orbitals":
                    float((psi_p - w.psi_site).abs().max() / w.psi_site.abs().max())}
        proj["fft"] = fft_projection(ctx, bd, coef, pts, psi_p)
        del psi_p, coef
        log("projection", proj)
    # the sustained matrix-core rate of this precision's instruction mix (no memory traffic):
    # the measured denominator of the executed rate, beside the datasheet peak
    _, ms0 = ctx.mfma_rate(prec, 2000)
    sustained, sus_ms = ctx.mfma_rate(prec, max(2000, int(2000 * 300.0 / max(ms0, 1e-3))))
    log(f"sustained matrix-core rate ({prec} mix): {sustained:.0f} TFLOP/s over {sus_ms:.0f} ms")
    ctx.close()
    del out_grid
    torch.cuda.empty_cache()

    # algorithmic work of the chi0 launch: per entry, per term, one complex MAC per (k, band)
    # (8 flop) plus the 4-flop Hadamard accumulate
    K = nk * nb
    flop_per_entry = w.n_terms * (8.0 * K + 4.0)
    achieved = entries * flop_per_entry / (kern_ms / 1e3) / 1e12
    peak = PEAKS_TFLOPS[prec]
    exec_factor = EXEC_FACTOR[prec]
    ctr = counters_for(w.name + ("_gamma" if args.gamma else ""), prec)
    traffic = ctr.get("hbm_bytes_per_launch") if ctr else None

    # oracle: timed exact pair sum on the baseline block (cpu_baseline), and the sampled
    # entries of the GPU results against the exact sum and against the same quadrature
    from oracle import quadrature as q
    cpu, cpu_fact = None, None
    errs = {}

    def rel(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())
    if not args.no_cpu:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max(i["num_threads"] for i in info) if info else os.cpu_count()
        tc = time.time()
        blk = cz.chi0_exact(cpu_block[0], cpu_block[1], w.energies, w.nocc)
        tcpu = time.time() - tc
        cpu = {"value": blk.size / tcpu, "unit": "chi0 entries/s", "cores": int(threads),
               "kind": "oracle",
               "sample": f"{blk.shape[0]} site rows x {blk.shape[1]} grid columns (seeded) of "
                         f"the same workload, exact band-pair sum, {tcpu:.1f} s",
               "host": host_info()}
        mu = q.mid_gap(w.energies, w.nocc)
        terms = cz.terms_for(w.energies, w.nocc, "time", w.n_terms, qd["scale"], mu)
        # the same factorised algorithm as the GPU path in NumPy on the host (context, not the
        # oracle): calibrated on 64 columns, then a block sized for about --cpu-seconds / 2
        tc = time.time()
        cpu_factorised(fact_rows, fact_cols[:, :, :256], w.nocc, *terms)
        per_col = (time.time() - tc) / 256
        mcol = int(max(256, min(fact_cols.shape[2], 0.5 * args.cpu_seconds / max(per_col, 1e-9))))
        tc = time.time()
        fb = cpu_factorised(fact_rows, fact_cols[:, :, :mcol], w.nocc, *terms)
        tf = time.time() - tc
        cpu_fact = {"value": fb.size / tf, "unit": "chi0 entries/s", "cores": int(threads),
                    "kind": "factorised imaginary-time algorithm (NumPy complex GEMM per term)",
                    "sample": f"{fb.shape[0]} site rows x {fb.shape[1]} grid columns (seeded) of "
                              f"the same workload, {w.n_terms} terms, {tf:.1f} s"}
        ex = cz.chi0_exact_entries(ps_s, pg_s, w.energies, w.nocc)
        qq = cz.chi0_quad_entries(ps_s, pg_s, w.nocc, 2, *terms)
        errs[f"{prec}_vs_exact"] = rel(got_low, ex)
        errs[f"{prec}_vs_same_quadrature"] = rel(got_low, qq)
        errs[f"{prec}_vs_exact_frobenius"] = float(np.linalg.norm(got_low - ex) / np.linalg.norm(ex))
        for p, g in got_p.items():
            errs[f"{p}_vs_exact"] = rel(g, ex)
            errs[f"{p}_vs_same_quadrature"] = rel(g, qq)
        errs["quadrature_vs_exact"] = rel(qq, ex)
        errs["entries_compared"] = int(ns)
        log("errors", errs)
        tiw = cz.terms_for(w.energies, w.nocc, f"time_iw:{args.omega}", w.n_terms, iw["scale"], mu)
        qiw = cz.chi0_iw_quad_entries(ps_s, pg_s, w.nocc, 2, *tiw)
        exiw = cz.chi0_iw_exact_entries(ps_s, pg_s, w.energies, w.nocc, args.omega, mu=mu)
        iw["rel_err_vs_same_quadrature"] = rel(got_iw, qiw)
        iw["rel_err_vs_exact"] = rel(got_iw, exiw)
        iw["quadrature_vs_exact"] = rel(qiw, exiw)
        iw["entries_compared"] = int(ns)
        log("chi0(i omega)", iw)

    # the batching workload (64 uneven sites, 87,960 rows x 110,592 columns): its site x grid
    # chi0 in one call (persistent launches over operand batches), node count picked from the
    # band-energy range, three sampled entries per site against the oracle
    batching = None
    if not args.no_batching and args.workload == "precision" and not args.gamma:
        tb = time.time()
        wb = configs.batching(device=dev)
        nrb, ncb = wb.nrows, wb.ngrid ** 3
        offs = wb.site_offsets
        brows = np.array([offs[k] + rng.integers(0, st.npts) for k, st in enumerate(wb.sites)
                          for _ in range(3)])
        bcols = rng.integers(0, ncb, brows.size)
        bps = wb.psi_site[:, :, torch.as_tensor(brows, device=dev)].cpu().numpy()
        bpg = wb.psi_grid[:, :, torch.as_tensor(bcols, device=dev)].cpu().numpy()
        ctx2 = P.Context(0)
        ctx2.set_orbitals(wb.energies, wb.nocc, wb.psi_grid, wb.grid_dV)
        ctx2.set_sites(wb.sites, wb.psi_site)
        wb.psi_grid = None
        torch.cuda.empty_cache()
        nt, terr = ctx2.make_quadrature_tol(1e-9, 24, 32)
        if not args.no_tune:
            ctx2.tune(prec)
        outb = torch.empty((nrb, ncb), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        log(f"batching workload ready in {time.time() - tb:.1f} s: {len(wb.sites)} sites, "
            f"{nrb} x {ncb}, {nt} terms")
        tb = time.time()
        ctx2.chi0(-1, P.COLS_GRID, prec, out=outb)
        torch.cuda.synchronize()
        call_s = time.time() - tb
        bms = ctx2.last_kernel_ms()
        gotb = outb[torch.as_tensor(brows, device=dev), torch.as_tensor(bcols, device=dev)]
        gotb = gotb.cpu().numpy()
        qb = ctx2.get_quadrature()
        v, bm, bn = ctx2.tuned_variant(prec, P.COLS_GRID)
        del outb
        torch.cuda.empty_cache()
        # the projection onto all 87,960 site points, direct and by FFT
        bproj = None
        if not args.no_projection:
            bd = wb.bands
            coef = torch.stack([c.T for c in bd.coef]).contiguous()
            gcart = bd.gvec * (2.0 * np.pi / bd.crystal.a)
            pts = np.concatenate([st.points() for st in wb.sites])
            ctx2.project_orbitals(bd.kpts, gcart, coef, bd.crystal.omega, pts[:64])
            torch.cuda.synchronize()
            tp = time.time()
            psi_d = ctx2.project_orbitals(bd.kpts, gcart, coef, bd.crystal.omega, pts)
            torch.cuda.synchronize()
            bproj = {"points": len(pts), "direct_call_ms": (time.time() - tp) * 1e3,
                     "fft": fft_projection(ctx2, bd, coef, pts, psi_d)}
            del psi_d, coef
            torch.cuda.empty_cache()
        ctx2.close()
        Kb = wb.nk * wb.nb
        batching = {"workload": "batching", "precision": prec, "sites": len(wb.sites),
                    "rows": nrb, "grid_columns": ncb, "terms": nt,
                    "terms_rule": "smallest n in 24..32 with per-pair error <= 1e-9",
                    "terms_rule_error": terr, "variant": v, "tile": [bm, bn],
                    "call_s": call_s, "kernels_ms": bms,
                    "entries_per_s": nrb * ncb / call_s,
                    "algorithmic_tflops": nrb * ncb * nt * (8.0 * Kb + 4.0) / call_s / 1e12,
                    "projection": bproj}
        if not args.no_cpu:
            tb_ = cz.terms_for(wb.energies, wb.nocc, "time", nt, qb["scale"])
            refb = cz.chi0_quad_entries(bps, bpg, wb.nocc, 2, *tb_)
            batching["rel_err_vs_same_quadrature"] = rel(gotb, refb)
            batching["entries_compared"] = int(brows.size)
        log("batching", batching)
        del wb

    # real orbitals at Gamma: the precision cell at one k-point, its orbitals made real
    # (workloads/realify.py); the F16F8 and FP64 site x grid launches from the real orbitals
    # beside the same launches from the complex ones, sampled against the oracle
    gamma_real = None
    if not args.no_gamma_real and args.workload == "precision" and not args.gamma:
        from workloads.realify import realify
        tg = time.time()
        wg = configs.precision(device=dev, gamma_only=True)
        (gre, sre), left = realify(wg.energies, [wg.psi_grid, wg.psi_site])
        ngc = wg.ngrid ** 3
        grows = rng.integers(0, wg.nrows, 64)
        gcols = rng.integers(0, ngc, 64)
        gr_t, gc_t = torch.as_tensor(grows, device=dev), torch.as_tensor(gcols, device=dev)
        outg = torch.empty((wg.nrows, ngc), dtype=torch.float64, device=dev)
        gamma_real = {"workload": "precision at Gamma", "rows": wg.nrows, "grid_columns": ngc,
                      "bands": wg.nb, "terms": wg.n_terms, "imag_left_after_realify": left}
        ctx3 = P.Context(0)
        ctx3.set_orbitals(wg.energies, wg.nocc, wg.psi_grid, wg.grid_dV)
        ctx3.set_sites(wg.sites, wg.psi_site)
        ctx3.make_quadrature(P.QUAD_TIME, wg.n_terms, 0.0)
        gscale = ctx3.get_quadrature()["scale"]
        for p in ("f16f8", "fp64"):
            ctx3.chi0(-1, P.COLS_GRID, p, out=outg)       # (the second call is the one timed)
            ctx3.chi0(-1, P.COLS_GRID, p, out=outg)
            gamma_real[p + "_complex_orbitals_ms"] = ctx3.last_kernel_ms()
        ctx3.close()
        wg.psi_grid = None
        torch.cuda.empty_cache()
        ctx3 = P.Context(0)
        ctx3.set_orbitals_real(wg.energies, wg.nocc, gre, wg.grid_dV)
        ctx3.set_sites(wg.sites, sre)
        ctx3.make_quadrature(P.QUAD_TIME, wg.n_terms, gscale)
        got_g = {}
        for p in ("f16f8", "fp64"):
            ctx3.chi0(-1, P.COLS_GRID, p, out=outg)
            ctx3.chi0(-1, P.COLS_GRID, p, out=outg)
            gamma_real[p + "_real_orbitals_ms"] = ctx3.last_kernel_ms()
            got_g[p] = outg[gr_t, gc_t].cpu().numpy()
        ctx3.close()
        if not args.no_cpu:
            tg_ = cz.terms_for(wg.energies, wg.nocc, "time", wg.n_terms, gscale)
            refg = cz.chi0_quad_entries(sre[:, :, gr_t].cpu().numpy().astype(np.complex128),
                                        gre[:, :, gc_t].cpu().numpy().astype(np.complex128),
                                        wg.nocc, 2, *tg_)
            for p in got_g:
                gamma_real[p + "_rel_err_vs_same_quadrature"] = rel(got_g[p], refg)
            gamma_real["entries_compared"] = int(grows.size)
        gamma_real["leg_s"] = time.time() - tg
        log("gamma real", gamma_real)
        del wg, gre, sre, outg
        torch.cuda.empty_cache()

    fp64 = paths.get("fp64", {})
    rec = {
        "metric": "chi0 entries/s + MFMA util: split-BF16 vs FP64 GPU path at stated rel. error",
        "value": value,
        "unit": "chi0 entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": w.name + ("_gamma" if args.gamma else ""), "precision": prec,
                   "rows": nrows, "grid_columns": ncols, "kpoints": nk, "bands": nb,
                   "occupied": w.nocc, "terms": w.n_terms,
                   "step": "quadrature + chi0 site x grid + chi0 site x site + W + loss + "
                           + f"adjoints ({adj_prec} products)",
                   "tuned": tuned},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "traffic_gb_per_s": traffic / (kern_ms / 1e3) / 1e9 if traffic else None,
                     "executed_mfma_tflops_equiv": achieved * exec_factor,
                     "executed_frac": achieved * exec_factor / peak,
                     "sustained_mfma_tflops_equiv": sustained,
                     "executed_frac_of_sustained": achieved * exec_factor / sustained,
                     "kernel": "chi0_kernel (site x grid)", "kernel_ms": kern_ms,
                     "flop_per_entry": flop_per_entry,
                     "mfma_busy": ctr.get("mfma_busy_frac") if ctr else None},
        "cpu_baseline": cpu,
        "cpu_factorised": cpu_fact,
        "chi0_kernel_entries_per_s": entries / (kern_ms / 1e3),
        "paths": paths,
        "speedup_vs_fp64": (fp64["kernel_ms"] / kern_ms) if fp64 else None,
        "split_bf16_speedup_vs_fp64": (fp64["kernel_ms"] / paths["bf16x2"]["kernel_ms"])
        if fp64 and "bf16x2" in paths else None,
        "rel_err": errs,
        "W_rel_err": w_err,
        "adjoint": adjoint,
        "projection": proj,
        "imag_freq": iw,
        "site_solves": solves,
        "batching": batching,
        "gamma_real": gamma_real,
        "pack_ms": pack_ms,
        "loss": float(loss.sum().item()),
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
