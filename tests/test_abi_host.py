"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
declared entry point, and validates band sets before touching a device."""
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lrs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lrs_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2005_07834_amd as P
    names = _declared()
    assert len(names) >= 15
    bound = {n for n, _, _ in P.SIGNATURES}
    for n in names:
        assert hasattr(P.lib, n), n
        assert n in bound, f"{n} has no binding"
    assert P.lib.lrs_version().decode().startswith("lrs")


def test_check_bands_status_codes():
    import paper_2005_07834_amd as P
    E = np.array([[-1.0, -0.5, 0.2, 0.9], [-0.9, -0.4, 0.3, 1.0]])
    assert P.check_bands(E, 2) == P.LRS_OK
    assert P.check_bands(E, 0) == P.LRS_EINVAL
    assert P.check_bands(E, 4) == P.LRS_EINVAL
    bad = E.copy()
    bad[1, 1] = math.nan
    assert P.check_bands(bad, 2) == P.LRS_ENONFINITE
    ov = E.copy()
    ov[1, 1] = 0.25          # occupied at k=1 above the unoccupied bottom at k=0
    assert P.check_bands(ov, 2) == P.LRS_ENOGAP
    # with the metallic regularisation the side of mu still decides occupation: a band set
    # that needs k-dependent occupied counts is refused, one with a gap is accepted
    assert P.check_bands(ov, 2, delta=0.01) == P.LRS_EUNSUPPORTED
    assert P.check_bands(E, 2, delta=0.01) == P.LRS_OK
    assert P.check_bands(E, 2, mu=-0.45, delta=0.01) == P.LRS_EUNSUPPORTED
    assert P.check_bands(E, 2, mu=0.1) == P.LRS_OK
    assert P.check_bands(E, 2, mu=-0.45) == P.LRS_ENOGAP  # mu below the valence top
    assert P.check_bands(E, 2, delta=-1.0) == P.LRS_EINVAL


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import ctypes as C
    import paper_2005_07834_amd as P
    h = C.c_void_p(1)
    st = P.lib.lrs_create(C.byref(h), 0, None)
    assert st == P.LRS_EDEVICE
    assert not h.value
    P.lib.lrs_destroy(None)                      # a NULL context is accepted
    assert P.lib.lrs_last_error(None) == b"null context"


def test_null_context_is_rejected():
    import paper_2005_07834_amd as P
    assert P.lib.lrs_compute_chi0(None, -1, 0, 0, None) == P.LRS_EINVAL
    assert P.lib.lrs_set_orbitals(None, 1, 2, 1, 2, None, 0.0, 0.0, None, 0, 0.0) == P.LRS_EINVAL
    assert P.lib.lrs_tune(None, 0) == P.LRS_EINVAL


def test_binding_argument_counts_match_header():
    """Every binding's argument list has as many entries as the header declaration."""
    import paper_2005_07834_amd as P
    src = open(os.path.join(ROOT, "include", "lrs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    decls = dict(re.findall(r"\b(lrs_[A-Za-z0-9_]+)\s*\(([^)]*)\)\s*;", src))
    for name, _, args in P.SIGNATURES:
        assert name in decls, name
        params = decls[name].strip()
        n = 0 if params in ("", "void") else params.count(",") + 1
        assert n == len(args), f"{name}: header {n} arguments, binding {len(args)}"


def test_product_path_never_uses_the_oracle():
    """The package (binding, build script, kernels) and the benchmark's timed path import
    nothing from oracle/: only tests, smoke() and bench.py's CPU baseline and error legs may."""
    pkg = os.path.join(ROOT, "paper_2005_07834_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", src, flags=re.M), f
                assert "oracle/" not in src and "oracle." not in src, f
    bench = open(os.path.join(ROOT, "bench.py")).read()
    step = bench[bench.index("    def step(record):"):bench.index("    for _ in range(args.warmup):")]
    assert "cz." not in step and "oracle" not in step


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits with a message, before touching any device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_missing_library_fails_loudly(tmp_path):
    """Without liblrs.so the package does not import (no fallback path exists)."""
    import shutil
    import subprocess
    import sys
    dst = tmp_path / "paper_2005_07834_amd"
    shutil.copytree(os.path.join(ROOT, "paper_2005_07834_amd"), dst,
                    ignore=shutil.ignore_patterns("*.so", "*.o", "_build", "__pycache__"))
    r = subprocess.run([sys.executable, "-c", "import paper_2005_07834_amd"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "ImportError" in r.stderr and "not built" in r.stderr


def test_profile_summaries(tmp_path):
    """profsum groups dispatches by (kernel, grid size), lists them in dispatch order, and sums
    a counter over the rows of one dispatch (the per-XCD or per-shader-engine rows)."""
    from paper_2005_07834_amd import profsum
    tr = tmp_path / "kernel_trace.csv"
    tr.write_text(
        "Kernel_Name,Dispatch_Id,Start_Timestamp,End_Timestamp,Grid_Size\n"
        "k<1>(int),3,1000000,4000000,256\n"
        "k<1>(int),1,0,2000000,256\n"
        "k<1>(int),2,0,500000,512\n"
        "other(int),4,0,100000000,256\n")
    lines = profsum.trace(str(tr), r"k<")
    assert len(lines) == 5 and "other" not in "".join(lines)
    assert lines[1].split()[:4] == ["2", "2.500", "2.000", "3.000"] and "256" in lines[1]
    assert lines[2].strip() == "each (ms): 2.000, 3.000"      # dispatch order, not row order
    assert lines[3].split()[:4] == ["1", "0.500", "0.500", "0.500"] and "512" in lines[3]
    pm = tmp_path / "counter_collection.csv"
    pm.write_text(
        "Kernel_Name,Dispatch_Id,Grid_Size,Counter_Name,Counter_Value\n"
        "k(int),1,256,FETCH_SIZE,10\n"
        "k(int),1,256,FETCH_SIZE,5\n"
        "k(int),2,256,FETCH_SIZE,20\n")
    lines = profsum.pmc(str(pm), ".")
    assert lines[1].split()[:3] == ["2", "FETCH_SIZE", "1.750000e+01"]
    assert lines[2].strip() == "each: 1.500000e+01, 2.000000e+01"
