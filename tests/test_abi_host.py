"""Host-only checks of the C-ABI: the library loads, exports every function
declared in include/spca.h, and rejects bad arguments before any device work
(these calls never reach HIP, so they run without a GPU)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

import paper_1212_4137_amd as spca
from paper_1212_4137_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spca.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spca_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    assert sorted(_declared()) == sorted(_lib.EXPORTED)


def test_header_constants_match_the_binding():
    """Status, warning, precision and flag values: the binding's constants are
    the header's #defines."""
    defs = dict(re.findall(r"#define\s+SPCA_([A-Z0-9_]+)\s+\(?(-?\d+)", open(HEADER).read()))
    names = {"CONVERGED": "CONVERGED", "MAXIT": "MAXIT", "DEGENERATE": "DEGENERATE",
             "ZERO": "ZERO", "WARN_NONE": "WARN_NONE",
             "WARN_ALL_DEGENERATE": "WARN_ALL_DEGENERATE", "WARN_ALL_ZERO": "WARN_ALL_ZERO",
             "WARN_NO_CONVERGED": "WARN_NO_CONVERGED", "PREC_FP32": "PREC_FP32",
             "PREC_BF16_POLISH": "PREC_BF16_POLISH", "FLAG_TIME_SAMPLED": "FLAG_TIME_SAMPLED",
             "FLAG_GRAPH": "FLAG_GRAPH", "FLAG_AUTOTUNE": "FLAG_AUTOTUNE",
             "GROUP_MAX_REQUESTS": "GROUP_MAX_REQUESTS", "GROUP_MAX_P": "GROUP_MAX_P",
             "GROUP_MAX_STARTS": "GROUP_MAX_STARTS"}
    for h, b in names.items():
        assert int(defs[h]) == getattr(spca, b), h


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", spca.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (spca_\w+)", out))
    missing = set(_declared()) - exported
    assert not missing, missing
    lib = spca.load()
    for name in _declared():
        assert hasattr(lib, name)


FAKE = ctypes.c_void_p(4096)  # never dereferenced: validation fails first


def _solve(**kw):
    args = dict(A=FAKE, n=10, p=20, lda=10, fid=1, sg=3.0, X0=FAKE, r=2, tol=1e-6,
                maxit=10)
    args.update(kw)
    x = (ctypes.c_double * 32)()
    sup = (ctypes.c_int32 * 32)()
    res = _lib.Result()
    lib = spca.load()
    rc = lib.spca_am_solve(args["A"], args["n"], args["p"], args["lda"], args["fid"],
                           args["sg"], args["X0"], args["r"], args["tol"], args["maxit"],
                           ctypes.cast(x, ctypes.c_void_p), ctypes.cast(sup, ctypes.c_void_p),
                           ctypes.byref(res))
    return rc, lib.spca_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(n=0), "n and p"), (dict(p=0), "n and p"), (dict(r=0), "r "),
    (dict(lda=5), "lda"), (dict(fid=0), "formulation"), (dict(fid=9), "formulation"),
    (dict(maxit=0), "maxit"), (dict(sg=0.0), "L0 constraint"), (dict(sg=21.0), "L0"),
    (dict(sg=2.5), "integral"), (dict(fid=3, sg=0.5), "L1 constraint"),
    (dict(fid=5, sg=-1.0), "gamma"), (dict(fid=7, sg=float("nan")), "finite"),
    (dict(fid=8, sg=float("inf")), "finite"), (dict(A=None), "NULL"),
])
def test_argument_validation(kw, msg):
    rc, err = _solve(**kw)
    assert rc == _lib.SPCA_EINVAL
    assert msg in err


def _group(reqs, count=None):
    """spca_am_solve_group on fake device pointers (validation only)."""
    count = len(reqs) if count is None else count
    probs = (_lib.Problem * max(len(reqs), 1))()
    opts = (_lib.SolveOpts * max(len(reqs), 1))()
    for q, kw in enumerate(reqs):
        a = dict(A=FAKE.value, n=10, p=20, lda=12, fid=1, sg=3.0, X0=FAKE.value, r=2, tol=1e-6,
                 maxit=10, precision=0, check_every=8, total=0, warm=0)
        a.update(kw)
        probs[q] = _lib.Problem(a["A"], a["n"], a["p"], a["lda"], a["fid"], a["sg"])
        opts[q] = _lib.SolveOpts(a["X0"], a["r"], a["tol"], a["maxit"], a["precision"], 0,
                                 a["check_every"], 0, a["total"], a["warm"], 0)
    outs = (_lib.Outputs * max(len(reqs), 1))()
    lib = spca.load()
    rc = lib.spca_am_solve_group(None, None, count, probs, opts, outs)
    return rc, lib.spca_last_error().decode()


@pytest.mark.parametrize("bad,msg", [
    (dict(p=12289, lda=12, sg=3.0), "SPCA_GROUP_MAX_P"), (dict(precision=1), "FP32"),
    (dict(total=5), "replacement"), (dict(warm=2, fid=3), "warm-up"),
    (dict(X0=None), "X0 may be NULL"), (dict(fid=9), "formulation"),
    (dict(check_every=0), "check_every"), (dict(A=None), "A must not be NULL"),
])
def test_group_argument_validation(bad, msg):
    """Each request of a group is checked, and the message names it."""
    rc, err = _group([{}, bad])
    assert rc == _lib.SPCA_EINVAL
    assert msg in err and "(request 1)" in err


def test_group_count_and_start_limits():
    rc, err = _group([{}], count=0)
    assert rc == _lib.SPCA_EINVAL and "count" in err
    rc, err = _group([dict(r=40000), dict(r=30000)])
    assert rc == _lib.SPCA_EINVAL and "SPCA_GROUP_MAX_STARTS" in err
    # well-formed requests pass the checks and fail only on the missing
    # context (no device work is reached)
    rc, err = _group([{}, dict(fid=8, sg=0.5, p=12288, lda=12)])
    assert rc == _lib.SPCA_EINVAL and "ctx" in err
    lib = spca.load()
    probs = (_lib.Problem * 2)(_lib.Problem(FAKE.value, 10, 20, 12, 1, 3.0),
                               _lib.Problem(FAKE.value, 30, 100, 32, 5, 0.1))
    opts = (_lib.SolveOpts * 2)(_lib.SolveOpts(FAKE.value, 2, 1e-6, 10, 0, 0, 8, 0, 0, 0, 0),
                                _lib.SolveOpts(FAKE.value, 5, 1e-6, 10, 0, 0, 8, 0, 0, 0, 0))
    b2 = lib.spca_group_workspace_bytes(2, probs, opts)
    b1 = lib.spca_group_workspace_bytes(1, probs, opts)
    assert b2 > b1 > 0


def test_server_group_limit_validation():
    lib = spca.load()
    assert lib.spca_server_set_group_limit(None, 4) == _lib.SPCA_EINVAL
    assert "server" in lib.spca_last_error().decode()


def test_gemm_argument_validation():
    lib = spca.load()
    rc = lib.spca_gemm_nt_f32(None, FAKE, 6, FAKE, 8, FAKE, 8, 4, 4, 6)
    assert rc == _lib.SPCA_EINVAL and "multiples of 4" in lib.spca_last_error().decode()
    rc = lib.spca_gemm_nt_f32(None, FAKE, 4, FAKE, 8, FAKE, 8, 4, 4, 6)
    assert rc == _lib.SPCA_EINVAL and "leading" in lib.spca_last_error().decode()


def test_x_update_argument_validation():
    lib = spca.load()
    rc = lib.spca_x_update(None, 1, FAKE, 20, 3, 20, 0.0, FAKE, 20, FAKE, FAKE)
    assert rc == _lib.SPCA_EINVAL
    rc = lib.spca_x_update(None, 9, FAKE, 20, 3, 20, 1.0, FAKE, 20, FAKE, FAKE)
    assert rc == _lib.SPCA_EINVAL
    # the allocation-free variant: same checks, and a batch whose chunked
    # scratch exceeds its fixed array is refused before anything is launched
    rc = lib.spca_x_update_noalloc(None, 1, FAKE, 20, 3, 20, 0.0, FAKE, 20, FAKE, FAKE)
    assert rc == _lib.SPCA_EINVAL
    rc = lib.spca_x_update_noalloc(None, 9, FAKE, 20, 3, 20, 1.0, FAKE, 20, FAKE, FAKE)
    assert rc == _lib.SPCA_EINVAL
    rc = lib.spca_x_update_noalloc(None, 1, FAKE, 200000, 100000, 200000, 5.0, FAKE,
                                   200000, FAKE, FAKE)
    assert rc == _lib.SPCA_EINVAL and "scratch" in lib.spca_last_error().decode()


def test_workspace_bytes_is_monotone():
    a = spca.workspace_bytes(100, 500, 1)
    b = spca.workspace_bytes(1000, 10000, 1024)
    assert 0 < a < b
    assert spca.workspace_bytes(0, 5, 1) == 0


def test_tuning_table_round_trip_and_plan_lookup():
    import paper_1212_4137_amd as m

    m.tune_table_clear()
    assert m.tune_table_export() == ""
    model = m.gemm_plan(1024, 10000, 1000, 1)
    # bucket(x) = round(2 log2 x): 1024 -> 20, 10000 -> 27, 1000 -> 20
    other = (model[0] + 1) % 6
    m.tune_table_import(f"4 1 20 27 20 {other} 1\n")
    assert m.gemm_plan(1024, 10000, 1000, 1) == (other, 1)
    assert m.gemm_plan(1100, 10500, 1050, 1) == (other, 1)  # same buckets
    assert m.gemm_plan(1024, 10000, 1000, 2) == m.gemm_plan(1024, 10000, 1000, 2)
    text = m.tune_table_export()
    assert text == f"4 1 20 27 20 {other} 1\n"
    for bad in ("4 1 x", "3 1 20 27 20 0 1", "4 1 20 27 20 99 1", "4 1 20 27 20 0 2"):
        with pytest.raises(m.SpcaError):
            m.tune_table_import(bad)
    assert m.tune_table_export() == text  # a rejected import changes nothing
    # an entry covers a K bucket (here 861..1218); its split count is capped
    # at what the exact K allows (at least 8 slabs of 32 per split), since
    # the solve sizes its split buffers for that
    m.tune_table_import("4 16 20 27 20 0 4\n")
    assert m.gemm_plan(1024, 10000, 1200, 16) == (0, 4)  # 38 slabs
    assert m.gemm_plan(1024, 10000, 870, 16) == (0, 2)   # 28 slabs
    m.tune_table_clear()
    assert m.gemm_plan(1024, 10000, 1000, 1) == model


def test_missing_library_fails_loudly(tmp_path):
    """Without the built HIP library the binding raises instead of falling
    back to anything else (there is no CPU path in the product)."""
    code = (
        "import paper_1212_4137_amd._lib as L\n"
        f"L.LIB_PATH = {str(tmp_path / 'absent.so')!r}\n"
        "L._lib = None\n"
        "try:\n"
        "    L.load()\n"
        "except ImportError as e:\n"
        "    print('raised', e)\n"
        "else:\n"
        "    print('loaded')\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         timeout=120)
    assert out.stdout.startswith("raised"), (out.stdout, out.stderr)


def test_package_does_not_import_the_oracle():
    """The product package and the oracle share no code: nothing under
    paper_1212_4137_amd/ imports oracle/ (and the reverse)."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for sub, other in (("paper_1212_4137_amd", "oracle"), ("oracle", "paper_1212_4137_amd")):
        for dirpath, _, files in os.walk(os.path.join(root, sub)):
            for f in files:
                if f.endswith((".py", ".hip", ".hpp", ".h", ".c", ".cpp")):
                    text = open(os.path.join(dirpath, f), errors="replace").read()
                    assert not re.search(rf"^\s*(import|from)\s+{other}\b", text, re.M), f
                    assert f'#include "{other}' not in text and f"../{other}/" not in text, f
