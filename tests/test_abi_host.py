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
    for bad in ("4 1 x", "3 1 20 27 20 0 1", "4 1 20 27 20 9 1", "4 1 20 27 20 0 2"):
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
