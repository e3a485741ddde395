"""Autotuned tile plans (SPCA_FLAG_AUTOTUNE): the tuner fills the table for
both products of a solve, results keep parity with the oracle, and solves
are bit-reproducible given the table (export, clear, import)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import compare_solve, gpu_stepper, to_device_colmajor, to_device_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def spca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4137_amd as m

    m.load()
    m.tune_table_clear()
    yield m
    m.tune_table_clear()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_autotune_fills_table_and_is_reproducible(spca, prec):
    spca.tune_table_clear()
    sp = workloads.spiked_matrix(51, 300, 3000, thetas=(60.0, 30.0), spike_nnz=20)
    X0n = workloads.random_unit_starts(52, 128, 3000)
    A, X0 = to_device_colmajor(sp.A), to_device_rows(X0n)
    kw = dict(tol=1e-8, maxit=200, precision=prec, polish_maxit=100, return_X=True)
    res = {}
    for fid in (1, 5):
        par = workloads.s_or_gamma_for(fid, sp.A, 20)
        res[fid] = spca.am_solve(A, fid, par, X0, flags=spca.FLAG_AUTOTUNE, **kw)
    lines = spca.tune_table_export().splitlines()
    eb = "2" if prec == "bf16" else "4"
    # the two products of the solve; a BF16 solve also tunes the FP32
    # products of its polish sub-solves: all 128 starts, then the best
    # still-running ones (up to 16, a size bucket per count)
    assert sum(ln.split()[0] == eb for ln in lines) == 2, lines
    n_fp32 = sum(ln.split()[0] == "4" for ln in lines)
    if prec == "fp32":
        assert len(lines) == 2, lines
    else:
        assert n_fp32 >= 2 and n_fp32 % 2 == 0 and len(lines) == 2 + n_fp32, lines
    if prec == "fp32":
        for fid in (1, 5):
            par = workloads.s_or_gamma_for(fid, sp.A, 20)
            ref = oracle.am_multi(sp.A.astype(np.float64), fid, par, X0n.astype(np.float64),
                                  1e-8, 200, nthreads=8)
            compare_solve(res[fid], ref, f"autotuned F{fid}", sp.A, fid, par, X0=X0n,
                          stepper=gpu_stepper(spca.am_solve, A, fid, par, X0, tol=1e-8))
    text = spca.tune_table_export()
    spca.tune_table_clear()
    spca.tune_table_import(text)
    assert spca.tune_table_export() == text
    for fid in (1, 5):
        par = workloads.s_or_gamma_for(fid, sp.A, 20)
        again = spca.am_solve(A, fid, par, X0, **kw)  # plans from the imported table
        assert again["objective"] == res[fid]["objective"]
        assert np.array_equal(again["f_per_start"], res[fid]["f_per_start"])
        assert torch.equal(again["X_final"], res[fid]["X_final"])
    spca.tune_table_clear()


def _bucket(x):
    """The tuning table's size bucket: round(2 log2 x)."""
    return int(round(2.0 * np.log2(x)))


@pytest.mark.parametrize("fid,prec", [(1, "fp32"), (6, "fp32"), (1, "bf16"), (6, "bf16")])
def test_every_tile_shape_gives_the_same_solve(spca, fid, prec):
    """A tuning-table entry forces each compiled tile shape on both products
    of a dense-only solve (one K split each, fixed work): each tile sums its
    K range in the same order whatever its shape, so every shape gives the
    same bits; the FP32 shape-0 result keeps parity with the oracle.  With
    BF16 storage the forced products are the BF16 phase's (the polish keeps
    its model plans), and the BF16-phase iterates and the polished results
    are the same bits for every shape."""
    n, p, r = 300, 2000, 64
    sp = workloads.spiked_matrix(53 + fid, n, p, thetas=(60.0, 30.0), spike_nnz=20)
    X0n = workloads.random_unit_starts(54 + fid, r, p)
    A, X0 = to_device_colmajor(sp.A), to_device_rows(X0n)
    par = workloads.s_or_gamma_for(fid, sp.A, 20, "literal")
    kw = dict(tol=-1.0, maxit=25, return_X=True, flags=spca.FLAG_DENSE_ONLY, precision=prec,
              polish_maxit=25 if prec == "bf16" else 0)
    eb = 2 if prec == "bf16" else 4
    first = None
    shape = 0
    while True:
        spca.tune_table_clear()
        try:
            # U^T = X^T A^T: M = r, N = n, K = p; V^T = Y^T A: M = r, N = p, K = n
            spca.tune_table_import(f"{eb} 16 {_bucket(r)} {_bucket(n)} {_bucket(p)} {shape} 1\n"
                                   f"{eb} 16 {_bucket(r)} {_bucket(p)} {_bucket(n)} {shape} 1\n")
        except spca.SpcaError:
            break  # past the last compiled shape
        got = spca.am_solve(A, fid, par, X0, **kw)
        assert spca.tune_table_export().split()[5] == str(shape)
        print(f"F{fid} shape {shape}: objective {got['objective']!r}", flush=True)
        if first is None and prec == "bf16":
            first = got
        elif first is None:
            first = got
            ref = oracle.am_multi(sp.A.astype(np.float64), fid, par, X0n.astype(np.float64),
                                  -1.0, 25, nthreads=8)
            g = dict(got)
            g["X_final"] = g["X_final"].cpu().numpy()
            compare_solve(g, ref, f"forced shape 0 F{fid}", sp.A, fid, par, X0=X0n,
                          stepper=gpu_stepper(spca.am_solve, A, fid, par, X0, tol=-1.0,
                                              flags=spca.FLAG_DENSE_ONLY))
        else:
            assert torch.equal(got["X_final"], first["X_final"]), shape
            assert np.array_equal(got["f_per_start"], first["f_per_start"]), shape
        shape += 1
    spca.tune_table_clear()
    assert shape >= 12, shape
