"""Graph-replayed iterations (SPCA_FLAG_GRAPH) give bit-identical results to
the eager launch sequence: every formulation, FP32 and BF16 storage, on the
default and on a created stream, with maxit not a multiple of the replayed
block, with and without the stop test, and with unrelated eager work between
solves."""
import numpy as np
import pytest

import workloads
from gpu_helpers import to_device_colmajor, to_device_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def spca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4137_amd as m

    m.load()
    return m


@pytest.fixture(scope="module")
def problem():
    sp = workloads.spiked_matrix(31, 300, 1500, thetas=(50.0, 25.0), spike_nnz=20)
    return sp.A, to_device_colmajor(sp.A), to_device_rows(
        workloads.random_unit_starts(32, 48, 1500))


def _same(a, b):
    assert np.array_equal(a["f_per_start"], b["f_per_start"])
    assert np.array_equal(a["iters_per_start"], b["iters_per_start"])
    assert np.array_equal(a["status_per_start"], b["status_per_start"])
    assert np.array_equal(a["x"], b["x"])
    assert a["objective"] == b["objective"] and a["best_start"] == b["best_start"]
    assert torch.equal(a["X_final"], b["X_final"])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("fid", range(1, 9))
def test_graph_matches_eager(spca, problem, fid, prec):
    print(f"graph case fid={fid} prec={prec}", flush=True)
    A_np, A, X0 = problem
    par = workloads.s_or_gamma_for(fid, A_np, 20, "scaled" if fid in (6, 8) else "literal")
    stream = torch.cuda.Stream()
    for tol, maxit in ((-1.0, 37), (1e-7, 200)):
        kw = dict(tol=tol, maxit=maxit, precision=prec, polish_maxit=20, check_every=8,
                  return_X=True)
        eager = spca.am_solve(A, fid, par, X0, **kw)
        for st in (None, stream):
            junk = torch.randn(1 << 16, device="cuda").sum()  # unrelated eager work
            g = spca.am_solve(A, fid, par, X0, flags=spca.FLAG_GRAPH, stream=st, **kw)
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            _same(eager, g)


def test_graph_with_maxit_below_block(spca, problem):
    A_np, A, X0 = problem
    a = spca.am_solve(A, 1, 20.0, X0, tol=-1.0, maxit=5, check_every=8, return_X=True)
    b = spca.am_solve(A, 1, 20.0, X0, tol=-1.0, maxit=5, check_every=8, return_X=True,
                      flags=spca.FLAG_GRAPH)
    _same(a, b)
    assert np.all(b["iters_per_start"] == 5)


@pytest.mark.parametrize("fid", [1, 5])
def test_graph_without_union_launches(spca, problem, fid):
    """With the union product disabled its kernels are left out of the
    launch sequence; the replayed graph still matches the eager solve, and
    both match the solve with the union product available whenever the
    planner picks no union product there."""
    A_np, A, X0 = problem
    par = workloads.s_or_gamma_for(fid, A_np, 20, "literal")
    kw = dict(tol=-1.0, maxit=40, check_every=8, return_X=True)
    eager = spca.am_solve(A, fid, par, X0, flags=spca.FLAG_NO_UNION, kernel_times=True, **kw)
    g = spca.am_solve(A, fid, par, X0, flags=spca.FLAG_NO_UNION | spca.FLAG_GRAPH, **kw)
    _same(eager, g)
    assert eager["kernel_times"]["iters_union"] == 0
    full = spca.am_solve(A, fid, par, X0, kernel_times=True, **kw)
    if full["kernel_times"]["iters_union"] == 0:
        _same(eager, full)
