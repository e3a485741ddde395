"""Grouped solves (spca_am_solve_group): requests of different shapes,
formulations, parameters, start counts, tolerances and limits iterated
together, every launch of an iteration covering all of them.

* Each request against the FP64 oracle on the same starts, with the parity
  protocol of the other solve tests (a differing start must pass the
  oracle-trajectory check, the FP64 fixed-point certificate or the
  step-by-step check of the GPU trajectory, rerun for k x-updates).
* A request gives the same bits alone and in a group (its K splits follow
  from its own n and p and the padding only adds exact zeros).
* The widest rows (p = 12288), a start e_i (X0 NULL), degenerate and zero
  starts, per-request limits, the solve-wide warnings, and an A whose
  leading dimension and address need the aligned copy."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import compare_solve, to_device_colmajor, to_device_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def spca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4137_amd as m

    m.load()
    return m


def _param(fid, A, s):
    return workloads.s_or_gamma_for(fid, A, s, "scaled" if fid in (6, 8) else "literal")


def _requests(seed):
    """A mix of small requests: all 8 formulations, n in [40, 700], p in
    [150, 3000], r in {1, 3, 16, 40}, different tol and maxit."""
    rng = np.random.default_rng(seed)
    specs = []
    for k, fid in enumerate([1, 2, 3, 4, 5, 6, 7, 8, 1, 5, 3, 8]):
        n = int(rng.integers(40, 700))
        p = int(rng.integers(150, 3000))
        r = int(rng.choice([1, 3, 16, 40]))
        sp = workloads.spiked_matrix(seed * 100 + k, n, p, thetas=(30.0, 15.0),
                                     spike_nnz=min(20, p // 4))
        s = int(rng.integers(3, 25))
        par = _param(fid, sp.A, s)
        X0 = workloads.random_unit_starts(seed * 100 + 50 + k, r, p)
        specs.append(dict(A_np=sp.A, X0_np=X0, fid=fid, par=par,
                          tol=float(rng.choice([1e-6, 1e-8])), maxit=int(rng.choice([60, 150]))))
    return specs


def _device(spec, X0=True):
    return dict(A=to_device_colmajor(spec["A_np"]),
                X0=to_device_rows(spec["X0_np"]) if X0 else None,
                formulation=spec["fid"], s_or_gamma=spec["par"], tol=spec["tol"],
                maxit=spec["maxit"])


def _group_stepper(spca, req):
    """stepper(k): the request alone (same bits as in the group), k x-updates."""
    def run(k):
        r = dict(req)
        r["maxit"] = k
        return spca.am_solve_group([r], return_X=True)[0]["X_final"].cpu().numpy()
    return run


def test_group_matches_oracle(spca):
    specs = _requests(7)
    reqs = [_device(sp) for sp in specs]
    print("group of", len(reqs), "requests", flush=True)
    got = spca.am_solve_group(reqs, return_X=True)
    for q, (sp, g) in enumerate(zip(specs, got)):
        print(f"request {q}: F{sp['fid']} n={sp['A_np'].shape[0]} p={sp['A_np'].shape[1]} "
              f"r={len(sp['X0_np'])} tol={sp['tol']} maxit={sp['maxit']}", flush=True)
        ref = oracle.am_multi(sp["A_np"], sp["fid"], sp["par"], sp["X0_np"], sp["tol"],
                              sp["maxit"], nthreads=8)
        g = dict(g)
        g["X_final"] = g["X_final"].cpu().numpy()
        compare_solve(g, ref, f"group request {q} F{sp['fid']}", sp["A_np"], sp["fid"],
                      sp["par"], X0=sp["X0_np"], stepper=_group_stepper(spca, reqs[q]))
        assert np.all(g["iters_per_start"] <= sp["maxit"])
        # the returned vector: unit norm, its FP64 objective is the reported one
        x = g["x"]
        if x.any():
            assert abs(np.linalg.norm(x) - 1.0) < 1e-12
            f_chk, _ = oracle.objective(sp["fid"], sp["A_np"], x, sp["par"])
            assert abs(f_chk - g["objective"]) <= 1e-9 * abs(f_chk)


def test_alone_equals_in_group_bitwise(spca):
    specs = _requests(11)
    reqs = [_device(sp) for sp in specs]
    together = spca.am_solve_group(reqs, return_X=True)
    # the same requests in another order and in two smaller groups
    order = list(range(len(reqs)))[::-1]
    rev = spca.am_solve_group([reqs[q] for q in order], return_X=True)
    for q in range(len(reqs)):
        print(f"alone vs group: request {q}", flush=True)
        alone = spca.am_solve_group([reqs[q]], return_X=True)[0]
        for other in (together[q], rev[order.index(q)]):
            for key in ("f_per_start", "iters_per_start", "status_per_start", "nnz_per_start",
                        "phi_per_start", "x"):
                assert np.array_equal(alone[key], other[key]), (q, key)
            assert torch.equal(alone["X_final"], other["X_final"]), q
            assert alone["objective"] == other["objective"]


def test_widest_rows_and_single_start(spca):
    """p = 12288 (the widest register-resident rows) beside a narrow request,
    and the start e_i (X0 NULL, r = 1)."""
    wide = workloads.spiked_matrix(workloads.SEED_BASE + 901, 60, 12288, thetas=(40.0,),
                                   spike_nnz=25)
    narrow = workloads.spiked_matrix(workloads.SEED_BASE + 902, 300, 200, thetas=(20.0,),
                                     spike_nnz=10)
    X0w = workloads.random_unit_starts(workloads.SEED_BASE + 903, 8, 12288)
    reqs = [dict(A=to_device_colmajor(wide.A), X0=to_device_rows(X0w), formulation=1,
                 s_or_gamma=25, tol=1e-8, maxit=100),
            dict(A=to_device_colmajor(narrow.A), X0=None, formulation=4, s_or_gamma=9.0,
                 tol=1e-8, maxit=100)]
    got = spca.am_solve_group(reqs, return_X=True)
    ref = oracle.am_multi(wide.A, 1, 25, X0w, 1e-8, 100, nthreads=8)
    g = dict(got[0])
    g["X_final"] = g["X_final"].cpu().numpy()
    compare_solve(g, ref, "group p=12288", wide.A, 1, 25, X0=X0w,
                  stepper=_group_stepper(spca, reqs[0]))
    # e_i at the column of largest norm (ties to the lowest index)
    norms = np.linalg.norm(narrow.A.astype(np.float64), axis=0)
    x0 = np.zeros((1, 200))
    x0[0, int(np.argmax(norms))] = 1.0
    ref1 = oracle.am_multi(narrow.A, 4, 9.0, x0, 1e-8, 100)
    g1 = dict(got[1])
    g1["X_final"] = g1["X_final"].cpu().numpy()
    compare_solve(g1, ref1, "group e_i start", narrow.A, 4, 9.0, X0=x0)


def test_degenerate_zero_and_warnings(spca):
    A_np = np.zeros((40, 60), np.float32)
    A_np[:, :10] = np.random.default_rng(25).standard_normal((40, 10))
    X0 = np.zeros((3, 60), np.float32)
    X0[0, 30] = 1.0                       # A x0 = 0: DEGENERATE
    X0[1, 2] = 1.0
    X0[2, :] = 1.0
    thr = float(np.max(np.linalg.norm(A_np.astype(np.float64), axis=0)))
    A = to_device_colmajor(A_np)
    reqs = [dict(A=A, X0=to_device_rows(X0), formulation=1, s_or_gamma=3, tol=1e-9, maxit=50),
            dict(A=A, X0=to_device_rows(X0[1:]), formulation=7, s_or_gamma=thr * 1.01,
                 tol=1e-9, maxit=50),
            dict(A=to_device_colmajor(np.zeros((8, 9), np.float32)),
                 X0=to_device_rows(np.ones((2, 9), np.float32)), formulation=2, s_or_gamma=2,
                 tol=1e-9, maxit=5),
            dict(A=A, X0=to_device_rows(X0[1:]), formulation=1, s_or_gamma=3, tol=1e-9,
                 maxit=1)]
    got = spca.am_solve_group(reqs)
    assert got[0]["status_per_start"][0] == spca.DEGENERATE
    assert got[0]["iters_per_start"][0] == 0
    assert got[0]["warning"] == spca.WARN_NONE
    ref = oracle.am_multi(A_np, 1, 3, X0, 1e-9, 50)
    assert abs(got[0]["objective"] - ref["f"][ref["best"]]) <= 1e-5 * ref["f"][ref["best"]]
    assert np.all(got[1]["status_per_start"] == spca.ZERO)
    assert got[1]["objective"] == 0.0 and got[1]["nnz"] == 0 and not got[1]["x"].any()
    assert got[1]["warning"] == spca.WARN_ALL_ZERO
    assert np.all(got[2]["status_per_start"] == spca.DEGENERATE)
    assert got[2]["warning"] == spca.WARN_ALL_DEGENERATE
    # maxit 1: its starts stop at their limit while the others go on
    assert np.all(got[3]["iters_per_start"] == 1)
    assert np.all(got[3]["status_per_start"] == spca.MAXIT)
    assert got[3]["warning"] == spca.WARN_NO_CONVERGED


def test_group_rejects_wide_rows(spca):
    A = to_device_colmajor(np.ones((4, 12289), np.float32))
    with pytest.raises(spca.SpcaError, match="SPCA_GROUP_MAX_P"):
        spca.am_solve_group([dict(A=A, X0=None, formulation=1, s_or_gamma=3)])


def test_unaligned_matrix_in_a_group(spca):
    """A request whose A has lda = 41 and a 4-byte offset (not 16-byte
    aligned): the group copies it to an aligned layout; its result matches
    the oracle and is the same with the matrix aligned."""
    n, p, lda = 37, 500, 41
    sp = workloads.spiked_matrix(workloads.SEED_BASE + 911, n, p, thetas=(25.0,), spike_nnz=12)
    base = torch.zeros(p * lda + 1, dtype=torch.float32)
    view = base[1:1 + p * lda].view(p, lda)
    view[:, :n] = torch.from_numpy(np.ascontiguousarray(sp.A.T))
    A_odd = base.cuda()[1:1 + p * lda].view(p, lda)[:, :n].t()
    assert A_odd.stride() == (1, lda) and A_odd.data_ptr() % 16 != 0
    X0 = workloads.random_unit_starts(workloads.SEED_BASE + 912, 12, p)
    other = _device(_requests(13)[0])
    req = dict(A=A_odd, X0=to_device_rows(X0), formulation=3, s_or_gamma=6.0, tol=1e-9,
               maxit=150)
    got = spca.am_solve_group([other, req], return_X=True)[1]
    aligned = spca.am_solve_group([dict(req, A=to_device_colmajor(sp.A))], return_X=True)[0]
    assert np.array_equal(got["f_per_start"], aligned["f_per_start"])
    assert torch.equal(got["X_final"], aligned["X_final"])
    ref = oracle.am_multi(sp.A, 3, 6.0, X0, 1e-9, 150)
    g = dict(got)
    g["X_final"] = g["X_final"].cpu().numpy()
    compare_solve(g, ref, "group unaligned A", sp.A, 3, 6.0, X0=X0,
                  stepper=_group_stepper(spca, req))
