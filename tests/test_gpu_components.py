"""Several components by deflation (spca_am_components): the GPU applies the
projection deflation implicitly; the oracle forms the deflated matrix
explicitly.  Per component the objective and the support agree; with s = p
(the power method) the components reproduce sigma_1, sigma_2, sigma_3."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import rel_err, to_device_colmajor, to_device_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def spca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4137_amd as m

    m.load()
    return m


@pytest.mark.parametrize("fid,par", [(1, 20.0), (2, 20.0), (3, 6.0), (7, None), (8, None),
                                     (5, None)])
def test_components_match_oracle(spca, fid, par):
    print(f"components case fid={fid}", flush=True)
    sp = workloads.spiked_matrix(121, 200, 1500, thetas=(150.0, 100.0, 70.0), spike_nnz=20)
    X0n = workloads.random_unit_starts(122, 16, 1500)
    if par is None:
        par = workloads.s_or_gamma_for(fid, sp.A, 20, "scaled")
    got = spca.am_components(to_device_colmajor(sp.A), fid, par, to_device_rows(X0n), 3,
                             tol=1e-9, maxit=400)
    ref = oracle.am_components(sp.A.astype(np.float64), fid, par, X0n.astype(np.float64), 3,
                               1e-9, 400, nthreads=8)
    for c in range(3):
        print(c, got[c]["objective"], ref[c]["f"], len(got[c]["support"]), flush=True)
        assert rel_err(got[c]["objective"], ref[c]["f"]) <= 1e-5, (fid, c)
        assert np.array_equal(got[c]["support"], np.flatnonzero(ref[c]["x"])), (fid, c)
        assert abs(np.linalg.norm(got[c]["x"]) - 1.0) < 1e-12


def test_components_of_the_power_method(spca):
    rng = np.random.default_rng(17)
    A = rng.standard_normal((300, 120)).astype(np.float32)
    sig = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    X0 = to_device_rows(workloads.random_unit_starts(18, 8, 120))
    got = spca.am_components(to_device_colmajor(A), 1, 120.0, X0, 3, tol=1e-12, maxit=3000)
    for c in range(3):
        assert rel_err(got[c]["objective"], sig[c]) <= 1e-5, (c, got[c]["objective"], sig[c])


def test_deflated_solve_graph_and_checks(spca):
    sp = workloads.spiked_matrix(123, 150, 800, thetas=(120.0, 80.0), spike_nnz=15)
    A = to_device_colmajor(sp.A)
    X0 = to_device_rows(workloads.random_unit_starts(124, 12, 800))
    a = spca.am_components(A, 1, 15.0, X0, 2, tol=1e-8, maxit=200)
    b = spca.am_components(A, 1, 15.0, X0, 2, tol=1e-8, maxit=200, flags=spca.FLAG_GRAPH)
    for c in range(2):
        assert a[c]["objective"] == b[c]["objective"]
        assert np.array_equal(a[c]["x"], b[c]["x"])
    with pytest.raises(spca.SpcaError):
        spca.am_components(A, 1, 15.0, X0, 0)
    with pytest.raises(spca.SpcaError):
        spca.am_components(A, 1, 15.0, X0, 17)
