"""The device generator (spca_generate_spiked) reproduces the host
counter-based generator bit for bit: whole matrices at small sizes, sampled
columns at the sizes of the large spiked workloads."""
import numpy as np
import pytest

from workloads import counter

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def spca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4137_amd as m

    m.load()
    return m


@pytest.mark.parametrize("seed,n,p,k", [(0, 1, 1, 0), (1, 37, 300, 0), (2, 257, 1000, 3),
                                        ((1 << 40) + 5, 300, 513, 16)])
def test_generate_matches_host(spca, seed, n, p, k):
    print(f"generate case seed={seed} n={n} p={p} k={k}", flush=True)
    thetas = list(np.linspace(50, 10, k))
    f = counter.spike_factors(seed, n, p, thetas, max(1, p // (2 * max(k, 1))))
    A = spca.generate_spiked(seed, n, p, thetas, f.U, f.V)
    got = A.cpu().numpy()
    ref = counter.spiked_matrix(seed, n, p, f)
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_generate_padded_lda(spca):
    f = counter.spike_factors(9, 130, 70, [20.0], 5)
    A = spca.generate_spiked(9, 130, 70, [20.0], f.U, f.V, lda=136)
    assert A.stride() == (1, 136)
    np.testing.assert_array_equal(A.cpu().numpy(), counter.spiked_matrix(9, 130, 70, f))


def test_generate_large_sampled_columns(spca):
    # 5000 x 50000 with four spikes (800 MB of FP32); 40 sampled columns,
    # including spike-support columns and the last one
    seed, n, p = 0xC3, 5000, 50000
    thetas = [120.0, 90.0, 70.0, 50.0]
    f = counter.spike_factors(seed, n, p, thetas, 100)
    A = spca.generate_spiked(seed, n, p, thetas, f.U, f.V)
    rng = np.random.default_rng(1)
    cols = np.unique(np.concatenate([rng.integers(0, p, 30), f.supports[0][:5],
                                     f.supports[3][:4], [p - 1]]))
    got = A[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    ref = counter.spiked_columns(seed, n, cols, f)
    np.testing.assert_array_equal(got, ref)
    del A
    torch.cuda.empty_cache()


def test_generate_rejects_bad_arguments(spca):
    with pytest.raises(RuntimeError):
        spca.generate_spiked(1, 10, 10, [1.0] * 17, np.zeros((10, 17)), np.zeros((10, 17)))
