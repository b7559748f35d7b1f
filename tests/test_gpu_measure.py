"""GPU parity of measurement (measure / measure! of Listing "instruct! and measure") against the
oracle: outcome probabilities element by element, sampled outcomes for the same uniform numbers
(equal, or on a CDF step the two cumulative sums place differently within rounding), the
collapsed state, full-size registers and the paper's example."""
import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

yb = None


@pytest.fixture(scope="module", autouse=True)
def gpu():
    global yb
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_10877_amd import binding

    yb = binding
    yb.init()
    yield


def check_samples(got, psi, n, locs, u, dtype):
    """Outcomes must equal the oracle's, except where u * total lies within rounding of a CDF
    step; there the GPU outcome must still satisfy the rule against the oracle's CDF."""
    want = oracle.sample(psi, n, locs, u)
    p = oracle.probs(psi, n, locs)
    cdf = np.cumsum(p, axis=1)
    tol = 1e-12 if dtype == 1 else 1e-5  # complex64 amplitudes carry ~1e-7 relative rounding
    B, S = u.shape
    bad = 0
    for b in range(B):
        tot = cdf[b, -1]
        for s in np.flatnonzero(got[b] != want[b]):
            x, t = int(got[b, s]), u[b, s] * tot
            lo = cdf[b, x - 1] if x > 0 else 0.0
            # the GPU outcome x must bracket the target within the rounding tolerance
            assert lo - tol <= t <= cdf[b, x] + tol, (b, s, x, int(want[b, s]), t, lo, cdf[b, x])
            assert p[b, x] > 0 or dtype == 0
            bad += 1
    return bad


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("n,B,locs", [
    (1, 1, [0]), (6, 3, [0, 1, 2, 3, 4, 5]), (10, 1, [3, 7]), (12, 5, [11, 0, 6]),
    (14, 2, list(range(14))), (13, 1, [2, 9, 4, 12, 0, 7, 1]), (9, 64, [0, 1, 2]), (16, 1, [15]),
    # 2^16 outcomes in 32 scanned chunks per slot, three slots, locs scattered (permuted first)
    (17, 3, [16, 0, 5, 9, 2, 13, 7, 11, 1, 15, 4, 8, 12, 3, 14, 6]),
])
def test_probs_and_samples_match_oracle(dtype, n, B, locs):
    psi = w.random_state(n, B, 100 + n)
    s = yb.State(n, B, dtype)
    s.upload(psi)
    p = yb.probs(s, locs)
    p_ref = oracle.probs(psi, n, locs)
    assert np.abs(p - p_ref).max() <= (1e-14 if dtype == 1 else 1e-6)
    u = np.random.default_rng(n + B).random((B, 257))
    got = yb.measure(s, locs, u)
    bad = check_samples(got, psi, n, locs, u, dtype)
    assert bad <= (0 if dtype == 1 else got.size // 100)
    np.testing.assert_array_equal(s.download(), psi.astype(s.np_dtype))  # measure leaves the state


def test_measure_listing_example():
    """X on (1-based) qubit 2 of zero_state(4): three shots read 0010."""
    s = yb.State(4, 1, 1)
    s.apply_gate("X", [1])
    out = yb.measure(s, [0, 1, 2, 3], np.array([[0.0, 0.37, 0.999]]))
    assert out.tolist() == [[0b0010] * 3]


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("n,B,locs", [(8, 4, [7, 2]), (11, 1, list(range(11))), (12, 3, [5])])
def test_collapse_matches_oracle(dtype, n, B, locs):
    psi = w.random_state(n, B, 300 + n)
    s = yb.State(n, B, dtype)
    s.upload(psi)
    u = np.random.default_rng(n).random(B)
    x, p = yb.measure_collapse(s, locs, u)
    want_x = oracle.sample(psi, n, locs, u[:, None])[:, 0]
    np.testing.assert_array_equal(x, want_x)
    post, p_ref = oracle.collapse(psi, n, locs, x)
    np.testing.assert_allclose(p, p_ref, rtol=1e-12 if dtype == 1 else 1e-5, atol=0)
    assert np.abs(s.download() - post).max() <= (1e-12 if dtype == 1 else 1e-5)
    # measuring again gives the same outcome with probability 1
    x2 = yb.measure(s, locs, np.random.default_rng(1).random((B, 16)))
    assert np.all(x2 == x[:, None])


@pytest.mark.parametrize("dtype", [0, 1])
def test_full_register_measure_at_22_qubits(dtype):
    """All 22 qubits of a random state (4M outcomes, several scan chunks per slot): probabilities
    on sampled outcomes against the oracle, every shot against the oracle's rule."""
    n = 22
    psi = w.random_state(n, 1, 22)
    s = yb.State(n, 1, dtype)
    s.upload(psi)
    locs = list(range(n))
    p = yb.probs(s, locs)[0]
    idx = np.random.default_rng(2).choice(1 << n, 500, replace=False)
    np.testing.assert_allclose(p[idx], np.abs(psi[idx, 0]) ** 2, rtol=1e-12 if dtype == 1 else 1e-6, atol=1e-18)
    u = np.random.default_rng(3).random((1, 4096))
    got = yb.measure(s, locs, u)
    bad = check_samples(got, psi, n, locs, u, dtype)
    assert bad <= (2 if dtype == 1 else 64)


def test_measure_validation():
    s = yb.State(5, 2, 0)
    with pytest.raises(yb.YaoError):
        yb.measure(s, [0, 0], np.zeros((2, 1)))
    with pytest.raises(yb.YaoError):
        yb.measure(s, [0], np.ones((2, 1)))          # u must be < 1
    with pytest.raises(yb.YaoError):
        yb.measure(s, [0], np.full((2, 1), -0.1))
