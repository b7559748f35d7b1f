"""The expectation entry point that allocates nothing (yao_expect_noalloc) against yao_expect and
the oracle, on two calls in a row (the second with a smaller state and batch), and its limits."""
import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def yb():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_10877_amd import binding

    binding.init()
    return binding


@pytest.mark.parametrize("dtype", [0, 1])
def test_noalloc_expect_matches_expect_twice(yb, dtype):
    tol = 1e-12 if dtype == 1 else 1e-5
    for n, B, seed in ((14, 48, 1), (9, 5, 2)):
        psi = w.random_state(n, B, seed)
        H = w.heisenberg(n)
        h = yb.PauliSum.from_workload(H)
        s = yb.State(n, B, dtype)
        s.upload(psi)
        e_na = yb.expect_noalloc(s, h)
        e_ref = yb.expect(s, h)
        e_orc = oracle.expect(H, psi)[0]
        np.testing.assert_allclose(e_na, e_ref, atol=tol, rtol=0)
        np.testing.assert_allclose(e_na, e_orc, atol=tol, rtol=0)


def test_noalloc_expect_random_terms_and_limits(yb):
    rng = np.random.default_rng(9)
    n, B = 11, 3
    terms = [(float(rng.normal()), "".join(rng.choice(list("IXYZ"), n))) for _ in range(40)]
    H = w.pauli_sum(n, terms)
    psi = w.random_state(n, B, 4)
    s = yb.State(n, B, 1)
    s.upload(psi)
    np.testing.assert_allclose(yb.expect_noalloc(s, yb.PauliSum.from_workload(H)), oracle.expect(H, psi)[0],
                               atol=1e-12, rtol=0)
    big = yb.State(12, 200, 0)
    with pytest.raises(yb.YaoError) as ei:
        yb.expect_noalloc(big, yb.PauliSum.from_workload(w.heisenberg(12)))
    assert ei.value.code == -1
    many = w.pauli_sum(n, [(1.0, "".join(rng.choice(list("IXYZ"), n))) for _ in range(4100)])
    with pytest.raises(yb.YaoError) as ei:
        yb.expect_noalloc(s, yb.PauliSum.from_workload(many))
    assert ei.value.code == -1
