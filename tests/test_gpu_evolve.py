"""GPU parity of the Krylov time evolution exp(-iHt) psi (time_evolve of Sec. "Matrix
Representation") against the oracle's exponential series: random Pauli sums and the Heisenberg
chain, batches, long times that need several substeps, and invariants at a larger size."""
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


def random_sum(n, nterms, seed):
    rng = np.random.default_rng(seed)
    return w.pauli_sum(n, [(float(rng.normal()), "".join(rng.choice(list("IXYZ"), n))) for _ in range(nterms)])


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("n,B,t,kind", [(4, 1, 0.3, "rand"), (8, 3, 0.1, "heis"), (10, 2, 1.7, "rand"),
                                        (12, 1, 0.5, "heis"), (9, 5, -0.8, "heis"), (7, 64, 0.25, "rand")])
def test_time_evolution_matches_oracle(dtype, n, B, t, kind):
    H = w.heisenberg(n) if kind == "heis" else random_sum(n, 3 * n, n)
    psi = w.random_state(n, B, 40 + n)
    s = yb.State(n, B, dtype)
    s.upload(psi)
    steps = yb.time_evolve(s, yb.PauliSum.from_workload(H), t)
    assert steps >= 1
    want = oracle.time_evolve(H, psi, t)
    err = np.abs(s.download() - want).max()
    assert err <= (1e-10 if dtype == 1 else 2e-5), err


def test_time_evolution_krylov_dims_and_tolerance():
    n = 10
    H = w.heisenberg(n)
    psi = w.random_state(n, 1, 5)
    want = oracle.time_evolve(H, psi, 2.0)
    for dim in (8, 16, 40):
        s = yb.State(n, 1, 1)
        s.upload(psi)
        steps = yb.time_evolve(s, yb.PauliSum.from_workload(H), 2.0, tol=1e-11, krylov_dim=dim)
        assert np.abs(s.download() - want).max() <= 1e-9
        if dim == 8:
            assert steps > 1


def test_time_evolution_listing_size():
    """The size of Listing "Hamiltonian evolution is faster with cache": a random 16-qubit state
    evolved for t = 0.1 under the Heisenberg chain, every amplitude against the oracle."""
    n = 16
    H = w.heisenberg(n)
    psi = w.random_state(n, 1, 16)
    want = oracle.time_evolve(H, psi, 0.1)
    for dtype in (1, 0):
        s = yb.State(n, 1, dtype)
        s.upload(psi)
        yb.time_evolve(s, yb.PauliSum.from_workload(H), 0.1)
        assert np.abs(s.download() - want).max() <= (1e-10 if dtype == 1 else 2e-5)


def test_time_evolution_invariants_at_22_qubits():
    """Heisenberg chain on 22 qubits: the norm and the energy are conserved and evolving forward
    and back returns the input."""
    n = 22
    h = yb.PauliSum.from_workload(w.heisenberg(n))
    psi = w.random_state(n, 1, 22)
    s = yb.State(n, 1, 1)
    s.upload(psi)
    e0 = yb.expect(s, h)[0]
    yb.time_evolve(s, h, 0.2)
    out = s.download()
    assert abs(np.linalg.norm(out) - 1) < 1e-11
    assert abs(yb.expect(s, h)[0] - e0) < 1e-9
    assert np.abs(out - psi).max() > 1e-3
    yb.time_evolve(s, h, -0.2)
    assert np.abs(s.download() - psi).max() <= 1e-10


def test_time_evolution_eigenstate_and_validation():
    """An eigenstate (all spins up is an eigenstate of the Heisenberg chain with E = n) only
    gains the phase exp(-i n t); the Krylov space closes after one vector."""
    n = 6
    s = yb.State(n, 1, 1)
    yb.time_evolve(s, yb.PauliSum.from_workload(w.heisenberg(n)), 0.7)
    out = s.download()[:, 0]
    assert abs(out[0] - np.exp(-1j * n * 0.7)) < 1e-12
    assert np.abs(out[1:]).max() < 1e-12
    with pytest.raises(yb.YaoError):
        yb.time_evolve(s, yb.PauliSum.from_workload(w.heisenberg(n)), float("nan"))
    with pytest.raises(yb.YaoError):
        yb.time_evolve(s, yb.PauliSum.from_workload(w.heisenberg(n)), 0.1, krylov_dim=100)
