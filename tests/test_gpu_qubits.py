"""GPU parity of qubit permutations (focus! / relax!) and the QFT kernel against the oracle: small
states element by element over several tiles and ragged batches, full-size states on sampled
outputs, and the paper's focus!/qft/relax! listing."""
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


def amp_tol(dtype, k=1):
    return 1e-13 if dtype == 1 else 2e-6 * np.sqrt(k) + 1e-6


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("n,B,seed", [(1, 1, 0), (5, 3, 1), (9, 1, 2), (13, 2, 3), (16, 1, 4), (12, 5, 5), (7, 64, 6)])
def test_permute_matches_oracle(dtype, n, B, seed):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n).tolist()
    psi = w.random_state(n, B, seed)
    a = yb.State(n, B, dtype)
    a.upload(psi)
    b = yb.State(n, B, dtype)
    yb.permute_qubits(a, b, perm)
    want = oracle.permute_qubits(psi, n, perm)
    np.testing.assert_array_equal(b.download(), want.astype(a.np_dtype))
    yb.permute_qubits(a, a, perm)  # in place
    np.testing.assert_array_equal(a.download(), want.astype(a.np_dtype))


@pytest.mark.parametrize("dtype", [0, 1])
def test_focus_qft_relax_listing(dtype):
    """Listing "focus! and relax!": rand_state(10), focus!(3,6,1,2), qft(4), relax!."""
    n, locs = 10, [2, 5, 0, 1]
    psi = w.random_state(n, 2, 77)
    s = yb.State(n, 2, dtype)
    s.upload(psi)
    yb.focus(s, locs)
    np.testing.assert_array_equal(s.download(), oracle.focus(psi, n, locs).astype(s.np_dtype))
    yb.qft(s, [0, 1, 2, 3])
    yb.relax(s, locs)
    want = oracle.qft(psi, n, locs)
    assert np.abs(s.download() - want).max() <= amp_tol(dtype, 4)
    # the same through the QFT kernel on the scattered qubits directly
    s.upload(psi)
    yb.qft(s, locs)
    assert np.abs(s.download() - want).max() <= amp_tol(dtype, 4)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("n,B,locs", [
    (3, 1, [0, 1, 2]), (8, 1, list(range(8))), (12, 1, list(range(12))), (14, 3, [13, 2, 7, 0, 9, 4]),
    (15, 1, list(range(15))), (11, 5, [10, 9, 8, 7, 6, 5, 4, 3, 2, 1, 0]), (9, 64, [1, 3, 5, 7]),
    (13, 2, [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12]),
    # single-slot states of >= 10 qubits (the register-radix passes): scattered, reversed and
    # partial qubit sets, so that tiles take code rows, free rows and filler rows
    (14, 1, [13, 2, 7, 0, 9, 4]), (13, 1, list(range(12, -1, -1))), (10, 1, [9, 0, 5]),
    (18, 1, [17, 3, 11, 0, 5, 9, 14, 1, 7, 12]), (16, 1, [4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 0, 1]),
])
def test_qft_matches_oracle(dtype, n, B, locs):
    psi = w.random_state(n, B, n + B)
    s = yb.State(n, B, dtype)
    s.upload(psi)
    yb.qft(s, locs)
    want = oracle.qft(psi, n, locs)
    got = s.download()
    assert np.abs(got - want).max() <= amp_tol(dtype, len(locs))
    yb.qft(s, locs, inverse=True)
    assert np.abs(s.download() - psi).max() <= 2 * amp_tol(dtype, len(locs))
    s.upload(want)
    yb.qft(s, locs, inverse=True)
    assert np.abs(s.download() - oracle.qft(want, n, locs, inverse=True)).max() <= amp_tol(dtype, len(locs))


def test_qft_equals_gate_circuit():
    """The QFT kernel against the gate circuit of Listing "QFT circuit" run through the
    library's own gate path (both GPU), and the oracle."""
    n = 11
    psi = w.random_state(n, 1, 3)
    a = yb.State(n, 1, 1)
    a.upload(psi)
    yb.qft(a, list(range(n)))
    b = yb.State(n, 1, 1)
    b.upload(psi)
    yb.forward(b, yb.Circuit.from_workload(w.qft_circuit(n)), [])
    assert np.abs(a.download() - b.download()).max() <= 1e-12


@pytest.mark.parametrize("dtype", [0, 1])
def test_qft_full_size_sampled(dtype):
    """QFT on all 22 qubits (several passes, 64 MiB complex128): sampled outputs against the
    oracle computed one by one, and the inverse restoring the input."""
    n = 22
    psi = w.random_state(n, 1, 22)
    s = yb.State(n, 1, dtype)
    s.upload(psi)
    locs = list(range(n))
    yb.qft(s, locs)
    got = s.download()
    idx = np.random.default_rng(5).choice(1 << n, 24, replace=False)
    want = oracle.qft(psi, n, locs, idx=idx)
    assert np.abs(got[idx] - want).max() <= (1e-12 if dtype == 1 else 1e-5)
    assert abs(np.linalg.norm(got) - 1) <= (1e-12 if dtype == 1 else 1e-5)
    yb.qft(s, locs, inverse=True)
    assert np.abs(s.download() - psi).max() <= (1e-12 if dtype == 1 else 2e-5)


@pytest.mark.parametrize("dtype", [0, 1])
def test_qft_scattered_qubits_full_size_sampled(dtype):
    """QFT on 14 scattered qubits of a 24-qubit state (single slot: register-radix passes whose
    tiles take code rows and filler rows): sampled outputs against the oracle computed one by
    one, and the inverse restoring the input."""
    n = 24
    locs = [23, 2, 17, 9, 0, 12, 5, 20, 14, 7, 1, 19, 11, 4]
    psi = w.random_state(n, 1, 31)
    s = yb.State(n, 1, dtype)
    s.upload(psi)
    yb.qft(s, locs)
    got = s.download()
    idx = np.random.default_rng(7).choice(1 << n, 24, replace=False)
    want = oracle.qft(psi, n, locs, idx=idx)
    assert np.abs(got[idx] - want).max() <= (1e-12 if dtype == 1 else 1e-5)
    yb.qft(s, locs, inverse=True)
    assert np.abs(s.download() - psi).max() <= (1e-12 if dtype == 1 else 2e-5)


@pytest.mark.parametrize("dtype", [0, 1])
def test_permute_full_size(dtype):
    """A 24-qubit permutation reversing the qubit order (every bit moves), against the oracle
    on sampled indices and exactly inverted by the inverse permutation."""
    n = 24
    perm = list(range(n - 1, -1, -1))
    psi = w.random_state(n, 1, 24)
    s = yb.State(n, 1, dtype)
    s.upload(psi)
    t = yb.State(n, 1, dtype)
    yb.permute_qubits(s, t, perm)
    got = t.download()
    idx = np.random.default_rng(1).choice(1 << n, 1000, replace=False)
    rev = np.array([int(format(i, f"0{n}b")[::-1], 2) for i in idx])
    np.testing.assert_array_equal(got[rev, 0], psi[idx, 0].astype(s.np_dtype))
    yb.permute_qubits(t, t, perm)
    np.testing.assert_array_equal(t.download(), s.download())


def test_permute_and_qft_validation():
    s = yb.State(5, 1, 0)
    for perm in ([0, 1, 2, 3, 3], [0, 1, 2, 3, 5], [0, 1, 2, 3]):
        with pytest.raises(yb.YaoError):
            yb.permute_qubits(s, s, perm + [0] * (5 - len(perm)) if len(perm) < 5 else perm)
    with pytest.raises(yb.YaoError):
        yb.qft(s, [0, 0])
    with pytest.raises(yb.YaoError):
        yb.focus(s, [5])
    big = yb.State(3, 2048, 1)
    with pytest.raises(yb.YaoError):
        yb.qft(big, [0, 1])
