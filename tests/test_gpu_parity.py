"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by element.

Tolerances: complex128 paths agree with the oracle to rounding (1e-10 and tighter); complex64
paths are held to |dE| <= 1e-5 and max gradient error <= 1e-4 * max(|g*|_inf, 1), and to
amplitude errors of a few float32 ulps times the gate count.
"""
import math

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


def amp_tol(dtype, ngates=1):
    return 1e-12 * max(1, ngates) if dtype == 1 else 2e-6 * math.sqrt(max(1, ngates)) + 1e-6


def grad_tol(dtype, g_ref):
    scale = max(1.0, float(np.abs(g_ref).max()) if g_ref.size else 1.0)
    return (1e-10 if dtype == 1 else 1e-4) * scale


DTYPES = [0, 1]


def run_gates_one_by_one(s, circ, params):
    for g in circ.gates:
        th = params[g.param] if g.param >= 0 else g.theta
        s.apply_gate(g.kind, g.locs, th, g.G, g.ctrls, g.cvals)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("seed", range(8))
def test_gate_instructions_match_oracle(dtype, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 11))
    B = int([1, 1, 3, 5, 64][seed % 5])
    circ = w.random_gate_list(n, 30, seed=700 + seed, kmax=min(3, n), max_ctrl=min(2, n - 1))
    params = w.angles(seed, circ.nparams)
    psi0 = w.random_state(n, B, seed)
    s = yb.State(n, B, dtype)
    s.upload(psi0)
    run_gates_one_by_one(s, circ, params)
    got = s.download()
    want = oracle.forward(circ, params, psi0)
    assert np.abs(got - want).max() <= amp_tol(dtype, len(circ.gates))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_dense_k_qubit_gate(dtype, k):
    n = 9
    rng = np.random.default_rng(k)
    U = w.random_unitary(1 << k, rng)
    locs = [int(x) for x in rng.permutation(n)[:k]]
    ctrl = [q for q in range(n) if q not in locs][:1]
    psi0 = w.random_state(n, 2, k)
    s = yb.State(n, 2, dtype)
    s.upload(psi0)
    s.apply(U, locs, ctrl, [0])
    want = oracle.apply_matrix(psi0, n, U, locs, ctrl, [0])
    assert np.abs(s.download() - want).max() <= amp_tol(dtype, 2 ** k)


@pytest.mark.parametrize("n,B,k,nctrl,seed", [(5, 1, 5, 0, 1), (6, 3, 4, 1, 2), (12, 1, 5, 2, 3), (14, 2, 4, 0, 4),
                                              (10, 64, 5, 1, 5), (13, 100, 4, 2, 6), (16, 1, 5, 1, 7),
                                              (13, 1, 4, 1, 8), (15, 1, 4, 0, 9), (14, 1, 5, 3, 10)])
def test_dense_blocks_on_matrix_cores(n, B, k, nctrl, seed):
    """4- and 5-qubit matrices on complex64 states (the FP32 matrix-core kernel, tiles staged in
    LDS): targets on low and high bits, controls of either value, batches up to 100 slots."""
    rng = np.random.default_rng(seed)
    U = w.random_unitary(1 << k, rng)
    perm = [int(x) for x in rng.permutation(n)]
    locs = perm[:k]
    if seed % 2:
        locs = [0] + [q for q in locs if q != 0][:k - 1]
    rest = [q for q in range(n) if q not in locs]
    ctrl = rest[:nctrl]
    cv = [int(v) for v in rng.integers(0, 2, nctrl)]
    psi0 = w.random_state(n, B, seed)
    s = yb.State(n, B, 0)
    s.upload(psi0)
    s.apply(U, locs, ctrl, cv)
    want = oracle.apply_matrix(psi0, n, U, locs, ctrl, cv)
    assert np.abs(s.download() - want).max() <= amp_tol(0, 2 ** k)


@pytest.mark.parametrize("dtype", DTYPES)
def test_state_create_is_zero_state_and_upload_roundtrip(dtype):
    s = yb.State(5, 3, dtype)
    np.testing.assert_array_equal(s.download(), w.zero_state(5, 3))
    psi = w.random_state(5, 3, 1)
    s.upload(psi)
    assert np.abs(s.download() - psi).max() <= (0 if dtype == 1 else 1e-7)
    s.reset()
    np.testing.assert_array_equal(s.download(), w.zero_state(5, 3))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,B", [(16, 1), (15, 4), (14, 9)])
def test_expectation_and_hpsi_over_several_tiles(dtype, n, B):
    """States wider than a tile: the observable's X-mask groups are split over several tile
    passes (H psi accumulated across them), and a mask wider than a tile falls back to the
    per-group kernels."""
    rng = np.random.default_rng(100 + n)
    terms = [(float(rng.normal()), "".join("IXYZ"[int(v)] for v in rng.integers(0, 4, n))) for _ in range(10)]
    wide = [(0.5, "X" * n), (-0.3, "Z" + "Y" * (n - 1))]
    for H in (w.heisenberg(n), w.pauli_sum(n, terms), w.pauli_sum(n, terms[:3] + wide)):
        psi = w.random_state(n, B, 5)
        s = yb.State(n, B, dtype)
        s.upload(psi)
        h = yb.PauliSum.from_workload(H)
        ref_psi = psi.astype(s.np_dtype).astype(np.complex128)
        re, _ = oracle.expect(H, ref_psi)
        np.testing.assert_allclose(yb.expect(s, h), re, atol=1e-11 if dtype == 1 else 2e-5)
        out = yb.State(n, B, dtype)
        np.testing.assert_allclose(yb.hpsi(s, h, out), re, atol=1e-11 if dtype == 1 else 2e-5)
        want = oracle.hpsi(H, ref_psi)
        assert np.abs(out.download() - want).max() <= (1e-12 if dtype == 1 else 1e-5) * max(1, np.abs(want).max())


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("B", [1, 4, 70])
def test_expectation_and_hpsi(dtype, B):
    n = 8
    rng = np.random.default_rng(B)
    terms = [(1.0, "".join("IXYZ"[int(v)] for v in rng.integers(0, 4, n))) for _ in range(12)]
    terms = [(float(rng.normal()), s) for _, s in terms]
    for H in (w.heisenberg(n), w.pauli_sum(n, terms)):
        psi = w.random_state(n, B, 3)
        s = yb.State(n, B, dtype)
        s.upload(psi)
        h = yb.PauliSum.from_workload(H)
        e = yb.expect(s, h)
        re, _ = oracle.expect(H, psi.astype(s.np_dtype).astype(np.complex128))
        np.testing.assert_allclose(e, re, atol=1e-12 if dtype == 1 else 1e-5)
        out = yb.State(n, B, dtype)
        e2 = yb.hpsi(s, h, out)
        np.testing.assert_allclose(e2, re, atol=1e-12 if dtype == 1 else 1e-5)
        want = oracle.hpsi(H, psi.astype(s.np_dtype).astype(np.complex128))
        assert np.abs(out.download() - want).max() <= (1e-12 if dtype == 1 else 1e-5) * max(1, np.abs(want).max())


@pytest.mark.parametrize("dtype", DTYPES)
def test_symbolic_differentiation_example_on_gpu(dtype):
    circ = w.symad_example()
    H = w.heisenberg(3)
    params = [0.5, 0.7, 0.8]
    e_ref, g_ref, _ = oracle.adjoint(H, circ, params, w.zero_state(3))
    s = yb.State(3, 1, dtype)
    e, g, drift = yb.backward(s, yb.Circuit.from_workload(circ), params, yb.PauliSum.from_workload(H))
    assert abs(e[0] - e_ref[0]) <= (1e-13 if dtype == 1 else 1e-6)
    assert np.abs(g - g_ref).max() <= (1e-13 if dtype == 1 else 1e-6)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("plain", [1, 0])
def test_plain_config_energy_and_150_gradients(dtype, plain):
    """10-qubit ansatz, depth 5, |0...0>, periodic Heisenberg: E and all 150 gradients."""
    yb.set_options(plain=plain)
    try:
        n, depth = 10, 5
        circ = w.hea_circuit(n, depth)
        H = w.heisenberg(n)
        params = w.angles(0, circ.nparams)
        e_ref, g_ref, _ = oracle.adjoint(H, circ, params, w.zero_state(n))
        s = yb.State(n, 1, dtype)
        e, g, drift = yb.backward(s, yb.Circuit.from_workload(circ), params, yb.PauliSum.from_workload(H))
        assert abs(e[0] - e_ref[0]) <= (1e-10 if dtype == 1 else 1e-5)
        assert np.abs(g - g_ref).max() <= grad_tol(dtype, g_ref)
        assert drift <= (1e-12 if dtype == 1 else 1e-5)
        psi_ref = oracle.forward(circ, params, w.zero_state(n))
        assert np.abs(s.download() - psi_ref).max() <= amp_tol(dtype, len(circ.gates))
    finally:
        yb.set_options(plain=0)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("plain", [1, 0])
def test_backward_random_circuits_batched(dtype, seed, plain):
    """Controlled rotations, inverse controls, shift gates, 2- and 3-qubit rot/dense gates,
    a batch of 3 random input states; per-slot and batch-summed gradients."""
    yb.set_options(plain=plain)
    try:
        n = 7
        circ = w.random_gate_list(n, 40, seed=900 + seed, kmax=3)
        H = w.pauli_sum(n, [(0.7, "XXIIYZI"), (-1.1, "ZIZIIII"), (0.4, "IYYIIIX"), (1.0, "IIIZZII")])
        params = w.angles(seed, circ.nparams)
        psi0 = w.random_state(n, 3, seed)
        e_ref, g_ref, _ = oracle.adjoint(H, circ, params, psi0)
        c = yb.Circuit.from_workload(circ)
        h = yb.PauliSum.from_workload(H)
        s = yb.State(n, 3, dtype)
        s.upload(psi0)
        e, g, drift = yb.backward(s, c, params, h)
        np.testing.assert_allclose(e, e_ref, atol=1e-10 if dtype == 1 else 1e-5)
        assert np.abs(g - g_ref).max() <= grad_tol(dtype, g_ref)
        s.upload(psi0)
        e, gs, _ = yb.backward(s, c, params, h, reduce_batch=True)
        assert np.abs(gs - g_ref.sum(axis=0)).max() <= 3 * grad_tol(dtype, g_ref)
    finally:
        yb.set_options(plain=0)


@pytest.mark.parametrize("dtype", DTYPES)
def test_edge_cases(dtype):
    # one qubit; a gate with every other qubit as control; a circuit without parameters
    s = yb.State(1, 1, dtype)
    s.apply_gate("H", [0])
    np.testing.assert_allclose(s.download()[:, 0], [2 ** -0.5, 2 ** -0.5], atol=1e-7)
    n = 6
    psi0 = w.random_state(n, 1, 0)
    s = yb.State(n, 1, dtype)
    s.upload(psi0)
    s.apply_gate("Ry", [3], 0.3, ctrls=[0, 1, 2, 4, 5], cvals=[1, 0, 1, 0, 1])
    want = oracle.apply_matrix(psi0, n, oracle.gate_matrix(w.Gate("Ry", (0,), param=0), 0.3), [3],
                               [0, 1, 2, 4, 5], [1, 0, 1, 0, 1])
    assert np.abs(s.download() - want).max() <= amp_tol(dtype)
    circ = w.ghz_circuit(n)
    s = yb.State(n, 1, dtype)
    e, g, drift = yb.backward(s, yb.Circuit.from_workload(circ), [], yb.PauliSum.from_workload(w.heisenberg(n)))
    assert abs(e[0] - n) < 1e-5 and g.size == 0
    empty = yb.Circuit(n)
    s.reset()
    e, g, drift = yb.backward(s, empty, [], yb.PauliSum.from_workload(w.heisenberg(n)))
    assert abs(e[0] - n) < 1e-6


def test_invalid_calls_leave_state_unchanged():
    s = yb.State(4, 1, 1)
    psi0 = w.random_state(4, 1, 2)
    s.upload(psi0)
    for kw in (dict(kind="X", locs=[4]), dict(kind="X", locs=[1], ctrls=[1]), dict(kind="Rx", locs=[0, 1])):
        with pytest.raises(yb.YaoError):
            s.apply_gate(**kw)
    with pytest.raises(yb.YaoError):
        s.apply(np.eye(4), [0, 0])
    np.testing.assert_array_equal(s.download(), psi0)


# ---------------------------------------------------------------------------------------
# Fused tile passes: several tiles and passes, ragged batches, controls outside the tile,
# 2- and 3-qubit gates in LDS and wider gates as standalone launches.
# ---------------------------------------------------------------------------------------

def with_gate_of_width(circ, k, seed):
    rng = np.random.default_rng(seed)
    q = rng.permutation(circ.n)
    g = w.Gate("dense", tuple(int(x) for x in q[:k]), ctrls=(int(q[k]),), cvals=(0,), G=w.random_unitary(1 << k, rng))
    gates = list(circ.gates)
    gates.insert(len(gates) // 2, g)
    return w.Circuit(circ.n, gates, circ.nparams)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,B,tq", [(5, 1, 0), (9, 3, 0), (13, 1, 0), (16, 1, 0), (14, 8, 6), (12, 100, 0), (15, 2, 5)])
def test_fused_forward_matches_oracle(dtype, n, B, tq):
    yb.set_options(plain=0, tile_qubits=tq)
    try:
        circ = w.random_gate_list(n, 60, seed=1000 + n + B, kmax=3, max_ctrl=2)
        circ = with_gate_of_width(circ, 4, n)
        params = w.angles(n, circ.nparams)
        psi0 = w.random_state(n, B, n)
        s = yb.State(n, B, dtype)
        s.upload(psi0)
        yb.forward(s, yb.Circuit.from_workload(circ), params)
        want = oracle.forward(circ, params, psi0)
        assert np.abs(s.download() - want).max() <= amp_tol(dtype, len(circ.gates))
    finally:
        yb.set_options(tile_qubits=0)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,B,tq", [(6, 1, 0), (12, 1, 0), (15, 1, 6), (11, 5, 0), (13, 2, 5)])
def test_fused_backward_matches_oracle(dtype, n, B, tq):
    yb.set_options(plain=0, tile_qubits=tq)
    try:
        circ = w.random_gate_list(n, 50, seed=2000 + n + B, kmax=3, max_ctrl=2)
        circ = with_gate_of_width(circ, 5, n)
        H = w.heisenberg(n)
        params = w.angles(n + 1, circ.nparams)
        psi0 = w.random_state(n, B, n)
        e_ref, g_ref, _ = oracle.adjoint(H, circ, params, psi0)
        s = yb.State(n, B, dtype)
        s.upload(psi0)
        e, g, drift = yb.backward(s, yb.Circuit.from_workload(circ), params, yb.PauliSum.from_workload(H))
        np.testing.assert_allclose(e, e_ref, atol=1e-10 if dtype == 1 else 1e-5)
        assert np.abs(g - g_ref).max() <= grad_tol(dtype, g_ref)
        assert drift <= (1e-11 if dtype == 1 else 1e-5)
    finally:
        yb.set_options(tile_qubits=0)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,B", [(10, 64), (12, 16), (9, 100)])
def test_fused_backward_many_batch_blocks(dtype, n, B):
    """Batches wider than one tile's batch bits: several batch blocks per pass, per-slot
    gradients and the batch-summed gradient (Sec. "Reverse Mode": batched gradients are
    summed) against the oracle."""
    circ = w.random_gate_list(n, 40, seed=2500 + n + B, kmax=3, max_ctrl=2)
    H = w.heisenberg(n)
    params = w.angles(n + 5, circ.nparams)
    psi0 = w.random_state(n, B, n + 7)
    e_ref, g_ref, _ = oracle.adjoint(H, circ, params, psi0)
    c, h = yb.Circuit.from_workload(circ), yb.PauliSum.from_workload(H)
    s = yb.State(n, B, dtype)
    s.upload(psi0)
    e, g, _ = yb.backward(s, c, params, h)
    np.testing.assert_allclose(e, e_ref, atol=1e-10 if dtype == 1 else 1e-5)
    assert np.abs(g - g_ref).max() <= grad_tol(dtype, g_ref)
    s.upload(psi0)
    e2, gsum, _ = yb.backward(s, c, params, h, reduce_batch=True)
    np.testing.assert_allclose(e2, e_ref, atol=1e-10 if dtype == 1 else 1e-5)
    gsum_ref = g_ref.sum(axis=0)
    assert np.abs(gsum - gsum_ref).max() <= B * grad_tol(dtype, g_ref)


@pytest.mark.parametrize("dtype", DTYPES)
def test_fused_hea_deep(dtype):
    """The workload ansatz at 14 qubits, depth 6: several passes and register groups per layer."""
    n, depth = 14, 6
    circ = w.hea_circuit(n, depth)
    H = w.heisenberg(n)
    params = w.angles(7, circ.nparams)
    e_ref, g_ref, _ = oracle.adjoint(H, circ, params, w.zero_state(n))
    s = yb.State(n, 1, dtype)
    e, g, drift = yb.backward(s, yb.Circuit.from_workload(circ), params, yb.PauliSum.from_workload(H))
    assert abs(e[0] - e_ref[0]) <= (1e-10 if dtype == 1 else 1e-5)
    assert np.abs(g - g_ref).max() <= grad_tol(dtype, g_ref)


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,B,tq", [(16, 1, 7), (15, 3, 6), (17, 1, 0)])
def test_permuted_layouts_between_passes(dtype, n, B, tq):
    """Deep layered circuits over tiles much narrower than the state: most passes store their
    tile with qubits moved onto other index bits, and the plan must restore qubit q to bit q at
    its end (also around a 5-qubit gate launched on its own in the reverse sweep)."""
    yb.set_options(plain=0, tile_qubits=tq)
    try:
        circ = with_gate_of_width(w.hea_circuit(n, 5), 5, n)
        H = w.heisenberg(n)
        params = w.angles(n + 3, circ.nparams)
        psi0 = w.random_state(n, B, n + 1)
        s = yb.State(n, B, dtype)
        s.upload(psi0)
        yb.forward(s, yb.Circuit.from_workload(circ), params)
        want = oracle.forward(circ, params, psi0)
        assert np.abs(s.download() - want).max() <= amp_tol(dtype, len(circ.gates))
        e_ref, g_ref, _ = oracle.adjoint(H, circ, params, psi0)
        s.upload(psi0)
        e, g, drift = yb.backward(s, yb.Circuit.from_workload(circ), params, yb.PauliSum.from_workload(H))
        np.testing.assert_allclose(e, e_ref, atol=1e-10 if dtype == 1 else 1e-5)
        assert np.abs(g - g_ref).max() <= grad_tol(dtype, g_ref)
        assert drift <= (1e-11 if dtype == 1 else 1e-5)
        assert np.abs(s.download() - want).max() <= amp_tol(dtype, len(circ.gates))
    finally:
        yb.set_options(tile_qubits=0)
