"""GPU parity at the workload sizes: full-size circuits against values the oracle stored
(tests/golden/make_golden.py), gradient modes, determinism and the drift bound."""
import os

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
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
    yb.set_options(plain=0, tile_qubits=0, checkpoint_every=0, drift_tol=0.0)


def golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            out[k] = np.array([float(x) for x in v])
    return out


def grad_ok(g, g_ref, rel):
    return np.abs(g - g_ref).max() <= rel * max(1.0, float(np.abs(g_ref).max()))


@pytest.fixture(scope="module")
def vqe20():
    n, depth = 20, 20
    circ = w.hea_circuit(n, depth)
    return (yb.Circuit.from_workload(circ), yb.PauliSum.from_workload(w.heisenberg(n)), w.angles(2, circ.nparams),
            golden("vqe20_adjoint.txt"))


@pytest.mark.parametrize("dtype,mode", [(0, 0), (1, 0), (0, 1), (0, 2)])
def test_vqe20_energy_and_1200_gradients(vqe20, dtype, mode):
    """Differentiation workload at full size: 20 qubits, depth 20, 1200 parameters."""
    circ, H, params, gold = vqe20
    s = yb.State(20, 1, dtype)
    e, g, drift = yb.backward(s, circ, params, H, mode=mode)
    assert abs(e[0] - gold["energy"][0]) <= (1e-9 if dtype == 1 else 1e-5)
    assert grad_ok(g[0], gold["grad"], 1e-9 if dtype == 1 else 1e-4)
    assert drift <= (1e-10 if dtype == 1 else 1e-5)


def test_vqe20_checkpoint_segments(vqe20):
    circ, H, params, gold = vqe20
    for every in (37, 200, 5000):
        yb.set_options(checkpoint_every=every)
        s = yb.State(20, 1, 0)
        e, g, _ = yb.backward(s, circ, params, H, mode=yb.GRAD_CHECKPOINT)
        assert abs(e[0] - gold["energy"][0]) <= 1e-5
        assert grad_ok(g[0], gold["grad"], 1e-4)
    yb.set_options(checkpoint_every=0)


def test_vqe20_batch64_per_slot_and_summed_gradients(vqe20):
    """The 20-qubit differentiation workload on a 64-slot batch (the shape the batched bench
    line times): 4 seeded input states placed on the slots in a seeded pattern; every slot's
    energy and 1200 gradients and the batch-summed gradient against stored oracle values."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    circ, H, params, _ = vqe20
    gold = golden("b64_states.txt")
    n, B = 20, 64
    pat = mg.b64_pattern(B)
    states = [w.random_state(n, 1, seed)[:, 0] for seed in mg.B64_SEEDS]
    psi0 = np.stack([states[j] for j in pat], axis=1)
    e_ref = np.array([gold[f"energy{j}"][0] for j in pat])
    g_ref = np.stack([gold[f"grad{j}"] for j in pat])
    s = yb.State(n, B, 0)
    s.upload(psi0)
    e, g, drift = yb.backward(s, circ, params, H)
    np.testing.assert_allclose(e, e_ref, atol=1e-5)
    assert grad_ok(g, g_ref, 1e-4)
    assert drift <= 1e-5
    s.upload(psi0)
    e2, gsum, _ = yb.backward(s, circ, params, H, reduce_batch=True)
    np.testing.assert_allclose(e2, e_ref, atol=1e-5)
    assert np.abs(gsum - g_ref.sum(axis=0)).max() <= 1e-4 * B * max(1.0, float(np.abs(g_ref).max()))


def test_backward_is_deterministic(vqe20):
    circ, H, params, _ = vqe20
    s = yb.State(20, 1, 0)
    e1, g1, _ = yb.backward(s, circ, params, H)
    s.reset()
    e2, g2, _ = yb.backward(s, circ, params, H)
    assert e1[0] == e2[0]
    assert np.array_equal(g1, g2)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("every", [1, 7, 50])
def test_checkpoint_modes_match_oracle(mode, every):
    yb.set_options(checkpoint_every=every)
    try:
        n = 9
        circ = w.random_gate_list(n, 45, seed=3000 + every, kmax=3)
        H = w.heisenberg(n)
        params = w.angles(every, circ.nparams)
        psi0 = w.random_state(n, 2, every)
        e_ref, g_ref, _ = oracle.adjoint(H, circ, params, psi0)
        for dtype in (0, 1):
            s = yb.State(n, 2, dtype)
            s.upload(psi0)
            e, g, _ = yb.backward(s, yb.Circuit.from_workload(circ), params, yb.PauliSum.from_workload(H), mode=mode)
            np.testing.assert_allclose(e, e_ref, atol=1e-10 if dtype == 1 else 1e-5)
            assert grad_ok(g, g_ref, 1e-10 if dtype == 1 else 1e-4)
    finally:
        yb.set_options(checkpoint_every=0)


@pytest.mark.parametrize("dtype", [0, 1])
def test_auto_falls_back_to_checkpoints_past_drift_tol(dtype):
    """AUTO runs the reversible sweep; with a drift bound below the rounding floor it restores
    the input and reruns checkpointed, and the results still match the oracle."""
    n = 9
    circ = w.random_gate_list(n, 60, seed=4242, kmax=3)
    H = w.heisenberg(n)
    params = w.angles(17, circ.nparams)
    psi0 = w.random_state(n, 3, 18)
    e_ref, g_ref, _ = oracle.adjoint(H, circ, params, psi0)
    c, h = yb.Circuit.from_workload(circ), yb.PauliSum.from_workload(H)
    tol_e, tol_g = (1e-10, 1e-10) if dtype == 1 else (1e-5, 1e-4)
    try:
        for drift_tol, fallback in ((1e-300, True), (0.0, False)):
            yb.set_options(drift_tol=drift_tol, checkpoint_every=13)
            s = yb.State(n, 3, dtype)
            s.upload(psi0)
            before = yb.auto_fallbacks()
            e, g, drift = yb.backward(s, c, params, h, mode=yb.GRAD_AUTO)
            assert yb.auto_fallbacks() - before == (1 if fallback else 0)
            assert drift <= (1e-10 if dtype == 1 else 1e-5)
            np.testing.assert_allclose(e, e_ref, atol=tol_e)
            assert grad_ok(g, g_ref, tol_g)
            out = oracle.forward(circ, params, psi0)
            got = s.download()
            assert np.abs(got - out).max() <= (1e-12 if dtype == 1 else 1e-5)
    finally:
        yb.set_options(drift_tol=0.0, checkpoint_every=0)


def test_auto_fallback_at_full_size(vqe20):
    """The 20-qubit differentiation workload through AUTO's fallback path."""
    circ, H, params, gold = vqe20
    yb.set_options(drift_tol=1e-300)
    try:
        s = yb.State(20, 1, 0)
        before = yb.auto_fallbacks()
        e, g, _ = yb.backward(s, circ, params, H, mode=yb.GRAD_AUTO)
        assert yb.auto_fallbacks() == before + 1
        assert abs(e[0] - gold["energy"][0]) <= 1e-5
        assert grad_ok(g[0], gold["grad"], 1e-4)
    finally:
        yb.set_options(drift_tol=0.0)


def test_strict_reversible_drift_bound_reports_error():
    """A drift bound below the rounding floor makes the reversible sweep report YAO_EDRIFT."""
    n = 8
    circ = w.hea_circuit(n, 3)
    yb.set_options(drift_tol=1e-30)
    try:
        s = yb.State(n, 1, 0)
        with pytest.raises(yb.YaoError) as ei:
            yb.backward(s, yb.Circuit.from_workload(circ), w.angles(0, circ.nparams),
                        yb.PauliSum.from_workload(w.heisenberg(n)))
        assert ei.value.code == -4
    finally:
        yb.set_options(drift_tol=0.0)


@pytest.mark.parametrize("dtype", [0, 1])
def test_random_su2_circuit_20q_observables(dtype):
    """Precision workload family at 20 qubits: Haar SU(2) layers + CZ pairings, depth 24."""
    gold = golden("rand20_observables.txt")
    n = 20
    circ = w.random_circuit(n, 24, seed=5)
    s = yb.State(n, 1, dtype)
    yb.forward(s, yb.Circuit.from_workload(circ), [])
    zz = yb.PauliSum.from_workload(w.pauli_sum(n, [(1.0, "ZZ" + "I" * (n - 2))]))
    x0 = yb.PauliSum.from_workload(w.pauli_sum(n, [(1.0, "X" + "I" * (n - 1))]))
    tol = 1e-10 if dtype == 1 else 2e-5
    assert abs(yb.expect(s, zz)[0] - gold["zz01"][0]) <= tol
    assert abs(yb.expect(s, x0)[0] - gold["x0"][0]) <= tol
    psi = s.download()[:, 0]
    assert abs(psi[0] - complex(*gold["amp0"])) <= (1e-12 if dtype == 1 else 1e-6)
    assert abs(psi[-1] - complex(*gold["amp_last"])) <= (1e-12 if dtype == 1 else 1e-6)
    assert abs(np.vdot(psi, psi).real - 1) <= (1e-12 if dtype == 1 else 1e-4)


@pytest.mark.parametrize("dtype", [1, 0])
def test_forward_25q_energy(dtype):
    """Forward at scale: 25 qubits, depth 20 (512 MiB complex128 / 256 MiB complex64)."""
    path = os.path.join(GOLDEN, "fwd25_energy.txt")
    if not os.path.exists(path):
        pytest.skip("fwd25 golden not generated")
    gold = golden("fwd25_energy.txt")
    n = 25
    circ = w.hea_circuit(n, 20)
    s = yb.State(n, 1, dtype)
    yb.forward(s, yb.Circuit.from_workload(circ), w.angles(1, circ.nparams))
    e = yb.expect(s, yb.PauliSum.from_workload(w.heisenberg(n)))
    assert abs(e[0] - gold["energy"][0]) <= (1e-9 if dtype == 1 else 1e-5)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("width", [1, 2, 3, 4, 5])
def test_forward_with_dense_fusion_matches_oracle(dtype, width):
    """Forward sweeps folding gates into dense blocks of up to `width` qubits (4 and 5 run on
    FP32 matrix cores for complex64 states; 1 merges runs of one-qubit gates)."""
    yb.set_options(fuse_width=width, autotune=0)
    try:
        n = 11
        circ = w.random_gate_list(n, 70, seed=4000 + width, kmax=3, max_ctrl=2)
        params = w.angles(width, circ.nparams)
        psi0 = w.random_state(n, 3, width)
        s = yb.State(n, 3, dtype)
        s.upload(psi0)
        yb.forward(s, yb.Circuit.from_workload(circ), params)
        want = oracle.forward(circ, params, psi0)
        tol = 1e-11 if dtype == 1 else 2e-5
        assert np.abs(s.download() - want).max() <= tol
    finally:
        yb.set_options(fuse_width=0, autotune=1)


@pytest.mark.parametrize("mfma", [1, 0])
def test_random_circuit_20q_fused_5q_blocks(mfma):
    """Precision workload family at 20 qubits with 5-qubit fusion on complex64 (matrix cores
    when mfma = 1) against the oracle's observables, and its fidelity with the complex128
    unfused path."""
    gold = golden("rand20_observables.txt")
    n = 20
    circ = yb.Circuit.from_workload(w.random_circuit(n, 24, seed=5))
    ref = yb.State(n, 1, 1)
    yb.set_options(autotune=0)
    try:
        yb.forward(ref, circ, [])
        yb.set_options(fuse_width=5, mfma=mfma)
        s = yb.State(n, 1, 0)
        yb.forward(s, circ, [])
    finally:
        yb.set_options(fuse_width=0, mfma=1, autotune=1)
    zz = yb.PauliSum.from_workload(w.pauli_sum(n, [(1.0, "ZZ" + "I" * (n - 2))]))
    assert abs(yb.expect(s, zz)[0] - gold["zz01"][0]) <= 2e-5
    assert abs(yb.expect(ref, zz)[0] - gold["zz01"][0]) <= 1e-10
    fid = abs(yb.inner(ref, s)[0]) ** 2
    assert fid >= 1 - 1e-5
    assert abs(abs(yb.inner(ref, ref)[0]) - 1) <= 1e-12


def test_inner_product_matches_numpy():
    n, B = 9, 4
    a = w.random_state(n, B, 1)
    b = w.random_state(n, B, 2)
    sa, sb = yb.State(n, B, 1), yb.State(n, B, 0)
    sa.upload(a)
    sb.upload(b)
    got = yb.inner(sa, sb)
    want = np.sum(a.conj() * b.astype(np.complex64).astype(np.complex128), axis=0)
    np.testing.assert_allclose(got, want, atol=1e-12)
