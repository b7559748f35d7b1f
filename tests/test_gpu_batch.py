"""GPU parity of the graph-recorded batch of uneven circuits (yao_batch_run) against the oracle:
energies and every gradient per circuit, replays with new parameters, autotuned and forced
fusion widths, re-recording after a circuit changes, batch lists called in turn, and the full
1024-circuit workload against stored oracle values."""
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
    yb.set_options(plain=0, tile_qubits=0, fuse_width=0, autotune=1)


def tol(dtype):
    # complex64 sweeps: |dE| <= 1e-5 and gradients within 1e-4 of the largest component;
    # complex128: rounding of FP64 arithmetic over a few hundred gates.
    return (1e-5, 1e-4) if dtype == 0 else (1e-10, 1e-9)


def make_batch(spec, dtype):
    states, circs, hams, params, refs = [], [], [], [], []
    for n, d, seed in spec:
        c = w.hea_circuit(n, d)
        H = w.heisenberg(n)
        states.append(yb.State(n, 1, dtype))
        circs.append(yb.Circuit.from_workload(c))
        hams.append(yb.PauliSum.from_workload(H))
        params.append(w.angles(seed, c.nparams))
        refs.append((c, H))
    return states, circs, hams, params, refs


def check(e, g, params, refs, dtype, which=None):
    te, tg = tol(dtype)
    for i in (range(len(refs)) if which is None else which):
        c, H = refs[i]
        e_ref, g_ref, _ = oracle.adjoint(H, c, params[i], w.zero_state(c.n))
        assert abs(e[i] - e_ref[0]) <= te, (i, c.n, e[i], e_ref[0])
        assert len(g[i]) == c.nparams
        if c.nparams == 0:
            continue
        scale = max(1.0, float(np.abs(g_ref[0]).max()))
        err = float(np.abs(g[i] - g_ref[0]).max())
        assert err <= tg * scale, (i, c.n, err)


SMALL = w.hetero_batch_spec(ncirc=24, seed=7, nmin=5, nmax=11, dmin=1, dmax=4)


@pytest.mark.parametrize("dtype", [0, 1])
def test_uneven_batch_matches_oracle(dtype):
    states, circs, hams, params, refs = make_batch(SMALL, dtype)
    e, g = yb.batch_run(states, circs, params, hams)
    check(e, g, params, refs, dtype)


def test_replays_with_new_parameters_and_eager_work_between():
    """The recorded graph is replayed with new angles; eager work on the bound stream runs
    between the replays; every replay matches the oracle."""
    states, circs, hams, params, refs = make_batch(SMALL[:10], 0)
    other = yb.State(9, 2, 0)
    H9 = yb.PauliSum.from_workload(w.heisenberg(9))
    for r in range(3):
        ps = [w.angles(5000 + 37 * r + i, len(p)) for i, p in enumerate(params)]
        e, g = yb.batch_run(states, circs, ps, hams)
        check(e, g, ps, [refs[i] for i in range(len(refs))], 0)
        yb.expect(other, H9)  # eager work between replays
        # the state of every circuit ends holding its output
        c0, _ = refs[0]
        out = states[0].download()
        ref = oracle.forward(c0, ps[0], w.zero_state(c0.n))
        assert np.abs(out - ref).max() <= 1e-5


def random_pauli_sum(n, nterms, seed):
    rng = np.random.default_rng(seed)
    terms = [(float(rng.uniform(-1, 1)), "".join("IXYZ"[int(k)] for k in rng.integers(0, 4, n))) for _ in range(nterms)]
    return w.pauli_sum(n, terms)


@pytest.mark.parametrize("dtype", [0, 1])
def test_small_circuits_general_gates(dtype):
    """Circuits whose state fits one tile run start to end in one workgroup each: random
    gates of every kind with controls and control values, 2- and 3-qubit dense gates, QFT,
    Haar-random layers and the paper's ansatz, under Heisenberg and random Pauli sums. Energies,
    gradients and the output states against the oracle. Circuits with parameterised 2- or
    3-qubit rotations cannot be bound on the device and take the pass path in the same batch."""
    circuits = []
    for i, n in enumerate([5, 6, 7, 8, 9, 10, 11, 12]):
        circuits.append(w.random_gate_list(n, 40, seed=6100 + i, kmax=3, max_ctrl=2))
        circuits.append(w.random_gate_list(n, 30, seed=6200 + i, kmax=1, max_ctrl=2))
    circuits += [w.qft_circuit(7), w.random_circuit(9, 3, seed=61), w.paper_variational_circuit(8, 2),
                 w.paper_variational_circuit(12, 3), w.ghz_circuit(12)]
    states, circs, hams, params, refs = [], [], [], [], []
    for i, c in enumerate(circuits):
        H = w.heisenberg(c.n) if i % 2 == 0 else random_pauli_sum(c.n, 6, 6300 + i)
        states.append(yb.State(c.n, 1, dtype))
        circs.append(yb.Circuit.from_workload(c))
        hams.append(yb.PauliSum.from_workload(H))
        params.append(w.angles(6400 + i, c.nparams))
        refs.append((c, H))
    for rep in range(2):
        if rep:
            params = [w.angles(6500 + i, len(p)) for i, p in enumerate(params)]
        e, g = yb.batch_run(states, circs, params, hams)
        check(e, g, params, refs, dtype)
        for i, (c, _) in enumerate(refs):
            ref = oracle.forward(c, params[i], w.zero_state(c.n))
            assert np.abs(states[i].download() - ref).max() <= (1e-5 if dtype == 0 else 1e-11), (i, c.n)


@pytest.mark.parametrize("dtype", [0, 1])
def test_uneven_batch_pass_path_matches_oracle(dtype):
    """States of 13..15 qubits span several tiles: the batch records their fused passes."""
    spec = w.hetero_batch_spec(ncirc=6, seed=9, nmin=13, nmax=15, dmin=1, dmax=3)
    states, circs, hams, params, refs = make_batch(spec, dtype)
    e, g = yb.batch_run(states, circs, params, hams)
    check(e, g, params, refs, dtype)


@pytest.mark.parametrize("width,tq", [(2, 6), (3, 0), (4, 7), (5, 0)])
def test_forced_fusion_width_and_tile(width, tq):
    """Fusion widths 4 and 5 put standalone dense blocks (matrix cores for complex64) into the
    graph; their matrices come from the uploaded program. (States of up to 12 qubits take the
    one-workgroup path, so most circuits here have more.)"""
    yb.set_options(autotune=0, fuse_width=width, tile_qubits=tq)
    try:
        spec = [(n, d, 300 + i) for i, (n, d) in enumerate([(6, 2), (13, 3), (14, 2), (13, 2), (15, 4)])]
        states, circs, hams, params, refs = make_batch(spec, 0)
        e, g = yb.batch_run(states, circs, params, hams)
        check(e, g, params, refs, 0)
        ps = [w.angles(77 + i, len(p)) for i, p in enumerate(params)]
        e, g = yb.batch_run(states, circs, ps, hams)
        check(e, g, ps, refs, 0)
    finally:
        yb.set_options(autotune=1, fuse_width=0, tile_qubits=0)


def test_autotuned_equals_untuned():
    spec = [(14, 3, 11), (12, 5, 12), (7, 2, 13)]
    states, circs, hams, params, refs = make_batch(spec, 0)
    e1, g1 = yb.batch_run(states, circs, params, hams)
    yb.set_options(autotune=0)
    try:
        e2, g2 = yb.batch_run(states, circs, params, hams)
    finally:
        yb.set_options(autotune=1)
    assert np.abs(np.array(e1) - np.array(e2)).max() <= 2e-5
    for a, b in zip(g1, g2):
        assert np.abs(a - b).max() <= 2e-4 * max(1.0, float(np.abs(b).max()))
    check(e1, g1, params, refs, 0)


def test_changed_circuit_is_recorded_anew():
    spec = [(6, 2, 21), (8, 2, 22)]
    states, circs, hams, params, refs = make_batch(spec, 1)
    e, g = yb.batch_run(states, circs, params, hams)
    check(e, g, params, refs, 1)
    # Append one more parametrised layer to circuit 1 (same parameter indices reused).
    c1, H1 = refs[1]
    extra = w.Circuit(c1.n, list(c1.gates) + [w.Gate("Ry", (3,), param=0)], c1.nparams)
    circs[1].push("Ry", (3,), param=0)
    refs[1] = (extra, H1)
    e, g = yb.batch_run(states, circs, params, hams)
    check(e, g, params, refs, 1)


@pytest.mark.parametrize("dtype", [0, 1])
def test_alternating_batch_lists_keep_their_graphs(dtype):
    """Two batch lists called in turn (and a third list sharing states and circuits with the
    first): each call replays the graph recorded for its own list, with new angles each time;
    every energy and gradient is checked against the oracle."""
    spec_a = [(7, 2, 41), (9, 3, 42), (13, 2, 43)]
    spec_b = [(6, 1, 44), (10, 2, 45), (12, 3, 46), (8, 2, 47)]
    sa, ca, ha, pa, ra = make_batch(spec_a, dtype)
    sb, cb, hb, pb, rb = make_batch(spec_b, dtype)
    for rep in range(3):
        pa = [w.angles(100 + 10 * rep + i, r[0].nparams) for i, r in enumerate(ra)]
        pb = [w.angles(200 + 10 * rep + i, r[0].nparams) for i, r in enumerate(rb)]
        e, g = yb.batch_run(sa, ca, pa, ha)
        check(e, g, pa, ra, dtype)
        e, g = yb.batch_run(sb, cb, pb, hb)
        check(e, g, pb, rb, dtype)
        # The first list's circuits in another order on the same states.
        e, g = yb.batch_run(sa[::-1], ca[::-1], pa[::-1], ha[::-1])
        check(e, g, pa[::-1], ra[::-1], dtype)


@pytest.mark.parametrize("dtype", [0, 1])
def test_same_structure_circuits_share_launches(dtype):
    """Circuits of one structure (same gates, same observable, same state shape) run every
    launch together over all of them, each with its own angles, state and scratch slice: five
    13-qubit and three 14-qubit ansatz circuits, beside a 13-qubit one under another observable
    and one with an extra gate (units of their own). Energies, gradients and output states
    against the oracle, then a replay with new angles."""
    base13, base14 = w.hea_circuit(13, 2), w.hea_circuit(14, 1)
    extra = w.Circuit(13, list(base13.gates) + [w.Gate("Ry", (5,), param=3)], base13.nparams)
    cases = [(base13, w.heisenberg(13))] * 5 + [(base14, w.heisenberg(14))] * 3
    cases += [(base13, random_pauli_sum(13, 7, 7100)), (extra, w.heisenberg(13))]
    states, circs, hams, params, refs = [], [], [], [], []
    for i, (c, H) in enumerate(cases):
        states.append(yb.State(c.n, 1, dtype))
        circs.append(yb.Circuit.from_workload(c))
        hams.append(yb.PauliSum.from_workload(H))
        params.append(w.angles(7200 + i, c.nparams))
        refs.append((c, H))
    for rep in range(2):
        if rep:
            params = [w.angles(7300 + i, len(p)) for i, p in enumerate(params)]
        e, g = yb.batch_run(states, circs, params, hams)
        check(e, g, params, refs, dtype)
        for i in (0, 4, 5, 7, 9):
            c = refs[i][0]
            ref = oracle.forward(c, params[i], w.zero_state(c.n))
            assert np.abs(states[i].download() - ref).max() <= (1e-5 if dtype == 0 else 1e-11), i


def test_circuit_without_parameters_and_observable_only():
    c = w.ghz_circuit(7)
    H = w.heisenberg(7)
    s = yb.State(7, 1, 1)
    e, g = yb.batch_run([s], [yb.Circuit.from_workload(c)], [np.zeros(0)], [yb.PauliSum.from_workload(H)])
    e_ref = oracle.energy(H, c, [], w.zero_state(7))
    assert abs(e[0] - e_ref[0]) <= 1e-12
    assert len(g[0]) == 0


def test_rejects_unsupported_states():
    c = w.hea_circuit(4, 1)
    s = yb.State(4, 1, 0)
    with pytest.raises(RuntimeError):
        yb.batch_run([s], [yb.Circuit.from_workload(c)], [w.angles(1, c.nparams)],
                     [yb.PauliSum.from_workload(w.heisenberg(4))])
    c6 = w.hea_circuit(6, 1)
    s2 = yb.State(6, 2, 0)
    with pytest.raises(RuntimeError):
        yb.batch_run([s2], [yb.Circuit.from_workload(c6)], [w.angles(1, c6.nparams)],
                     [yb.PauliSum.from_workload(w.heisenberg(6))])


def test_full_1024_circuit_workload():
    """1024 circuits, qubits uniform in 8..20 and depth in 4..16, in one recorded batch: the
    replay is bit-identical, and every circuit with n <= 16 plus 8 per n in 17..20 matches the
    energy and every gradient the oracle stored (tests/golden/make_golden.py c4)."""
    import os
    spec = w.hetero_batch_spec()
    states, circs, hams, params, refs = make_batch(spec, 0)
    e, g = yb.batch_run(states, circs, params, hams)
    e2, g2 = yb.batch_run(states, circs, params, hams)  # replay
    assert np.array_equal(np.array(e), np.array(e2))
    for a, b in zip(g, g2):
        assert np.array_equal(a, b)
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "c4_batch.npz"))
    idx, off = gold["index"], gold["offset"]
    assert len(idx) == sum(1 for n, _, _ in spec if n <= 16) + 4 * 8
    te, tg = tol(0)
    for j, i in enumerate(idx):
        g_ref = gold["grad"][off[j]:off[j + 1]]
        assert abs(e[i] - gold["energy"][j]) <= te, (i, spec[i], e[i], gold["energy"][j])
        assert len(g[i]) == len(g_ref)
        err = float(np.abs(g[i] - g_ref).max())
        assert err <= tg * max(1.0, float(np.abs(g_ref).max())), (i, spec[i], err)
