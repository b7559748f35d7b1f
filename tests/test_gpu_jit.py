"""Run-time compiled forward passes (yao_options.jit) against the oracle: the ansatz workload
and random one-qubit gate lists with controls on register bits, other tile bits and qubits
outside the tile, in both dtypes; the compiled kernels read the matrices from the bound
records, so new angles after compiling must give new results; states of a batch and passes
with LDS-applied gates keep the generic kernels in the same sweep."""
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
    yb.set_options(jit=1, autotune=0, fuse_width=0)
    yield
    assert yb.jit_stats()["failures"] == 0
    yb.set_options(jit=3, autotune=1, fuse_width=0)


def tol(dtype, ngates):
    return 2e-6 * np.sqrt(ngates) + 1e-6 if dtype == 0 else 1e-11


def run_forward(c, params, dtype):
    s = yb.State(c.n, 1, dtype)
    yb.forward(s, yb.Circuit.from_workload(c), params)
    return s.download()


def random_bindable(n, ngates, seed):
    """One-qubit gates of the kinds the device binds (fixed gates, Rx, Ry, Rz, phase shift),
    each with up to two controls of random value anywhere in the register."""
    rng = np.random.default_rng(seed)
    kinds = ["X", "Y", "Z", "H", "S", "Sdag", "T", "Tdag", "Rx", "Ry", "Rz", "shift"]
    gates, p = [], 0
    for _ in range(ngates):
        kind = kinds[rng.integers(len(kinds))]
        q = rng.permutation(n)
        nc = int(rng.integers(0, 3))
        ctrls = tuple(int(x) for x in q[1:1 + nc])
        cvals = tuple(int(v) for v in rng.integers(0, 2, nc))
        if kind in ("Rx", "Ry", "Rz", "shift"):
            gates.append(w.Gate(kind, (int(q[0]),), param=p, ctrls=ctrls, cvals=cvals))
            p += 1
        else:
            gates.append(w.Gate(kind, (int(q[0]),), ctrls=ctrls, cvals=cvals))
    return w.Circuit(n, gates, p)


CASES = [("hea", 13, 3, 0), ("hea", 14, 4, 1), ("hea", 16, 5, 0), ("rand", 13, 60, 0), ("rand", 15, 80, 1),
         ("rand", 14, 90, 0)]


@pytest.mark.parametrize("kind,n,d,dtype", CASES)
@pytest.mark.parametrize("width", [0, 1])
def test_compiled_forward_matches_oracle(kind, n, d, dtype, width):
    yb.set_options(jit=1, autotune=0, fuse_width=width)
    if kind == "hea":
        c = w.hea_circuit(n, d)
    else:
        c = random_bindable(n, d, seed=800 + n + d)
    circ = yb.Circuit.from_workload(c)
    for rep in range(3):
        params = w.angles(900 + 17 * rep + n, c.nparams)
        s = yb.State(n, 1, dtype)
        l0 = yb.jit_stats()["fwd_launches"]
        yb.forward(s, circ, params)
        assert yb.jit_stats()["fwd_launches"] > l0, "no compiled pass ran"
        want = oracle.forward(c, params, w.zero_state(n))
        err = np.abs(s.download() - want).max()
        assert err <= tol(dtype, len(c.gates)), (rep, err)


def test_compiled_forward_inside_backward():
    """yao_backward's forward sweep takes the compiled passes too; energy and gradients match."""
    yb.set_options(jit=1, autotune=0, fuse_width=1)
    c = w.hea_circuit(14, 3)
    H = w.heisenberg(14)
    circ, h = yb.Circuit.from_workload(c), yb.PauliSum.from_workload(H)
    for rep in range(2):
        params = w.angles(950 + rep, c.nparams)
        s = yb.State(14, 1, 0)
        l0 = yb.jit_stats()["fwd_launches"]
        e, g, _ = yb.backward(s, circ, params, h)
        assert yb.jit_stats()["fwd_launches"] > l0, "the forward sweep did not use the compiled passes"
        e_ref, g_ref, _ = oracle.adjoint(H, c, params, w.zero_state(14))
        assert abs(e - e_ref[0]) <= 1e-5
        assert np.abs(np.asarray(g).ravel() - g_ref[0]).max() <= 1e-4 * max(1.0, np.abs(g_ref[0]).max())


def test_batched_and_lds_passes_keep_generic_kernels():
    """A batch of 3 slots and a circuit with 2-qubit gates (LDS-applied) in the same sweep
    as compiled passes of other circuits: all results match the oracle."""
    yb.set_options(jit=1, autotune=0, fuse_width=0)
    c = w.hea_circuit(13, 2)
    params = w.angles(977, c.nparams)
    s = yb.State(13, 3, 0)
    circ = yb.Circuit.from_workload(c)
    for _ in range(2):
        s.reset()
        yb.forward(s, circ, params)
    want = oracle.forward(c, params, w.zero_state(13, 3))
    assert np.abs(s.download() - want).max() <= tol(0, len(c.gates))
    c2 = w.random_gate_list(13, 40, seed=978, kmax=3, max_ctrl=1)
    p2 = w.angles(979, c2.nparams)
    for _ in range(2):
        got = run_forward(c2, p2, 0)
    assert np.abs(got - oracle.forward(c2, p2, w.zero_state(13))).max() <= tol(0, len(c2.gates))


@pytest.mark.parametrize("kind,n,d,dtype", [("hea", 13, 3, 0), ("hea", 14, 2, 1), ("hea", 16, 4, 0),
                                            ("rand", 13, 70, 0), ("rand", 15, 60, 1)])
def test_compiled_reverse_sweep_matches_oracle(kind, n, d, dtype):
    """Reverse passes compiled with their gradients: energy and every gradient against the
    oracle's adjoint, for two angle sets after compiling (the compiled code reads the
    bound records)."""
    yb.set_options(jit=1, autotune=0, fuse_width=0)
    c = w.hea_circuit(n, d) if kind == "hea" else random_bindable(n, d, seed=1100 + n + d)
    H = w.heisenberg(n)
    circ, h = yb.Circuit.from_workload(c), yb.PauliSum.from_workload(H)
    for rep in range(2):
        params = w.angles(1200 + 31 * rep + n, c.nparams)
        s = yb.State(n, 1, dtype)
        l0 = yb.jit_stats()["bwd_launches"]
        e, g, _ = yb.backward(s, circ, params, h)
        assert yb.jit_stats()["bwd_launches"] > l0, "the reverse sweep did not use the compiled passes"
        e_ref, g_ref, _ = oracle.adjoint(H, c, params, w.zero_state(n))
        te, tg = (1e-5, 1e-4) if dtype == 0 else (1e-10, 1e-9)
        assert abs(e - e_ref[0]) <= te, (rep, e, e_ref[0])
        scale = max(1.0, float(np.abs(g_ref[0]).max()))
        assert np.abs(np.asarray(g).ravel() - g_ref[0]).max() <= tg * scale, rep
        # The state keeps the forward sweep's output (the reverse sweep runs on its own copy).
        want = oracle.forward(c, params, w.zero_state(n))
        assert np.abs(s.download() - want).max() <= tol(dtype, len(c.gates))


def test_compiled_passes_inside_batch_units():
    """Circuits whose programs were compiled before a batch is recorded run their compiled
    passes inside the batch graph, over a unit of same-structure circuits (grid z, each circuit
    its own state and records): energies, gradients and output states against the oracle."""
    yb.set_options(jit=1, autotune=0, fuse_width=0)
    c = w.hea_circuit(13, 2)
    H = w.heisenberg(13)
    circs = [yb.Circuit.from_workload(c) for _ in range(3)]
    hams = [yb.PauliSum.from_workload(H) for _ in range(3)]
    states = [yb.State(13, 1, 0) for _ in range(3)]
    params = [w.angles(1300 + i, c.nparams) for i in range(3)]
    # Compile every circuit's forward and reverse programs through the eager path first.
    for i in range(3):
        yb.backward(states[i], circs[i], params[i], hams[i])
    st0 = yb.jit_stats()
    e, g = yb.batch_run(states, circs, params, hams)
    st1 = yb.jit_stats()
    # The graph was recorded with the compiled kernels (counted when recorded).
    assert st1["fwd_launches"] > st0["fwd_launches"] and st1["bwd_launches"] > st0["bwd_launches"]
    for rep in range(2):
        if rep:
            params = [w.angles(1400 + i, c.nparams) for i in range(3)]
            e, g = yb.batch_run(states, circs, params, hams)
        for i in range(3):
            e_ref, g_ref, _ = oracle.adjoint(H, c, params[i], w.zero_state(13))
            assert abs(e[i] - e_ref[0]) <= 1e-5, (rep, i)
            assert np.abs(g[i] - g_ref[0]).max() <= 1e-4 * max(1.0, float(np.abs(g_ref[0]).max())), (rep, i)
            want = oracle.forward(c, params[i], w.zero_state(13))
            assert np.abs(states[i].download() - want).max() <= tol(0, len(c.gates)), (rep, i)
