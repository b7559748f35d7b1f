"""GPU parity of the faithful gradient (eq. shiftrule, every shifted circuit in one register)
against the oracle's shift rule per gate occurrence and against the adjoint gradient where the
rule is exact."""
import os

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

yb = None
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    global yb
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_10877_amd import binding

    yb = binding
    yb.init()
    yield


def grad_tol(dtype, g_ref):
    return (1e-10 if dtype == 1 else 1e-4) * max(1.0, float(np.abs(g_ref).max()))


@pytest.mark.parametrize("dtype", [0, 1])
def test_shift_rule_10q_workload(dtype):
    """The 10-qubit, depth-5 ansatz (150 parameters): the rule's gradient equals the oracle's
    rule per occurrence and the adjoint gradient (uncontrolled rotations)."""
    n, depth = 10, 5
    circ = w.hea_circuit(n, depth)
    H = w.heisenberg(n)
    params = w.angles(0, circ.nparams)
    psi0 = w.zero_state(n)
    s = yb.State(n, 1, dtype)
    e, g = yb.shift_grad(s, yb.Circuit.from_workload(circ), params, yb.PauliSum.from_workload(H))
    g_sh = oracle.shift_grad_gates(H, circ, params, psi0)[0]
    e_ref, g_adj, _ = oracle.adjoint(H, circ, params, psi0)
    assert abs(e - e_ref[0]) <= (1e-10 if dtype == 1 else 1e-5)
    assert np.abs(g - g_sh).max() <= grad_tol(dtype, g_sh)
    assert np.abs(g - g_adj[0]).max() <= grad_tol(dtype, g_adj[0])
    np.testing.assert_array_equal(s.download()[:, 0], psi0[:, 0].astype(s.np_dtype))  # input unchanged


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("n,seed", [(6, 1), (9, 2), (14, 3)])
def test_shift_rule_controlled_and_shared(dtype, n, seed):
    """Random gates with controls (the rule's value for controlled rotations differs from the
    derivative, and the GPU must reproduce the rule), shift gates, rotations with dense
    generators and parameters shared by several gates, from a random input state."""
    circ = w.random_gate_list(n, 40, seed=6000 + seed, kmax=2, max_ctrl=2)
    shared = w.Circuit(n, [w.Gate(g.kind, g.locs, g.ctrls, g.cvals,
                                  param=(g.param % 7) if g.param >= 0 else -1, theta=g.theta, G=g.G)
                           for g in circ.gates], min(7, circ.nparams))
    params = w.angles(seed, shared.nparams)
    psi0 = w.random_state(n, 1, seed)
    H = w.heisenberg(n)
    s = yb.State(n, 1, dtype)
    s.upload(psi0)
    e, g = yb.shift_grad(s, yb.Circuit.from_workload(shared), params, yb.PauliSum.from_workload(H))
    g_sh = oracle.shift_grad_gates(H, shared, params, psi0)[0]
    assert abs(e - oracle.energy(H, shared, params, psi0)[0]) <= (1e-10 if dtype == 1 else 1e-5)
    assert np.abs(g - g_sh).max() <= grad_tol(dtype, g_sh)


def test_shift_rule_20q_workload_matches_adjoint_golden():
    """The 20-qubit differentiation workload (1200 parameters, 2401 circuits in one register of
    32 qubits): every gradient against the stored oracle adjoint gradient, and 24 against the
    oracle's stored shift-rule values."""
    def golden(name):
        out = {}
        for line in open(os.path.join(GOLDEN, name)):
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            out[k] = np.array([float(x) for x in v])
        return out
    gold = golden("vqe20_adjoint.txt")
    fd = golden("fd20.txt")
    n, depth = 20, 20
    circ = w.hea_circuit(n, depth)
    s = yb.State(n, 1, 0)
    e, g = yb.shift_grad(s, yb.Circuit.from_workload(circ), w.angles(2, circ.nparams),
                         yb.PauliSum.from_workload(w.heisenberg(n)))
    assert abs(e - gold["energy"][0]) <= 1e-5
    assert np.abs(g - gold["grad"]).max() <= grad_tol(0, gold["grad"])
    idx = fd["index"].astype(int)
    assert np.abs(g[idx] - fd["shift"]).max() <= grad_tol(0, fd["shift"])
