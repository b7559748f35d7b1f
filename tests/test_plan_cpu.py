"""Host checks of the pass planner (no GPU): each plan is run on the host the way the pass
kernels run it -- tiles gathered through the plan's qubit layout, ops from their device
records on tile bits, tiles stored back through each pass's bit permutation, standalone gates
on the layout's index bits -- and compared with the gates applied one by one."""
import numpy as np
import pytest

import workloads as w
from paper_1912_10877_amd import binding as yb


def with_wide_gate(circ, k, seed):
    rng = np.random.default_rng(seed)
    q = rng.permutation(circ.n)
    g = w.Gate("dense", tuple(int(x) for x in q[:k]), ctrls=(int(q[k]),), cvals=(1,), G=w.random_unitary(1 << k, rng))
    gates = list(circ.gates)
    gates.insert(len(gates) // 3, g)
    return w.Circuit(circ.n, gates, circ.nparams)


@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("n,depth,tq", [(14, 6, 0), (16, 8, 0), (16, 5, 7), (13, 4, 5)])
def test_layered_plans_match_gate_by_gate(n, depth, tq, dtype, reverse):
    circ = w.hea_circuit(n, depth)
    c = yb.Circuit.from_workload(circ)
    err, npass = yb.plan_selfcheck(c, w.angles(n + depth, circ.nparams), dtype, reverse, tq)
    assert err < 1e-11, (err, npass)
    assert npass >= 1


@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("n,seed", [(13, 1), (15, 2), (16, 3)])
def test_random_plans_with_wide_gates_match_gate_by_gate(n, seed, reverse):
    """2- and 3-qubit gates (LDS ops, dense register blocks), controls inside and outside the
    tile, and 4- and 5-qubit gates that run as standalone launches inside permuted layouts."""
    circ = w.random_gate_list(n, 150, seed=seed, kmax=3, max_ctrl=2)
    circ = with_wide_gate(with_wide_gate(circ, 4, seed), 5, seed + 7)
    c = yb.Circuit.from_workload(circ)
    for tq in (0, 6):
        err, npass = yb.plan_selfcheck(c, w.angles(seed, circ.nparams), 0, reverse, tq)
        assert err < 1e-11, (tq, err, npass)


def test_layout_planner_beats_one_layer_per_pass():
    """On a layered ansatz whose CNOT chain spans every qubit, tiles of 12 of 16 qubits cover the
    16-qubit depth-12 circuit in well under one pass per layer."""
    circ = w.hea_circuit(16, 12)
    c = yb.Circuit.from_workload(circ)
    for reverse in (False, True):
        err, npass = yb.plan_selfcheck(c, w.angles(3, circ.nparams), 0, reverse, 0)
        assert err < 1e-11
        assert npass <= 8, npass


@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("seed", [1, 2])
def test_gates_sharing_only_controls_reorder_correctly(seed, reverse):
    """Rotations on low qubits controlled by a shared set of high qubits (with different control
    values, the shape of the shifted-circuit register of the faithful gradient), mixed with
    CNOTs whose targets are those control qubits: the planner lets gates that share only
    control qubits pass each other, but never past a gate that targets one of them."""
    rng = np.random.default_rng(seed)
    n, hi = 16, [12, 13, 14, 15]
    gates, p = [], 0
    for layer in range(6):
        for q in range(12):
            gates.append(w.Gate("Rx", (q,), param=p))
            p += 1
            if rng.random() < 0.5:
                cv = tuple(int(v) for v in rng.integers(0, 2, len(hi)))
                gates.append(w.Gate(["Rx", "Ry", "Rz"][int(rng.integers(3))], (q,), ctrls=tuple(hi), cvals=cv,
                                    theta=float(rng.uniform(0, 6.3))))
        for q in range(11):
            gates.append(w.Gate("X", (q + 1,), ctrls=(q,)))
        gates.append(w.Gate("X", (hi[layer % 4],), ctrls=(int(rng.integers(12)),)))
    circ = w.Circuit(n, gates, p)
    c = yb.Circuit.from_workload(circ)
    for tq in (0, 6):
        err, npass = yb.plan_selfcheck(c, w.angles(seed, p), 1, reverse, tq)
        assert err < 1e-11, (tq, err, npass)
