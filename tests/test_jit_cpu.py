"""Host-only checks of the run-time compiled passes: the generated source of each pass of a
device-bound program compiles for gfx950 (hipRTC, no GPU), passes outside the compiled form
are left to the generic kernel, and circuits the device cannot bind are refused."""
import pytest

import workloads as w
from paper_1912_10877_amd import binding as yb


@pytest.mark.parametrize("n,depth,dtype", [(8, 2, 0), (10, 2, 1)])
@pytest.mark.parametrize("reverse", [False, True])
def test_ansatz_passes_all_compile(n, depth, dtype, reverse):
    circ = yb.Circuit.from_workload(w.hea_circuit(n, depth))
    npass, njit = yb.jit_selfcheck(circ, dtype, reverse=reverse)
    assert npass >= 1 and njit == npass


def test_controlled_one_qubit_gates_compile():
    gates = [w.Gate("Rx", (0,), param=0), w.Gate("X", (3,), ctrls=(7, 1), cvals=(1, 0)),
             w.Gate("Ry", (5,), param=1, ctrls=(2,), cvals=(0,)), w.Gate("shift", (8,), param=2, ctrls=(0,), cvals=(1,)),
             w.Gate("H", (6,)), w.Gate("Z", (4,), ctrls=(8,), cvals=(1,))]
    circ = yb.Circuit.from_workload(w.Circuit(9, gates, 3))
    for reverse in (False, True):
        npass, njit = yb.jit_selfcheck(circ, 0, reverse=reverse)
        assert njit == npass


def test_two_qubit_gates_stay_generic():
    # A 2-qubit gate is applied in LDS by the generic kernel; its pass is not compiled.
    gates = [w.Gate("Rx", (q,), param=q) for q in range(8)]
    gates.append(w.Gate("dense", (1, 2), G=w.random_unitary(4, __import__("numpy").random.default_rng(3))))
    circ = yb.Circuit.from_workload(w.Circuit(8, gates, 8))
    npass, njit = yb.jit_selfcheck(circ, 1)
    assert njit < npass


def test_unbindable_circuit_is_refused():
    c = w.random_gate_list(8, 20, seed=6, kmax=1, max_ctrl=1)
    assert any(g.kind == "rot" and g.param >= 0 for g in c.gates)  # a parametrised generator
    with pytest.raises(RuntimeError):
        yb.jit_selfcheck(yb.Circuit.from_workload(c), 0)
