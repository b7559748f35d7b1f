"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, and the
host-only calls (circuits, observables) validate their arguments."""
import ctypes

import numpy as np
import pytest

from paper_1912_10877_amd import binding as yb


def test_library_exports_every_declared_symbol():
    L = yb.lib()
    names = yb.header_symbols()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_circuit_push_validation():
    c = yb.Circuit(4)
    c.push("Rx", [0], param=0)
    c.push("X", [1], ctrls=[0])
    c.push("rot", [0, 1], param=3, G=np.kron(np.array([[0, 1], [1, 0]]), np.array([[0, 1], [1, 0]])))
    c.push("rot", [2], param=1, G=np.array([[0, -1j], [1j, 0]]))      # Y: Hermitian and reflexive
    assert c.nparams == 4
    bad = [
        dict(kind="Rx", locs=[4], param=0),             # loc out of range
        dict(kind="dense", locs=[0, 0], G=np.eye(4)),   # repeated qubit
        dict(kind="X", locs=[1], ctrls=[1]),            # control on the target
        dict(kind="X", locs=[1], ctrls=[0], cvals=[2]), # control value not 0/1
        dict(kind="X", locs=[0], param=2),              # fixed gate with a parameter
        dict(kind="rot", locs=[0], param=0),            # rot without generator
        dict(kind="Rx", locs=[0, 1], param=0),          # one-qubit kind on two qubits
        dict(kind="dense", locs=[0, 1, 2, 3, 0, 1], G=np.eye(64)),  # k too large / repeated
        dict(kind="rot", locs=[0], param=0, G=np.diag([1.0, 2.0])),        # Hermitian, G G != 1
        dict(kind="rot", locs=[0], param=0, G=np.array([[0, 1], [0, 0]])),  # not Hermitian
        dict(kind="rot", locs=[0], param=0, G=np.array([[0, 1j], [1j, 0]])),  # G G = -1, anti-Hermitian
        dict(kind="rot", locs=[0, 1], param=0, G=np.kron(np.eye(2), np.diag([1.0, 1.0 + 1e-9]))),
    ]
    for kw in bad:
        with pytest.raises(yb.YaoError) as ei:
            c.push(**kw)
        assert ei.value.code == -1
    assert c.nparams == 4


def test_pauli_sum_validation():
    yb.PauliSum(3, [1.0], [0b011], [0b010])
    with pytest.raises(yb.YaoError):
        yb.PauliSum(3, [1.0], [0b1000], [0])
    with pytest.raises(yb.YaoError):
        yb.PauliSum(3, [float("nan")], [1], [0])


def test_options_roundtrip_and_validation():
    o = yb.get_options()
    yb.set_options(plain=1, tile_qubits=10)
    assert yb.get_options().plain == 1 and yb.get_options().tile_qubits == 10
    with pytest.raises(yb.YaoError):
        yb.set_options(fuse_width=9)
    yb.set_options(plain=o.plain, tile_qubits=o.tile_qubits, fuse_width=o.fuse_width)


def test_state_calls_without_device_fail_cleanly():
    """With no gfx950 device visible, allocation reports YAO_ENODEV instead of crashing."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(yb.YaoError) as ei:
        yb.State(3)
    assert ei.value.code == -5
