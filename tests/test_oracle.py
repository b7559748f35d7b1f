"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here checks the oracle against something other than itself: values the paper
prints, full Kronecker-product matrices built with numpy, library routines (scipy's expm,
numpy's ifft and eigvalsh), closed forms, invariants and finite differences.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads as w

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

PAULI = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], complex),
    "Y": np.array([[0, -1j], [1j, 0]], complex),
    "Z": np.array([[1, 0], [0, -1]], complex),
}
P0 = np.array([[1, 0], [0, 0]], complex)
P1 = np.array([[0, 0], [0, 1]], complex)


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out[key] = [float(v) for v in vals]
    return out


# ---------------------------------------------------------------------------------------
# Full-register matrices built only from numpy.kron (qubit 0 is the rightmost factor).
# ---------------------------------------------------------------------------------------

def kron_list(ops):
    """ops[q] acts on qubit q; returns kron(ops[n-1], ..., ops[0])."""
    m = np.ones((1, 1), complex)
    for op in ops:
        m = np.kron(op, m)
    return m


def embed_operator(n, U, locs, ctrls=(), cvals=()):
    """F = Pi (U on locs) + (1 - Pi): U expanded in the Pauli basis of its k qubits, each
    term placed with kron; Pi is the projector onto the control configuration."""
    k = len(locs)
    d = 1 << k
    Uemb = np.zeros((1 << n, 1 << n), complex)
    for code in range(4 ** k):
        letters = ["IXYZ"[(code >> (2 * j)) & 3] for j in range(k)]  # letters[j] on locs[j]
        sig = np.ones((1, 1), complex)
        for j in range(k):
            sig = np.kron(PAULI[letters[j]], sig)
        c = np.trace(sig.conj().T @ U) / d
        if abs(c) < 1e-15:
            continue
        ops = [PAULI["I"]] * n
        for j, q in enumerate(locs):
            ops[q] = PAULI[letters[j]]
        Uemb += c * kron_list(ops)
    ops = [PAULI["I"]] * n
    for c_, v in zip(ctrls, cvals):
        ops[c_] = P1 if v else P0
    Pi = kron_list(ops)
    return Pi @ Uemb + (np.eye(1 << n) - Pi)


def dense_hamiltonian(n, periodic=True):
    H = np.zeros((1 << n, 1 << n), complex)
    nb = n if periodic else n - 1
    for i in range(nb):
        j = (i + 1) % n
        for s in "XYZ":
            ops = [PAULI["I"]] * n
            ops[i] = PAULI[s]
            ops[j] = PAULI[s]
            H += kron_list(ops)
    return H


def gate_full_matrix(n, g, theta):
    """Full-register matrix of one gate, from expm / literal matrices and kron."""
    if g.kind in ("Rx", "Ry", "Rz"):
        U = scipy.linalg.expm(-1j * theta / 2 * PAULI[g.kind[1].upper()])
    elif g.kind == "rot":
        U = scipy.linalg.expm(-1j * theta / 2 * g.G)
    elif g.kind == "shift":
        U = np.diag([1, np.exp(1j * theta)])
    elif g.kind == "dense":
        U = g.G
    else:
        U = {"X": PAULI["X"], "Y": PAULI["Y"], "Z": PAULI["Z"],
             "H": np.array([[1, 1], [1, -1]]) / math.sqrt(2), "S": np.diag([1, 1j]), "Sdag": np.diag([1, -1j]),
             "T": np.diag([1, np.exp(1j * math.pi / 4)]), "Tdag": np.diag([1, np.exp(-1j * math.pi / 4)])}[g.kind]
    return embed_operator(n, np.asarray(U, complex), g.locs, g.ctrls, g.cvals)


# ---------------------------------------------------------------------------------------
# Paper's printed values.
# ---------------------------------------------------------------------------------------

def test_symbolic_differentiation_example():
    """App. "Symbolic Differentiation": E and the three gradients printed for Float64."""
    gold = read_golden("symad_3q.txt")
    circ = w.symad_example()
    e, g, back = oracle.adjoint(w.heisenberg(3), circ, gold["params"], w.zero_state(3))
    assert abs(e[0] - gold["energy"][0]) <= 1e-14
    np.testing.assert_allclose(g[0], gold["grad"], rtol=0, atol=1e-14)
    assert np.abs(back - w.zero_state(3)).max() < 1e-14


def test_symbolic_example_needs_periodic_heisenberg():
    """The open chain of the Listing "Heisenberg Hamiltonian" does not give the printed E."""
    gold = read_golden("symad_3q.txt")
    e_open = oracle.energy(w.heisenberg(3, periodic=False), w.symad_example(), gold["params"], w.zero_state(3))
    assert abs(e_open[0] - gold["energy"][0]) > 0.1


def test_instruct_x_little_endian():
    """Listing "instruct! and measure": X on (1-based) qubit 2 of zero_state(4) reads 0010."""
    circ = w.Circuit(4, [w.Gate("X", (1,))], 0)
    psi = oracle.forward(circ, None, w.zero_state(4))
    assert np.argmax(np.abs(psi[:, 0])) == 0b0010
    assert abs(abs(psi[2, 0]) - 1) < 1e-15
    bits = [(2 >> q) & 1 for q in range(4)]
    assert bits == [0, 1, 0, 0]


def test_hadamard_decomposition_convention():
    """Listing "gate decomposition": Rz(pi/2) Rx(pi/2) Rz(pi/2) is H up to the global phase -i."""
    rz = oracle.gate_matrix(w.Gate("Rz", (0,), param=0), math.pi / 2)
    rx = oracle.gate_matrix(w.Gate("Rx", (0,), param=0), math.pi / 2)
    Hm = oracle.gate_matrix(w.Gate("H", (0,)))
    np.testing.assert_allclose(rz @ rx @ rz, -1j * Hm, atol=1e-15)


def test_qft_tree_angles():
    """Listing "quantum Fourier transform": qft(3) angles pi/2 and pi/4 in that order."""
    c = w.qft_circuit(3)
    assert [g.kind for g in c.gates] == ["H", "shift", "shift", "H", "shift", "H"]
    assert c.gates[1].theta == 1.5707963267948966 and c.gates[1].ctrls == (1,)
    assert c.gates[2].theta == 0.7853981633974483 and c.gates[2].ctrls == (2,)


def test_paper_ansatz_gate_counts():
    """Listing "10000-layer VQE": Rz 200000, Rx 100010, CNOT 100000, 300010 parameters."""
    c = w.paper_variational_circuit(10, 10000)
    cnt = c.gate_counts()
    assert cnt[("Rz", 0)] == 200000
    assert cnt[("Rx", 0)] == 100010
    assert cnt[("X", 1)] == 100000
    assert c.nparams == 300010


# ---------------------------------------------------------------------------------------
# Gate semantics against Kronecker-product matrices (library routine: numpy.kron).
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_apply_matches_kronecker(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 7))
    k = int(rng.integers(1, min(3, n) + 1))
    q = rng.permutation(n)
    locs = tuple(int(x) for x in q[:k])
    nc = int(rng.integers(0, min(2, n - k) + 1))
    ctrls = tuple(int(x) for x in q[k:k + nc])
    cvals = tuple(int(x) for x in rng.integers(0, 2, nc))
    U = w.random_unitary(1 << k, rng)
    B = int(rng.integers(1, 4))
    psi = w.random_state(n, B, seed)
    F = embed_operator(n, U, locs, ctrls, cvals)
    got = oracle.apply_matrix(psi, n, U, locs, ctrls, cvals)
    np.testing.assert_allclose(got, F @ psi, atol=1e-13)


def test_locs_order_is_bit_order_of_matrix_index():
    """kron(A, B) on locs (l0, l1) puts B on l0 (reading: locs[j] is bit j of U's index)."""
    rng = np.random.default_rng(7)
    A = w.random_unitary(2, rng)
    Bm = w.random_unitary(2, rng)
    n = 3
    psi = w.random_state(n, 1, 3)
    got = oracle.apply_matrix(psi, n, np.kron(A, Bm), (2, 0))
    want = kron_list([A, PAULI["I"], Bm]) @ psi  # ops[q] acts on qubit q: B on l0 = 2, A on l1 = 0
    np.testing.assert_allclose(got, want, atol=1e-14)


@pytest.mark.parametrize("seed", range(6))
def test_circuit_matches_kronecker_product(seed):
    n = 4
    circ = w.random_gate_list(n, 12, seed=100 + seed, kmax=3)
    params = w.angles(seed, circ.nparams)
    psi = w.random_state(n, 2, seed)
    want = psi.copy()
    for g in circ.gates:
        th = params[g.param] if g.param >= 0 else g.theta
        want = gate_full_matrix(n, g, th) @ want
    got = oracle.forward(circ, params, psi)
    np.testing.assert_allclose(got, want, atol=1e-12)


@pytest.mark.parametrize("kind", ["Rx", "Ry", "Rz", "shift", "rot"])
def test_gate_matrix_and_derivative_vs_expm(kind):
    rng = np.random.default_rng(11)
    G = w.random_pauli_matrix(2, rng) if kind == "rot" else None
    g = w.Gate(kind, (0, 1) if kind == "rot" else (0,), param=0, G=G)
    th, h = 1.234, 1e-6

    def ref(t):
        if kind == "shift":
            return np.diag([1, np.exp(1j * t)])
        gen = G if kind == "rot" else PAULI[kind[1].upper()]
        return scipy.linalg.expm(-1j * t / 2 * gen)

    np.testing.assert_allclose(oracle.gate_matrix(g, th), ref(th), atol=1e-14)
    np.testing.assert_allclose(oracle.gate_deriv(g, th), (ref(th + h) - ref(th - h)) / (2 * h), atol=1e-9)


def test_dagger_rule_rotation():
    """Sec. "Manipulating Quantum Circuits": R(theta)^dagger = R(-theta)."""
    for kind in ("Rx", "Ry", "Rz"):
        g = w.Gate(kind, (0,), param=0)
        np.testing.assert_allclose(oracle.gate_matrix(g, 0.9).conj().T, oracle.gate_matrix(g, -0.9), atol=1e-15)


# ---------------------------------------------------------------------------------------
# Closed forms.
# ---------------------------------------------------------------------------------------

def bit_reverse(x, n):
    return int(format(x, f"0{n}b")[::-1], 2)


@pytest.mark.parametrize("n", [1, 3, 4, 6])
def test_qft_closed_form(n):
    """QFT |x> = N^{-1/2} sum_y exp(2 pi i rev(x) y / N) |y>, qubit-reversed output as in
    App. "Extending QBIR" (invorder then sqrt(N) ifft)."""
    N = 1 << n
    circ = w.qft_circuit(n)
    for x in range(N):
        psi = np.zeros((N, 1), complex)
        psi[x] = 1
        got = oracle.forward(circ, None, psi)[:, 0]
        y = np.arange(N)
        want = np.exp(2j * math.pi * bit_reverse(x, n) * y / N) / math.sqrt(N)
        np.testing.assert_allclose(got, want, atol=1e-13)
    psi = w.random_state(n, 1, 5)[:, 0]
    perm = np.array([bit_reverse(i, n) for i in range(N)])
    want = math.sqrt(N) * np.fft.ifft(psi[perm])
    np.testing.assert_allclose(oracle.forward(circ, None, psi)[:, 0], want, atol=1e-13)


def test_iqft_undoes_qft():
    """Listing "inverse QFT": reversed order, negated shift angles, H unchanged."""
    n = 5
    q = w.qft_circuit(n)
    inv = w.Circuit(n, [w.Gate(g.kind, g.locs, g.ctrls, g.cvals, theta=-g.theta) for g in reversed(q.gates)], 0)
    psi = w.random_state(n, 2, 9)
    back = oracle.forward(inv, None, oracle.forward(q, None, psi))
    np.testing.assert_allclose(back, psi, atol=1e-13)


@pytest.mark.parametrize("n", [3, 5, 8])
def test_ghz_state_and_energy(n):
    psi = oracle.forward(w.ghz_circuit(n), None, w.zero_state(n))[:, 0]
    want = np.zeros(1 << n, complex)
    want[0] = want[-1] = 1 / math.sqrt(2)
    np.testing.assert_allclose(psi, want, atol=1e-15)
    re, im = oracle.expect(w.heisenberg(n), psi)
    assert abs(re[0] - n) < 1e-13 and abs(im[0]) < 1e-14


def test_zero_angles_energy_and_gradient():
    n = 6
    circ = w.hea_circuit(n, 3)
    e, g, _ = oracle.adjoint(w.heisenberg(n), circ, np.zeros(circ.nparams), w.zero_state(n))
    assert abs(e[0] - n) < 1e-13
    assert np.abs(g).max() < 1e-13


def bloch_after_rx_rz_rx(a, b, c):
    return np.array([math.sin(a) * math.sin(b),
                     -math.sin(a) * math.cos(b) * math.cos(c) - math.cos(a) * math.sin(c),
                     -math.sin(a) * math.cos(b) * math.sin(c) + math.cos(a) * math.cos(c)])


def product_energy(n, params):
    r = [bloch_after_rx_rz_rx(*params[3 * q:3 * q + 3]) for q in range(n)]
    return sum(float(np.dot(r[i], r[(i + 1) % n])) for i in range(n))


def test_product_state_energy_and_gradient_closed_form():
    """Without the CNOTs the state is a product of single-qubit states, so each bond gives
    the dot product of the two Bloch vectors; its derivative pins the adjoint gradient."""
    n = 7
    full = w.hea_circuit(n, 1)
    circ = w.Circuit(n, [g for g in full.gates if g.kind != "X"], full.nparams)
    params = w.angles(3, circ.nparams)
    e, g, _ = oracle.adjoint(w.heisenberg(n), circ, params, w.zero_state(n))
    assert abs(e[0] - product_energy(n, params)) < 1e-13
    h = 1e-5
    for k in range(circ.nparams):
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        fd = (product_energy(n, pp) - product_energy(n, pm)) / (2 * h)
        assert abs(g[0, k] - fd) < 1e-8


@pytest.mark.parametrize("n,e0", [(4, -8.0), (6, -11.2111025509), (8, -14.6043736357)])
def test_hamiltonian_against_dense_matrix(n, e0):
    """H psi against the kron-built matrix; eigvalsh gives the ground energy, a lower bound."""
    H = dense_hamiltonian(n)
    assert abs(np.linalg.eigvalsh(H)[0] - e0) < 1e-9
    psi = w.random_state(n, 2, n)
    np.testing.assert_allclose(oracle.hpsi(w.heisenberg(n), psi), H @ psi, atol=1e-13)
    circ = w.hea_circuit(n, 2)
    e = oracle.energy(w.heisenberg(n), circ, w.angles(n, circ.nparams), w.zero_state(n))
    assert e[0] >= e0 - 1e-12


def test_heisenberg_bond_is_twice_swap_minus_one():
    """sigma.sigma = 2 SWAP - 1 on each bond: E = 2 sum_b Re<psi|SWAP_b|psi> - n_bonds, with
    SWAP done as a numpy index permutation."""
    n = 6
    psi = w.random_state(n, 1, 21)[:, 0]
    idx = np.arange(1 << n)
    total = 0.0
    for i in range(n):
        j = (i + 1) % n
        bi, bj = (idx >> i) & 1, (idx >> j) & 1
        swapped = idx & ~((1 << i) | (1 << j)) | (bi << j) | (bj << i)
        total += 2 * np.real(np.vdot(psi, psi[swapped])) - 1
    re, im = oracle.expect(w.heisenberg(n), psi)
    assert abs(re[0] - total) < 1e-13 and abs(im[0]) < 1e-14


def test_pauli_string_phases():
    """Y|0> = i|1>, Y|1> = -i|0>: Y_0 Y_1 on |00> is -|11>."""
    n = 2
    psi = w.zero_state(n)
    out = oracle.pauli_apply(n, psi, 0b11, 0b11)[:, 0]
    np.testing.assert_allclose(out, [0, 0, 0, -1], atol=1e-15)


# ---------------------------------------------------------------------------------------
# Invariants and gradient pins.
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_norm_preserved_and_uncompute_returns_input(seed):
    n = 6
    circ = w.random_gate_list(n, 40, seed=300 + seed, kmax=3)
    params = w.angles(seed, circ.nparams)
    psi = w.random_state(n, 2, seed)
    out = oracle.forward(circ, params, psi)
    np.testing.assert_allclose(np.sum(np.abs(out) ** 2, axis=0), [1, 1], atol=1e-13)
    _, _, back = oracle.adjoint(w.heisenberg(n), circ, params, psi)
    np.testing.assert_allclose(back, psi, atol=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_adjoint_gradient_vs_finite_differences(seed):
    """Central differences with h = 1e-4 in FP64 on random circuits with controlled
    rotations, shift gates, multi-qubit rot gates and dense gates."""
    n = 5
    circ = w.random_gate_list(n, 25, seed=500 + seed, kmax=3)
    params = w.angles(seed, circ.nparams)
    psi = w.random_state(n, 2, seed)
    H = w.heisenberg(n)
    _, g, _ = oracle.adjoint(H, circ, params, psi)
    fd = oracle.fd_grad(H, circ, params, psi, h=1e-4)
    for k, v in fd.items():
        np.testing.assert_allclose(g[:, k], v, atol=2e-7)


def test_parameter_shift_exact_for_uncontrolled_rotations():
    """eq. shiftrule is exact for Rx/Rz with reflexive generators."""
    n = 5
    circ = w.hea_circuit(n, 2)
    params = w.angles(0, circ.nparams)
    H = w.heisenberg(n)
    _, g, _ = oracle.adjoint(H, circ, params, w.zero_state(n))
    sh = oracle.shift_grad(H, circ, params, w.zero_state(n))
    for k, v in sh.items():
        assert abs(g[0, k] - v[0]) < 1e-12


def test_parameter_shift_does_not_hold_for_controlled_rotation():
    """The controlled Ry of the appendix example has a non-reflexive full generator."""
    gold = read_golden("symad_3q.txt")
    sh = oracle.shift_grad(w.heisenberg(3), w.symad_example(), gold["params"], w.zero_state(3), which=[1])
    assert abs(sh[1][0] - gold["grad"][1]) > 0.1


def test_batched_register_is_independent_states():
    """Sec. "Batched Quantum Registers": each slot evolves alone; the paper's batched
    gradient is the sum over slots."""
    n = 5
    circ = w.hea_circuit(n, 2)
    params = w.angles(1, circ.nparams)
    H = w.heisenberg(n)
    psi = w.random_state(n, 3, 4)
    e, g, _ = oracle.adjoint(H, circ, params, psi)
    for b in range(3):
        e1, g1, _ = oracle.adjoint(H, circ, params, psi[:, b:b + 1])
        assert abs(e[b] - e1[0]) < 1e-14
        np.testing.assert_allclose(g[b], g1[0], atol=1e-14)


def test_shared_parameter_gradients_add():
    """Sec. "Reverse Mode": reusing a parameter accumulates its gradient."""
    n = 3
    gates = [w.Gate("Rx", (0,), param=0), w.Gate("X", (1,), ctrls=(0,)), w.Gate("Ry", (1,), param=1),
             w.Gate("Rx", (2,), param=0), w.Gate("Rz", (0,), ctrls=(2,), cvals=(0,), param=1)]
    circ = w.Circuit(n, gates, 2)
    params = np.array([0.4, 1.3])
    H = w.heisenberg(n)
    _, g, _ = oracle.adjoint(H, circ, params, w.zero_state(n))
    fd = oracle.fd_grad(H, circ, params, w.zero_state(n))
    assert abs(g[0, 0] - fd[0][0]) < 1e-8 and abs(g[0, 1] - fd[1][0]) < 1e-8


def test_haar_su2_inputs_are_special_unitary():
    rng = np.random.default_rng(0)
    for _ in range(20):
        U = w.haar_su2(rng)
        np.testing.assert_allclose(U @ U.conj().T, np.eye(2), atol=1e-14)
        assert abs(np.linalg.det(U) - 1) < 1e-14


# ---------------------------------------------------------------------------------------
# Qubit management, QFT emulation, measurement, time evolution, faithful gradient.
# ---------------------------------------------------------------------------------------

def numpy_permute(psi, n, perm):
    """Qubit q -> position perm[q] through numpy's transpose of the [2]*n tensor (tensor axis
    a holds qubit n-1-a)."""
    B = psi.shape[1]
    t = psi.reshape([2] * n + [B])
    axes = [0] * n
    for q in range(n):
        axes[n - 1 - perm[q]] = n - 1 - q
    return np.transpose(t, axes + [n]).reshape(1 << n, B)


@pytest.mark.parametrize("seed", range(4))
def test_permute_qubits_matches_numpy_transpose(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 7))
    perm = rng.permutation(n).tolist()
    psi = w.random_state(n, 3, seed)
    np.testing.assert_array_equal(oracle.permute_qubits(psi, n, perm), numpy_permute(psi, n, perm))


def test_focus_relax_listing_example():
    """Listing "focus! and relax!": focus!(reg, (3,6,1,2)) on a 10-qubit register, qft(4) on
    the active qubits, relax! back, equals the QFT circuit placed on those qubits."""
    n, locs = 10, [2, 5, 0, 1]  # 1-based (3, 6, 1, 2)
    psi = w.random_state(n, 2, 77)
    f = oracle.focus(psi, n, locs)
    # the 4 active qubits are the lowest; the QFT circuit acts on them
    q4 = w.qft_circuit(4)
    circ_low = w.Circuit(n, list(q4.gates), 0)
    got = oracle.relax(oracle.forward(circ_low, None, f), n, locs)
    placed = w.Circuit(n, [w.Gate(g.kind, tuple(locs[q] for q in g.locs), tuple(locs[c] for c in g.ctrls), g.cvals,
                                  theta=g.theta) for g in q4.gates], 0)
    np.testing.assert_allclose(got, oracle.forward(placed, None, psi), atol=1e-13)
    np.testing.assert_allclose(oracle.relax(f, n, locs), psi, atol=0)
    # active qubit j of the focused register is qubit locs[j] of the original
    x = w.zero_state(n)
    x[:, 0] = 0
    x[(1 << 5) | (1 << 1), 0] = 1  # qubits 5 and 1 set
    fx = oracle.focus(x, n, locs)
    assert np.argmax(np.abs(fx[:, 0])) == (1 << 1) | (1 << 3)


@pytest.mark.parametrize("n,locs", [(4, [0, 1, 2, 3]), (6, [5, 1, 3]), (7, [2, 6, 0, 4, 1])])
def test_qft_definition_matches_circuit_and_fft(n, locs):
    """The QFT by its matrix definition on locs equals the gate circuit of Listing "QFT circuit"
    placed on locs, and on all qubits equals sqrt(N) ifft after reversing the qubit order
    (App. "Extending QBIR", with numpy's FFT); the inverse undoes it."""
    psi = w.random_state(n, 2, n + len(locs))
    k = len(locs)
    qk = w.qft_circuit(k)
    placed = w.Circuit(n, [w.Gate(g.kind, tuple(locs[q] for q in g.locs), tuple(locs[c] for c in g.ctrls), g.cvals,
                                  theta=g.theta) for g in qk.gates], 0)
    got = oracle.qft(psi, n, locs)
    np.testing.assert_allclose(got, oracle.forward(placed, None, psi), atol=1e-13)
    np.testing.assert_allclose(oracle.qft(got, n, locs, inverse=True), psi, atol=1e-13)
    if locs == list(range(n)):
        N = 1 << n
        perm = np.array([bit_reverse(i, n) for i in range(N)])
        for b in range(2):
            np.testing.assert_allclose(got[:, b], math.sqrt(N) * np.fft.ifft(psi[perm, b]), atol=1e-13)
    idx = [3, 17 % (1 << n), (1 << n) - 1]
    np.testing.assert_allclose(oracle.qft(psi, n, locs, idx=idx), got[idx], atol=0)


def test_measure_listing_example():
    """Listing "instruct! and measure": X on (1-based) qubit 2 of zero_state(4); three shots all
    read 0010."""
    psi = oracle.forward(w.Circuit(4, [w.Gate("X", (1,))], 0), None, w.zero_state(4))
    out = oracle.sample(psi, 4, [0, 1, 2, 3], np.array([[0.0, 0.37, 0.999]]))
    assert out.tolist() == [[0b0010] * 3]


def test_probs_closed_forms():
    n = 5
    ghz = oracle.forward(w.ghz_circuit(n), None, w.zero_state(n))
    p = oracle.probs(ghz, n, list(range(n)))[0]
    want = np.zeros(1 << n)
    want[0] = want[-1] = 0.5
    np.testing.assert_allclose(p, want, atol=1e-15)
    np.testing.assert_allclose(oracle.probs(ghz, n, [3, 1])[0], [0.5, 0, 0, 0.5], atol=1e-15)
    # product state Rx(a_q)|0>: P(bit q = 1) = sin^2(a_q / 2), marginals multiply
    a = np.random.default_rng(3).uniform(0, 2 * math.pi, n)
    circ = w.Circuit(n, [w.Gate("Rx", (q,), theta=a[q]) for q in range(n)], 0)
    psi = oracle.forward(circ, None, w.zero_state(n))
    locs = [4, 0, 2]
    p1 = np.sin(a / 2) ** 2
    want = np.array([np.prod([p1[q] if (x >> j) & 1 else 1 - p1[q] for j, q in enumerate(locs)])
                     for x in range(8)])
    np.testing.assert_allclose(oracle.probs(psi, n, locs)[0], want, atol=1e-15)


def test_probs_and_sampling_rule():
    """probs against |psi|^2 summed with numpy; the inverse-CDF rule on a distribution with
    zeros (p = 1/4 at outcomes 0, 2, 3, 5, so the CDF is exact): zero-probability outcomes never
    come out, and u on a CDF step moves to the next outcome; shot frequencies of a random state
    within 5 sigma."""
    n = 6
    psi = w.random_state(n, 2, 12)
    locs = [1, 4]
    t = (np.abs(psi) ** 2).reshape([2] * n + [2])
    want = np.zeros((2, 4))
    for i in range(1 << n):
        x = ((i >> 1) & 1) | (((i >> 4) & 1) << 1)
        want[:, x] += np.abs(psi[i]) ** 2
    np.testing.assert_allclose(oracle.probs(psi, n, locs), want, atol=1e-15)
    amp = np.array([0.5, 0, 0.5, 0.5, 0, 0.5, 0, 0])[:, None]  # p = 1/4 at 0, 2, 3, 5: exact
    u = np.array([[0.0, 0.2499, 0.25, 0.5, 0.74, 0.75, 0.999]])
    assert oracle.sample(amp, 3, [0, 1, 2], u).tolist() == [[0, 0, 2, 3, 3, 5, 5]]
    shots = 200000
    u = np.random.default_rng(7).random((2, shots))
    out = oracle.sample(psi, n, [0, 2, 5], u)
    p = oracle.probs(psi, n, [0, 2, 5])
    for b in range(2):
        freq = np.bincount(out[b], minlength=8) / shots
        assert np.all(np.abs(freq - p[b]) <= 5 * np.sqrt(p[b] * (1 - p[b]) / shots) + 1e-12)


def test_collapse_projects_and_renormalises():
    n = 7
    psi = w.random_state(n, 3, 31)
    locs = [6, 2]
    outcome = [1, 3, 0]
    post, p = oracle.collapse(psi, n, locs, outcome)
    pr = oracle.probs(psi, n, locs)
    np.testing.assert_allclose(p, [pr[b, outcome[b]] for b in range(3)], atol=1e-15)
    np.testing.assert_allclose(np.sum(np.abs(post) ** 2, axis=0), 1.0, atol=1e-14)
    pp = oracle.probs(post, n, locs)
    for b in range(3):
        assert abs(pp[b, outcome[b]] - 1) < 1e-14
        keep = [i for i in range(1 << n) if (((i >> 6) & 1) | (((i >> 2) & 1) << 1)) == outcome[b]]
        np.testing.assert_allclose(post[keep, b], psi[keep, b] / math.sqrt(p[b]), atol=1e-15)


def dense_pauli_sum(H):
    n = H.n
    M = np.zeros((1 << n, 1 << n), complex)
    for c, x, z in zip(H.coef, H.xmask, H.zmask):
        ops = []
        for q in range(n):
            bx, bz = (int(x) >> q) & 1, (int(z) >> q) & 1
            ops.append(PAULI["Y" if bx and bz else ("X" if bx else ("Z" if bz else "I"))])
        M += c * kron_list(ops)
    return M


@pytest.mark.parametrize("n,t", [(4, 0.1), (4, 1.3), (6, 0.7)])
def test_time_evolution_against_expm(n, t):
    """exp(-iHt) psi by the exponential series against scipy's expm of the dense H."""
    rng = np.random.default_rng(n)
    H = w.pauli_sum(n, [(float(rng.normal()), "".join(rng.choice(list("IXYZ"), n))) for _ in range(3 * n)])
    psi = w.random_state(n, 2, 5)
    want = scipy.linalg.expm(-1j * t * dense_pauli_sum(H)) @ psi
    np.testing.assert_allclose(oracle.time_evolve(H, psi, t), want, atol=1e-12)


def test_time_evolution_closed_forms_and_invariants():
    n = 8
    h = np.random.default_rng(1).normal(size=n)
    Hz = w.pauli_sum(n, [(h[q], "I" * q + "Z" + "I" * (n - q - 1)) for q in range(n)])
    psi = w.random_state(n, 1, 3)
    t = 2.1
    phase = np.array([np.exp(-1j * t * sum(h[q] * (1 - 2 * ((i >> q) & 1)) for q in range(n))) for i in range(1 << n)])
    np.testing.assert_allclose(oracle.time_evolve(Hz, psi, t)[:, 0], phase * psi[:, 0], atol=1e-12)
    H = w.heisenberg(n)
    a = oracle.time_evolve(H, psi, 0.4)
    b = oracle.time_evolve(H, oracle.time_evolve(H, psi, 0.25), 0.15)
    np.testing.assert_allclose(a, b, atol=1e-12)
    assert abs(np.linalg.norm(a) - 1) < 1e-12
    assert abs(oracle.expect(H, a)[0][0] - oracle.expect(H, psi)[0][0]) < 1e-11


def test_shift_rule_per_gate_occurrence():
    """Every gate occurrence shifted on its own: with unshared parameters this is the shift rule
    of the oracle; with a parameter shared by several uncontrolled rotations it is the exact
    derivative (finite differences), where shifting the parameter everywhere at once is not."""
    n = 4
    circ = w.hea_circuit(n, 2)
    params = w.angles(8, circ.nparams)
    psi0 = w.random_state(n, 2, 8)
    sg = oracle.shift_grad_gates(w.heisenberg(n), circ, params, psi0)
    ref = oracle.shift_grad(w.heisenberg(n), circ, params, psi0)
    for p in range(circ.nparams):
        np.testing.assert_allclose(sg[:, p], ref[p], atol=1e-13)
    shared = w.Circuit(n, [w.Gate(g.kind, g.locs, g.ctrls, g.cvals, param=(g.param % 5) if g.param >= 0 else -1)
                           for g in circ.gates], 5)
    p5 = w.angles(9, 5)
    sg = oracle.shift_grad_gates(w.heisenberg(n), shared, p5, psi0)
    fd = oracle.fd_grad(w.heisenberg(n), shared, p5, psi0, h=1e-5)
    for p in range(5):
        np.testing.assert_allclose(sg[:, p], fd[p], atol=1e-8)
    naive = oracle.shift_grad(w.heisenberg(n), shared, p5, psi0)
    assert max(abs(naive[p][0] - fd[p][0]) for p in range(5)) > 1e-3


def test_adjoint_at_20_qubits_matches_stored_differences():
    """The 20-qubit differentiation workload: the oracle's adjoint gradient (computed here)
    against central differences and the shift rule of 24 seeded parameters, both taken from
    oracle energies alone (tests/golden/make_golden.py fd20)."""
    gold = read_golden("fd20.txt")
    n, depth = 20, 20
    circ = w.hea_circuit(n, depth)
    e, g, _ = oracle.adjoint(w.heisenberg(n), circ, w.angles(2, circ.nparams), w.zero_state(n))
    idx = [int(k) for k in gold["index"]]
    np.testing.assert_allclose(g[0, idx], gold["shift"], atol=1e-10)
    np.testing.assert_allclose(g[0, idx], gold["fd"], atol=1e-6)
