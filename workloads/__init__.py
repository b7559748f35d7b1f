"""Seeded synthetic inputs for the state-vector method (circuits, observables, angles).

This module is the only code that the oracle side and the HIP side both use. It describes
*what* to compute -- which gate sits on which qubits with which parameter, which Pauli
strings make up an observable, which random numbers were drawn -- and holds none of the
method's arithmetic: no state update, no expectation, no gate matrix of a named gate
(each side builds those from its own definitions). Random numbers that the method needs
(angles, Haar-random SU(2) entries, pairings) are drawn here and passed to both sides.

Conventions (Yao paper, Sec. "Instructions on Quantum Registers"): qubits are 0-based
here (the paper counts from 1) and qubit q is bit q of the amplitude index. Parameters
are numbered in the order the gates are listed, which is the depth-first order of the
paper's `parameters` (Sec. "Reverse Mode").
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Gate kinds. Each side maps these names onto its own gate definitions.
FIXED_KINDS = ("X", "Y", "Z", "H", "S", "Sdag", "T", "Tdag")
PARAM_KINDS = ("Rx", "Ry", "Rz", "shift", "rot")
MATRIX_KINDS = ("dense",)
ALL_KINDS = FIXED_KINDS + PARAM_KINDS + MATRIX_KINDS


@dataclasses.dataclass(frozen=True)
class Gate:
    """One instruction: `kind` on `locs`, active when every ctrls[m] reads cvals[m].

    `param` >= 0 selects the circuit parameter that gives the angle; otherwise `theta`
    is the fixed angle. `G` is the generator of a "rot" gate (Hermitian, G^2 = 1) or the
    matrix of a "dense" gate, 2^k x 2^k, row index r = sum_j bit(locs[j]) << j.
    """

    kind: str
    locs: Tuple[int, ...]
    ctrls: Tuple[int, ...] = ()
    cvals: Tuple[int, ...] = ()
    param: int = -1
    theta: float = 0.0
    G: Optional[np.ndarray] = None

    def __post_init__(self):
        if self.kind not in ALL_KINDS:
            raise ValueError(f"unknown gate kind {self.kind!r}")
        if len(self.cvals) != len(self.ctrls):
            object.__setattr__(self, "cvals", tuple(1 for _ in self.ctrls))


@dataclasses.dataclass
class Circuit:
    n: int
    gates: List[Gate]
    nparams: int

    def gate_counts(self):
        out = {}
        for g in self.gates:
            key = (g.kind, len(g.ctrls))
            out[key] = out.get(key, 0) + 1
        return out


@dataclasses.dataclass
class PauliSum:
    """H = sum_t coef[t] * P_t; P_t has X on bits of x only, Z on bits of z only, Y on both."""

    n: int
    coef: np.ndarray  # float64 [T]
    xmask: np.ndarray  # uint64 [T]
    zmask: np.ndarray  # uint64 [T]

    @property
    def nterms(self):
        return len(self.coef)


def pauli_sum(n: int, terms: Sequence[Tuple[float, str]]) -> PauliSum:
    """Build a PauliSum from (coef, string) pairs; string[q] is the Pauli letter on qubit q."""
    coef, xs, zs = [], [], []
    for c, s in terms:
        if len(s) != n:
            raise ValueError("Pauli string length must equal n")
        x = z = 0
        for q, ch in enumerate(s):
            if ch in "XY":
                x |= 1 << q
            if ch in "ZY":
                z |= 1 << q
            if ch not in "IXYZ":
                raise ValueError(ch)
        coef.append(float(c))
        xs.append(x)
        zs.append(z)
    return PauliSum(n, np.array(coef, np.float64), np.array(xs, np.uint64), np.array(zs, np.uint64))


def heisenberg(n: int, periodic: bool = True) -> PauliSum:
    """sum over bonds (i, i+1) of X_iX_{i+1} + Y_iY_{i+1} + Z_iZ_{i+1}, coupling +1.

    The Listing "Heisenberg Hamiltonian" builds the open chain; the appendix example
    (App. "Symbolic Differentiation") is reproduced only by the periodic one, which the
    workloads use. Terms are ordered bond by bond, X then Y then Z.
    """
    nb = n if periodic else n - 1
    coef, xs, zs = [], [], []
    for i in range(nb):
        j = (i + 1) % n
        m = (1 << i) | (1 << j)
        for sig in "XYZ":
            coef.append(1.0)
            xs.append(m if sig in "XY" else 0)
            zs.append(m if sig in "YZ" else 0)
    return PauliSum(n, np.array(coef, np.float64), np.array(xs, np.uint64), np.array(zs, np.uint64))


def hea_circuit(n: int, depth: int, periodic: bool = False) -> Circuit:
    """Hardware-efficient ansatz of the workloads: per layer Rx.Rz.Rx on every qubit
    (applied Rx, then Rz, then Rx), then CNOT(i -> i+1) for i = 0..n-2 in ascending order
    (periodic=True adds n-1 -> 0). Parameter (l*n + q)*3 + j is gate j of qubit q in layer l.
    """
    gates = []
    for l in range(depth):
        for q in range(n):
            base = (l * n + q) * 3
            gates.append(Gate("Rx", (q,), param=base + 0))
            gates.append(Gate("Rz", (q,), param=base + 1))
            gates.append(Gate("Rx", (q,), param=base + 2))
        last = n if periodic else n - 1
        for i in range(last):
            gates.append(Gate("X", ((i + 1) % n,), ctrls=(i,), cvals=(1,)))
    return Circuit(n, gates, 3 * n * depth)


def paper_variational_circuit(n: int, depth: int) -> Circuit:
    """The paper's own ansatz shape (Listing "10000-layer VQE" gate counts): a first rotor
    layer Rx.Rz, depth-1 middle layers Rz.Rx.Rz, a last layer Rz.Rx, with a periodic CNOT
    chain after every rotor layer but the last. Gives 2nd Rz, n(d+1) Rx, nd CNOT and
    3nd + n parameters. The exact gate order inside a layer is an inference from those
    counts; it is only used for structure checks.
    """
    gates, p = [], 0
    for l in range(depth + 1):
        for q in range(n):
            if l == 0:
                kinds = ("Rx", "Rz")
            elif l == depth:
                kinds = ("Rz", "Rx")
            else:
                kinds = ("Rz", "Rx", "Rz")
            for kd in kinds:
                gates.append(Gate(kd, (q,), param=p))
                p += 1
        if l < depth:
            for i in range(n):
                gates.append(Gate("X", ((i + 1) % n,), ctrls=(i,), cvals=(1,)))
    return Circuit(n, gates, p)


def qft_circuit(n: int) -> Circuit:
    """QFT as in Listing "quantum Fourier transform": for each qubit i, H on i, then for
    j > i a shift(2*pi / 2^(j-i+1)) on i controlled by j."""
    gates = []
    for i in range(n):
        gates.append(Gate("H", (i,)))
        for j in range(i + 1, n):
            gates.append(Gate("shift", (i,), ctrls=(j,), cvals=(1,), theta=2 * math.pi / 2 ** (j - i + 1)))
    return Circuit(n, gates, 0)


def ghz_circuit(n: int) -> Circuit:
    gates = [Gate("H", (0,))]
    for i in range(n - 1):
        gates.append(Gate("X", (i + 1,), ctrls=(i,), cvals=(1,)))
    return Circuit(n, gates, 0)


def angles(seed: int, nparams: int) -> np.ndarray:
    """Angles uniform in [0, 2*pi) from numpy's default generator with this seed."""
    return np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, nparams)


def haar_su2(rng: np.random.Generator) -> np.ndarray:
    """[[a, -conj(b)], [b, conj(a)]] with (Re a, Im a, Re b, Im b) a normalised Gaussian
    4-vector, i.e. uniform on the 3-sphere, which is Haar measure on SU(2)."""
    v = rng.standard_normal(4)
    v = v / np.sqrt(np.sum(v * v))
    a = complex(v[0], v[1])
    b = complex(v[2], v[3])
    return np.array([[a, -b.conjugate()], [b, a.conjugate()]], np.complex128)


def random_circuit(n: int, depth: int, seed: int) -> Circuit:
    """Precision workload: per layer a Haar-random SU(2) on every qubit, then CZ on the
    pairs (pi[2m], pi[2m+1]) of a fresh seeded random permutation pi of the qubits."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(depth):
        for q in range(n):
            gates.append(Gate("dense", (q,), G=haar_su2(rng)))
        perm = rng.permutation(n)
        for m in range(n // 2):
            a, b = int(perm[2 * m]), int(perm[2 * m + 1])
            gates.append(Gate("Z", (b,), ctrls=(a,), cvals=(1,)))
    return Circuit(n, gates, 0)


def random_gate_list(n: int, ngates: int, seed: int, kmax: int = 3, max_ctrl: int = 2,
                     with_params: bool = True) -> Circuit:
    """Property-test workload: random kinds, locations, controls and control values."""
    rng = np.random.default_rng(seed)
    gates, p = [], 0
    kinds = list(FIXED_KINDS) + (list(PARAM_KINDS) if with_params else []) + ["dense"]
    for _ in range(ngates):
        kind = kinds[rng.integers(len(kinds))]
        k = 1
        if kind in ("dense", "rot"):
            k = int(rng.integers(1, min(kmax, n) + 1))
        qubits = rng.permutation(n)
        locs = tuple(int(x) for x in qubits[:k])
        nc = int(rng.integers(0, min(max_ctrl, n - k) + 1))
        ctrls = tuple(int(x) for x in qubits[k:k + nc])
        cvals = tuple(int(x) for x in rng.integers(0, 2, nc))
        G = None
        if kind == "dense":
            G = random_unitary(2 ** k, rng)
        elif kind == "rot":
            G = random_pauli_matrix(k, rng)
        if kind in PARAM_KINDS:
            gates.append(Gate(kind, locs, ctrls, cvals, param=p, G=G))
            p += 1
        else:
            gates.append(Gate(kind, locs, ctrls, cvals, theta=0.0, G=G))
    return Circuit(n, gates, p)


def random_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random d x d unitary from the QR decomposition of a complex Gaussian matrix,
    with the phases of R's diagonal moved into Q."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return (q * ph).astype(np.complex128)


_PAULI_LETTERS = {
    "I": np.eye(2, dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], np.complex128),
    "Z": np.array([[1, 0], [0, -1]], np.complex128),
}


def pauli_string_matrix(s: str) -> np.ndarray:
    """Dense matrix of a Pauli string used as a rot generator; s[j] acts on locs[j],
    i.e. on bit j of the matrix index (so s[0] is the rightmost Kronecker factor)."""
    m = np.ones((1, 1), np.complex128)
    for ch in s:
        m = np.kron(_PAULI_LETTERS[ch], m)
    return m


def random_pauli_matrix(k: int, rng: np.random.Generator) -> np.ndarray:
    while True:
        s = "".join("IXYZ"[int(i)] for i in rng.integers(0, 4, k))
        if s != "I" * k:
            return pauli_string_matrix(s)


def symad_example():
    """The 3-qubit circuit of App. "Symbolic Differentiation" (paper qubits 1..3 -> 0..2):
    put(2=>Rx(a)), control(2, 1=>Ry(b)), put((1,2)=>rot(kron(X,X), c)); a,b,c = params 0,1,2."""
    gates = [
        Gate("Rx", (1,), param=0),
        Gate("Ry", (0,), ctrls=(1,), cvals=(1,), param=1),
        Gate("rot", (0, 1), param=2, G=pauli_string_matrix("XX")),
    ]
    return Circuit(3, gates, 3)


def hetero_batch_spec(ncirc: int = 1024, seed: int = 4, nmin: int = 8, nmax: int = 20,
                      dmin: int = 4, dmax: int = 16):
    """Sizes of the uneven batch: qubits uniform in nmin..nmax, depth uniform in dmin..dmax;
    circuit c takes its angles from seed 1000 + c."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, ncirc)
    ds = rng.integers(dmin, dmax + 1, ncirc)
    return [(int(n), int(d), 1000 + c) for c, (n, d) in enumerate(zip(ns, ds))]


def random_state(n: int, batch: int, seed: int) -> np.ndarray:
    """Normalised complex Gaussian states, layout [2^n][batch] (batch innermost)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((1 << n, batch)) + 1j * rng.standard_normal((1 << n, batch))
    z /= np.sqrt(np.sum(np.abs(z) ** 2, axis=0, keepdims=True))
    return np.ascontiguousarray(z.astype(np.complex128))


def zero_state(n: int, batch: int = 1) -> np.ndarray:
    z = np.zeros((1 << n, batch), np.complex128)
    z[0, :] = 1.0
    return z
