"""Python face of the FP64 CPU oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of the
benchmark use this; the product path never does. It shares no code with the HIP path and
imports nothing from it; circuits and observables come from the `workloads` module, which
only describes inputs.

Finite differences and the parameter-shift rule (Sec. "Forward Mode", eq. shiftrule) are
written here on top of the oracle's energy; they pin the oracle's adjoint gradient. Time
evolution (Sec. "Matrix Representation": time_evolve) is the exponential series of -iHt applied
through the oracle's H psi.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from workloads import Circuit, Gate, PauliSum

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

MAXK = 6
MAXC = 8
_KIND = {"X": 0, "Y": 1, "Z": 2, "H": 3, "S": 4, "Sdag": 5, "T": 6, "Tdag": 7,
         "Rx": 8, "Ry": 9, "Rz": 10, "shift": 11, "rot": 12, "dense": 13}


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (OpenMP over output indices only)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared", SRC_PATH, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Gate(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int), ("param", ctypes.c_int), ("k", ctypes.c_int), ("nctrl", ctypes.c_int),
        ("locs", ctypes.c_int * MAXK), ("ctrls", ctypes.c_int * MAXC), ("cvals", ctypes.c_int * MAXC),
        ("theta", ctypes.c_double), ("G", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i, l, d = ctypes.c_int, ctypes.c_long, ctypes.c_double
        L.orc_apply_op.argtypes = [i, l, P, P, P, i, P, i, P, P, i]
        L.orc_apply.argtypes = [i, l, P, P, i, P, i, P, P]
        L.orc_forward.argtypes = [i, l, P, i, P, P]
        L.orc_hpsi.argtypes = [i, l, P, P, i, P, P, P]
        L.orc_expect.argtypes = [i, l, P, i, P, P, P, P, P]
        L.orc_energy.argtypes = [i, l, P, i, P, P, i, P, P, P, P]
        L.orc_adjoint.argtypes = [i, l, P, i, P, P, i, i, P, P, P, P, P, P]
        L.orc_gate_matrix.argtypes = [P, d, P]
        L.orc_gate_matrix.restype = l
        L.orc_gate_deriv.argtypes = [P, d, P]
        L.orc_gate_deriv.restype = l
        L.orc_num_threads.restype = i
        L.orc_permute_qubits.argtypes = [i, l, P, P, P]
        L.orc_qft_at.argtypes = [i, l, P, i, P, i, l, P, P]
        L.orc_probs.argtypes = [i, l, P, i, P, P]
        L.orc_sample.argtypes = [i, l, P, i, P, l, P, P]
        L.orc_collapse.argtypes = [i, l, P, i, P, P, P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


class _GateArray:
    """ctypes array of gates; keeps the generator matrices alive."""

    def __init__(self, gates):
        self.keep = []
        self.arr = (_Gate * max(1, len(gates)))()
        for t, g in enumerate(gates):
            s = self.arr[t]
            s.kind = _KIND[g.kind]
            s.param = g.param
            s.k = len(g.locs)
            s.nctrl = len(g.ctrls)
            if s.k > MAXK or s.nctrl > MAXC:
                raise ValueError("gate too wide for the oracle")
            for j, q in enumerate(g.locs):
                s.locs[j] = q
            for j, (c, v) in enumerate(zip(g.ctrls, g.cvals)):
                s.ctrls[j] = c
                s.cvals[j] = v
            s.theta = g.theta
            if g.G is not None:
                G = _c128(g.G)
                self.keep.append(G)
                s.G = G.ctypes.data
            else:
                s.G = None
        self.n = len(gates)

    @property
    def ptr(self):
        return ctypes.cast(self.arr, ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def gate_matrix(g, theta=None) -> np.ndarray:
    ga = _GateArray([g])
    d = 1 << len(g.locs)
    U = np.zeros(d * d, np.complex128)
    th = g.theta if theta is None else theta
    if lib().orc_gate_matrix(ga.ptr, th, _ptr(U)) < 0:
        raise ValueError(g.kind)
    return U.reshape(d, d)


def gate_deriv(g, theta) -> np.ndarray:
    ga = _GateArray([g])
    d = 1 << len(g.locs)
    D = np.zeros(d * d, np.complex128)
    if lib().orc_gate_deriv(ga.ptr, theta, _ptr(D)) < 0:
        raise ValueError(g.kind)
    return D.reshape(d, d)


def _state(psi, n):
    psi = _c128(psi)
    if psi.ndim == 1:
        psi = psi.reshape(-1, 1)
    if psi.shape[0] != (1 << n):
        raise ValueError("state must be [2^n][batch]")
    return np.ascontiguousarray(psi), psi.shape[1]


def apply_matrix(psi, n, U, locs, ctrls=(), cvals=None):
    """Return F psi for matrix U on locs with controls (psi is [2^n] or [2^n][B])."""
    psi, B = _state(psi, n)
    out = psi.copy()
    U = _c128(U)
    cvals = tuple(cvals) if cvals is not None else tuple(1 for _ in ctrls)
    locs_a = np.array(locs, np.int32)
    ctrls_a = np.array(ctrls if ctrls else [0], np.int32)
    cvals_a = np.array(cvals if cvals else [0], np.int32)
    lib().orc_apply(n, B, _ptr(out), _ptr(U), len(locs), _ptr(locs_a), len(ctrls), _ptr(ctrls_a), _ptr(cvals_a))
    return out


def forward(circ: Circuit, params, psi0):
    psi, B = _state(psi0, circ.n)
    out = psi.copy()
    ga = _GateArray(circ.gates)
    p = np.ascontiguousarray(np.asarray(params if params is not None else [0.0], np.float64))
    lib().orc_forward(circ.n, B, _ptr(out), ga.n, ga.ptr, _ptr(p))
    return out


def _ham(H: PauliSum):
    return (np.ascontiguousarray(H.coef, np.float64), np.ascontiguousarray(H.xmask, np.uint64),
            np.ascontiguousarray(H.zmask, np.uint64))


def hpsi(H: PauliSum, psi):
    psi, B = _state(psi, H.n)
    out = np.zeros_like(psi)
    c, x, z = _ham(H)
    lib().orc_hpsi(H.n, B, _ptr(psi), _ptr(out), H.nterms, _ptr(c), _ptr(x), _ptr(z))
    return out


def pauli_apply(n, psi, xmask, zmask):
    return hpsi(PauliSum(n, np.array([1.0]), np.array([xmask], np.uint64), np.array([zmask], np.uint64)), psi)


def expect(H: PauliSum, psi):
    """(Re, Im) of <psi|H|psi> per batch slot."""
    psi, B = _state(psi, H.n)
    re = np.zeros(B)
    im = np.zeros(B)
    c, x, z = _ham(H)
    lib().orc_expect(H.n, B, _ptr(psi), H.nterms, _ptr(c), _ptr(x), _ptr(z), _ptr(re), _ptr(im))
    return re, im


def energy(H: PauliSum, circ: Circuit, params, psi0):
    psi, B = _state(psi0, circ.n)
    ga = _GateArray(circ.gates)
    p = np.ascontiguousarray(np.asarray(params if params is not None and len(params) else [0.0], np.float64))
    e = np.zeros(B)
    c, x, z = _ham(H)
    lib().orc_energy(circ.n, B, _ptr(psi), ga.n, ga.ptr, _ptr(p), H.nterms, _ptr(c), _ptr(x), _ptr(z), _ptr(e))
    return e


def adjoint(H: PauliSum, circ: Circuit, params, psi0):
    """Energy [B], gradient [B][nparams] and the uncomputed input state, by the paper's
    reverse mode with uncomputation."""
    psi, B = _state(psi0, circ.n)
    ga = _GateArray(circ.gates)
    p = np.ascontiguousarray(np.asarray(params if params is not None and len(params) else [0.0], np.float64))
    e = np.zeros(B)
    g = np.zeros((B, max(1, circ.nparams)))
    back = np.zeros_like(psi)
    c, x, z = _ham(H)
    lib().orc_adjoint(circ.n, B, _ptr(psi), ga.n, ga.ptr, _ptr(p), circ.nparams, H.nterms, _ptr(c), _ptr(x),
                      _ptr(z), _ptr(e), _ptr(g), _ptr(back))
    return e, g[:, :circ.nparams], back


def fd_grad(H, circ, params, psi0, h=1e-4, which=None):
    """Central finite differences (E(p+h) - E(p-h)) / 2h, per batch slot."""
    params = np.asarray(params, np.float64)
    idx = range(circ.nparams) if which is None else which
    out = {}
    for k in idx:
        pp = params.copy()
        pp[k] += h
        pm = params.copy()
        pm[k] -= h
        out[k] = (energy(H, circ, pp, psi0) - energy(H, circ, pm, psi0)) / (2 * h)
    return out


def shift_grad(H, circ, params, psi0, which=None):
    """Parameter-shift rule (eq. shiftrule): (E(p + pi/2) - E(p - pi/2)) / 2; exact only for
    rotations whose generator is reflexive and that are not controlled."""
    params = np.asarray(params, np.float64)
    idx = range(circ.nparams) if which is None else which
    out = {}
    for k in idx:
        pp = params.copy()
        pp[k] += math.pi / 2
        pm = params.copy()
        pm[k] -= math.pi / 2
        out[k] = 0.5 * (energy(H, circ, pp, psi0) - energy(H, circ, pm, psi0))
    return out


# --------------------------------------------------------------------------------------------
# focus! / relax! (Sec. "Active qubits and environment qubits")
# --------------------------------------------------------------------------------------------

def permute_qubits(psi, n, perm):
    """The register with qubit q moved to position perm[q]."""
    psi, B = _state(psi, n)
    perm = np.ascontiguousarray(np.asarray(perm, np.int32))
    if sorted(perm.tolist()) != list(range(n)):
        raise ValueError("perm must be a permutation of 0..n-1")
    out = np.empty_like(psi)
    lib().orc_permute_qubits(n, B, _ptr(psi), _ptr(out), _ptr(perm))
    return out


def focus_perm(n, locs):
    """focus!(reg, locs): locs[j] becomes active qubit j; the other qubits follow in order."""
    locs = list(locs)
    rest = [q for q in range(n) if q not in locs]
    perm = [0] * n
    for j, q in enumerate(locs + rest):
        perm[q] = j
    return perm


def focus(psi, n, locs):
    return permute_qubits(psi, n, focus_perm(n, locs))


def relax(psi, n, locs):
    """relax!(reg, locs): the inverse of focus!(reg, locs)."""
    fp = focus_perm(n, locs)
    inv = [0] * n
    for q, j in enumerate(fp):
        inv[j] = q
    return permute_qubits(psi, n, inv)


# --------------------------------------------------------------------------------------------
# QFT on a set of qubits (Listing "QFT circuit"; App. "Extending QBIR: emulating QFT circuit")
# --------------------------------------------------------------------------------------------

def qft(psi, n, locs, inverse=False, idx=None):
    """QFT (or its inverse) on the qubits locs by its matrix definition; idx: the output
    indices to compute (all when None). Returns [len(idx)][B]."""
    psi, B = _state(psi, n)
    locs_a = np.ascontiguousarray(np.asarray(locs, np.int32))
    idx = np.arange(1 << n, dtype=np.int64) if idx is None else np.ascontiguousarray(np.asarray(idx, np.int64))
    out = np.zeros((len(idx), B), np.complex128)
    lib().orc_qft_at(n, B, _ptr(psi), len(locs_a), _ptr(locs_a), int(bool(inverse)), len(idx), _ptr(idx), _ptr(out))
    return out


# --------------------------------------------------------------------------------------------
# measure / measure! (Listing "instruct! and measure")
# --------------------------------------------------------------------------------------------

def probs(psi, n, locs):
    """[B][2^k] probabilities of the outcomes of the qubits locs (locs[j] -> bit j)."""
    psi, B = _state(psi, n)
    locs_a = np.ascontiguousarray(np.asarray(locs, np.int32))
    out = np.zeros((B, 1 << len(locs_a)))
    lib().orc_probs(n, B, _ptr(psi), len(locs_a), _ptr(locs_a), _ptr(out))
    return out


def sample(psi, n, locs, u):
    """Outcomes [B][nshots] for the uniform numbers u [B][nshots] by inverse-CDF sampling."""
    psi, B = _state(psi, n)
    locs_a = np.ascontiguousarray(np.asarray(locs, np.int32))
    u = np.ascontiguousarray(np.asarray(u, np.float64).reshape(B, -1))
    out = np.zeros(u.shape, np.int64)
    lib().orc_sample(n, B, _ptr(psi), len(locs_a), _ptr(locs_a), u.shape[1], _ptr(u), _ptr(out))
    return out


def collapse(psi, n, locs, outcome):
    """measure! after the outcome is known: (projected and renormalised state, p[B])."""
    psi, B = _state(psi, n)
    psi = psi.copy()
    locs_a = np.ascontiguousarray(np.asarray(locs, np.int32))
    oc = np.ascontiguousarray(np.asarray(outcome, np.int64).reshape(B))
    p = np.zeros(B)
    lib().orc_collapse(n, B, _ptr(psi), len(locs_a), _ptr(locs_a), _ptr(oc), _ptr(p))
    return psi, p


# --------------------------------------------------------------------------------------------
# Time evolution exp(-iHt) psi (Sec. "Matrix Representation", time_evolve)
# --------------------------------------------------------------------------------------------

def time_evolve(H: PauliSum, psi, t):
    """exp(-i H t) psi by the exponential series: t is cut into m equal steps with
    |dt| * sum_t |c_t| <= 1/2 (sum |c_t| bounds the spectral norm of H), and each step sums
    (-i H dt)^j psi / j! until the term falls below 1e-18 of the partial sum."""
    psi, B = _state(psi, H.n)
    bound = float(np.abs(np.asarray(H.coef, np.float64)).sum())
    m = max(1, int(math.ceil(abs(t) * bound / 0.5)))
    dt = t / m
    v = psi.copy()
    for _ in range(m):
        term = v.copy()
        acc = v.copy()
        for j in range(1, 200):
            term = (-1j * dt / j) * hpsi(H, term)
            acc += term
            if np.abs(term).max() <= 1e-18 * max(1e-300, np.abs(acc).max()):
                break
        v = acc
    return v


# --------------------------------------------------------------------------------------------
# Faithful gradient of every gate occurrence (Sec. "Forward Mode", eq. shiftrule)
# --------------------------------------------------------------------------------------------

def shift_grad_gates(H, circ, params, psi0):
    """grad[B][nparams]: for every parametrised gate occurrence k with parameter p,
    (E(angle of gate k + pi/2) - E(angle of gate k - pi/2)) / 2 is added to grad[p] (only that
    occurrence shifted, so a shared parameter gets the sum over its gates)."""
    params = np.asarray(params, np.float64)
    psi, B = _state(psi0, circ.n)
    P = circ.nparams
    grad = np.zeros((B, P))
    for k, g in enumerate(circ.gates):
        if g.param < 0:
            continue
        gates = list(circ.gates)
        gates[k] = Gate(g.kind, g.locs, ctrls=g.ctrls, cvals=g.cvals, param=P, theta=g.theta, G=g.G)
        c2 = Circuit(circ.n, gates, P + 1)
        ep = energy(H, c2, np.append(params, params[g.param] + math.pi / 2), psi)
        em = energy(H, c2, np.append(params, params[g.param] - math.pi / 2), psi)
        grad[:, g.param] += 0.5 * (ep - em)
    return grad
