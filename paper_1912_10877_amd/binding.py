"""ctypes binding of libyao.so (include/yao.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts Python objects to
the C ABI's plain pointers and sizes, raises on error codes, and lets torch own device
memory (states can wrap torch tensors) and pick the stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libyao.so")

C64, C128 = 0, 1
GRAD_REVERSIBLE, GRAD_CHECKPOINT, GRAD_AUTO = 0, 1, 2
GATE_CODES = {"X": 0, "Y": 1, "Z": 2, "H": 3, "S": 4, "Sdag": 5, "T": 6, "Tdag": 7,
              "Rx": 8, "Ry": 9, "Rz": 10, "shift": 11, "rot": 12, "dense": 13}
STATUS = {-1: "YAO_EINVAL", -2: "YAO_ENOMEM", -3: "YAO_EHIP", -4: "YAO_EDRIFT", -5: "YAO_ENODEV"}


class YaoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("plain", ctypes.c_int), ("tile_qubits", ctypes.c_int), ("fuse_width", ctypes.c_int),
                ("checkpoint_every", ctypes.c_int), ("drift_tol", ctypes.c_double), ("mfma", ctypes.c_int),
                ("autotune", ctypes.c_int), ("jit", ctypes.c_int)]


_lib = None
P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double
PP = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "yao_init": [],
    "yao_set_stream": [P],
    "yao_synchronize": [],
    "yao_set_options": [P],
    "yao_get_options": [P],
    "yao_state_create": [I, I, I, PP],
    "yao_state_wrap": [P, I, I, I, PP],
    "yao_state_destroy": [P],
    "yao_state_reset": [P],
    "yao_state_upload": [P, P, ctypes.c_size_t],
    "yao_state_download": [P, P, ctypes.c_size_t],
    "yao_state_info": [P, PP, P, P, P],
    "yao_apply": [P, P, I, P, I, P, P],
    "yao_apply_gate": [P, I, D, P, P, I, I, P, P],
    "yao_pauli_sum_create": [I, I, P, P, P, PP],
    "yao_pauli_sum_destroy": [P],
    "yao_expect": [P, P, P],
    "yao_expect_noalloc": [P, P, P],
    "yao_hpsi": [P, P, P, P],
    "yao_inner": [P, P, P, P],
    "yao_circuit_create": [I, PP],
    "yao_circuit_destroy": [P],
    "yao_circuit_push": [P, I, I, D, P, P, I, I, P, P],
    "yao_circuit_nparams": [P, P],
    "yao_forward": [P, P, P],
    "yao_backward": [P, P, P, P, I, I, P, P, P],
    "yao_batch_run": [I, P, P, P, P, P, P],
    "yao_auto_fallbacks": [P],
    "yao_permute_qubits": [P, P, P],
    "yao_focus": [P, P, I],
    "yao_relax": [P, P, I],
    "yao_qft": [P, P, I, I],
    "yao_probs": [P, P, I, P],
    "yao_time_evolve": [P, P, D, D, I, P],
    "yao_shift_grad": [P, P, P, P, P, P],
    "yao_measure": [P, P, I, I, P, P],
    "yao_measure_collapse": [P, P, I, P, P, P],
    "yao_profile_enable": [I],
    "yao_profile_read": [I, P, P, P, P],
    "yao_plan_selfcheck": [P, P, I, I, I, P, P],
    "yao_jit_selfcheck": [P, I, I, I, P, P],
    "yao_jit_stats": [P],
}


def lib():
    """Load libyao.so; raises if it was not built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.yao_last_error.argtypes = []
        L.yao_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise YaoError(code, lib().yao_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(seq):
    return np.ascontiguousarray(np.asarray(list(seq) if seq is not None else [], np.int32))


def _c128_flat(m):
    m = np.ascontiguousarray(np.asarray(m, np.complex128))
    return m.view(np.float64).reshape(-1).copy()


def init():
    _check(lib().yao_init())


def set_stream(stream_ptr: int | None):
    _check(lib().yao_set_stream(stream_ptr))


def use_torch_stream():
    import torch
    set_stream(torch.cuda.current_stream().cuda_stream)


def synchronize():
    _check(lib().yao_synchronize())


def get_options() -> Options:
    o = Options()
    _check(lib().yao_get_options(ctypes.byref(o)))
    return o


def set_options(**kw):
    o = get_options()
    for k, v in kw.items():
        setattr(o, k, v)
    _check(lib().yao_set_options(ctypes.byref(o)))
    return o


class State:
    """A register of n qubits and batch B (layout [2^n][B], batch innermost).

    With `tensor` given (a torch complex64/complex128 CUDA tensor of 2^n * B elements) the
    state wraps torch-owned memory; otherwise the library allocates |0...0>.
    """

    def __init__(self, n: int, batch: int = 1, dtype: int = C64, tensor=None):
        self.n, self.batch, self.dtype = n, batch, dtype
        self.tensor = tensor
        h = ctypes.c_void_p()
        if tensor is not None:
            if not tensor.is_contiguous() or tensor.numel() != (1 << n) * batch:
                raise ValueError("tensor must be contiguous with 2^n * batch elements")
            _check(lib().yao_state_wrap(tensor.data_ptr(), n, batch, dtype, ctypes.byref(h)))
        else:
            _check(lib().yao_state_create(n, batch, dtype, ctypes.byref(h)))
        self.h = h

    @property
    def np_dtype(self):
        return np.complex64 if self.dtype == C64 else np.complex128

    def destroy(self):
        if self.h:
            _check(lib().yao_state_destroy(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self.h and _lib is not None:
                _lib.yao_state_destroy(self.h)
        except Exception:
            pass

    def reset(self):
        _check(lib().yao_state_reset(self.h))

    def upload(self, arr):
        a = np.ascontiguousarray(np.asarray(arr, self.np_dtype).reshape(1 << self.n, self.batch))
        _check(lib().yao_state_upload(self.h, _ptr(a), a.nbytes))

    def download(self) -> np.ndarray:
        a = np.empty((1 << self.n, self.batch), self.np_dtype)
        _check(lib().yao_state_download(self.h, _ptr(a), a.nbytes))
        return a

    def device_ptr(self) -> int:
        p = ctypes.c_void_p()
        _check(lib().yao_state_info(self.h, ctypes.byref(p), None, None, None))
        return p.value

    def apply(self, U, locs, ctrls=(), cvals=None):
        U = _c128_flat(U)
        locs, ctrls = _i32(locs), _i32(ctrls)
        cv = None if cvals is None else _i32(cvals)
        _check(lib().yao_apply(self.h, _ptr(U), len(locs), _ptr(locs), len(ctrls), _ptr(ctrls), _ptr(cv)))

    def apply_gate(self, kind: str, locs, theta=0.0, G=None, ctrls=(), cvals=None):
        Gf = None if G is None else _c128_flat(G)
        locs, ctrls = _i32(locs), _i32(ctrls)
        cv = None if cvals is None else _i32(cvals)
        _check(lib().yao_apply_gate(self.h, GATE_CODES[kind], float(theta), _ptr(Gf), _ptr(locs), len(locs),
                                    len(ctrls), _ptr(ctrls), _ptr(cv)))


class PauliSum:
    def __init__(self, n, coef, xmask, zmask):
        self.n = n
        self._c = np.ascontiguousarray(np.asarray(coef, np.float64))
        self._x = np.ascontiguousarray(np.asarray(xmask, np.uint64))
        self._z = np.ascontiguousarray(np.asarray(zmask, np.uint64))
        h = ctypes.c_void_p()
        _check(lib().yao_pauli_sum_create(n, len(self._c), _ptr(self._c), _ptr(self._x), _ptr(self._z), ctypes.byref(h)))
        self.h = h

    @classmethod
    def from_workload(cls, ps):
        return cls(ps.n, ps.coef, ps.xmask, ps.zmask)

    def __del__(self):
        try:
            if self.h and _lib is not None:
                _lib.yao_pauli_sum_destroy(self.h)
        except Exception:
            pass


class Circuit:
    def __init__(self, n: int):
        self.n = n
        h = ctypes.c_void_p()
        _check(lib().yao_circuit_create(n, ctypes.byref(h)))
        self.h = h

    def push(self, kind: str, locs, param=-1, theta=0.0, G=None, ctrls=(), cvals=None):
        Gf = None if G is None else _c128_flat(G)
        locs, ctrls = _i32(locs), _i32(ctrls)
        cv = None if cvals is None else _i32(cvals)
        _check(lib().yao_circuit_push(self.h, GATE_CODES[kind], int(param), float(theta), _ptr(Gf), _ptr(locs),
                                      len(locs), len(ctrls), _ptr(ctrls), _ptr(cv)))

    @classmethod
    def from_workload(cls, circ):
        c = cls(circ.n)
        for g in circ.gates:
            c.push(g.kind, g.locs, g.param, g.theta, g.G, g.ctrls, g.cvals)
        return c

    @property
    def nparams(self) -> int:
        v = ctypes.c_int()
        _check(lib().yao_circuit_nparams(self.h, ctypes.byref(v)))
        return v.value

    def __del__(self):
        try:
            if self.h and _lib is not None:
                _lib.yao_circuit_destroy(self.h)
        except Exception:
            pass


def _params(p):
    return np.ascontiguousarray(np.asarray(p if p is not None and len(p) else [0.0], np.float64))


def expect(state: State, H: PauliSum) -> np.ndarray:
    e = np.zeros(state.batch)
    _check(lib().yao_expect(state.h, H.h, _ptr(e)))
    return e


def expect_noalloc(state: State, H: PauliSum) -> np.ndarray:
    """yao_expect_noalloc: the expectation with every device buffer in the library's static array."""
    e = np.zeros(state.batch)
    _check(lib().yao_expect_noalloc(state.h, H.h, _ptr(e)))
    return e


def hpsi(state: State, H: PauliSum, out: State, with_energy=True):
    e = np.zeros(state.batch) if with_energy else None
    _check(lib().yao_hpsi(state.h, H.h, out.h, _ptr(e)))
    return e


def inner(a: State, b: State) -> np.ndarray:
    """<a_b|b_b> per batch slot (complex128 numpy array)."""
    re = np.zeros(a.batch)
    im = np.zeros(a.batch)
    _check(lib().yao_inner(a.h, b.h, _ptr(re), _ptr(im)))
    return re + 1j * im


def forward(state: State, circ: Circuit, params):
    p = _params(params)
    _check(lib().yao_forward(state.h, circ.h, _ptr(p)))


def backward(state: State, circ: Circuit, params, H: PauliSum, mode=GRAD_REVERSIBLE, reduce_batch=False):
    """Returns (energy[B], grad[B][P] or grad[P], drift)."""
    p = _params(params)
    P_ = circ.nparams
    e = np.zeros(state.batch)
    g = np.zeros(max(1, P_) if reduce_batch else max(1, P_) * state.batch)
    drift = ctypes.c_double()
    _check(lib().yao_backward(state.h, circ.h, _ptr(p), H.h, mode, int(reduce_batch), _ptr(e), _ptr(g),
                              ctypes.byref(drift)))
    if reduce_batch:
        return e, g[:P_], drift.value
    return e, g[:P_ * state.batch].reshape(state.batch, P_) if P_ else np.zeros((state.batch, 0)), drift.value


def permute_qubits(src: State, dst: State, perm):
    """dst = src with qubit q moved to index bit perm[q] (dst may be src)."""
    p = _i32(perm)
    _check(lib().yao_permute_qubits(src.h, dst.h, _ptr(p)))


def focus(state: State, locs):
    """focus!: qubit locs[j] becomes qubit j, the others follow in ascending order."""
    l = _i32(locs)
    _check(lib().yao_focus(state.h, _ptr(l), len(l)))


def relax(state: State, locs):
    """relax!: undoes focus(state, locs)."""
    l = _i32(locs)
    _check(lib().yao_relax(state.h, _ptr(l), len(l)))


def qft(state: State, locs, inverse=False):
    """QFT (or its inverse) on the qubits locs, in place."""
    l = _i32(locs)
    _check(lib().yao_qft(state.h, _ptr(l), len(l), int(bool(inverse))))


def shift_grad(state: State, circ: Circuit, params, H: PauliSum):
    """(energy, grad[P]) by the shift rule over every gate occurrence, one batched register."""
    p = _params(params)
    e = np.zeros(1)
    g = np.zeros(max(1, circ.nparams))
    _check(lib().yao_shift_grad(state.h, circ.h, _ptr(p), H.h, _ptr(e), _ptr(g)))
    return e[0], g[:circ.nparams]


def time_evolve(state: State, H: PauliSum, t: float, tol: float = 0.0, krylov_dim: int = 0) -> int:
    """psi <- exp(-i H t) psi in place; returns the number of Krylov substeps."""
    steps = ctypes.c_int()
    _check(lib().yao_time_evolve(state.h, H.h, float(t), float(tol), int(krylov_dim), ctypes.byref(steps)))
    return steps.value


def probs(state: State, locs) -> np.ndarray:
    """[B][2^k] probabilities of the outcomes of the qubits locs."""
    l = _i32(locs)
    out = np.zeros((state.batch, 1 << len(l)))
    _check(lib().yao_probs(state.h, _ptr(l), len(l), _ptr(out)))
    return out


def measure(state: State, locs, u) -> np.ndarray:
    """Outcomes [B][nshots] for the caller's uniform numbers u [B][nshots] in [0, 1)."""
    l = _i32(locs)
    u = np.ascontiguousarray(np.asarray(u, np.float64).reshape(state.batch, -1))
    out = np.zeros(u.shape, np.uint64)
    _check(lib().yao_measure(state.h, _ptr(l), len(l), u.shape[1], _ptr(u), _ptr(out)))
    return out.astype(np.int64)


def measure_collapse(state: State, locs, u):
    """measure!: (outcome[B], probability[B]) from one uniform number per slot; the state
    collapses."""
    l = _i32(locs)
    u = np.ascontiguousarray(np.asarray(u, np.float64).reshape(state.batch))
    out = np.zeros(state.batch, np.uint64)
    p = np.zeros(state.batch)
    _check(lib().yao_measure_collapse(state.h, _ptr(l), len(l), _ptr(u), _ptr(out), _ptr(p)))
    return out.astype(np.int64), p


def auto_fallbacks() -> int:
    """AUTO backward calls that fell back to the checkpointed sweep since the library loaded."""
    v = ctypes.c_long()
    _check(lib().yao_auto_fallbacks(ctypes.byref(v)))
    return v.value


def batch_run(states: Sequence[State], circs: Sequence[Circuit], params: Sequence[np.ndarray],
              hams: Sequence[PauliSum]):
    """Energy and gradient of independent circuits in one replay of the graph recorded for this
    list (recorded on its first call)."""
    m = len(states)
    ps = [_params(p) for p in params]
    grads = [np.zeros(max(1, c.nparams)) for c in circs]
    e = np.zeros(m)
    arr = lambda objs: (ctypes.c_void_p * m)(*[o.h.value for o in objs])
    parr = (ctypes.c_void_p * m)(*[p.ctypes.data for p in ps])
    garr = (ctypes.c_void_p * m)(*[g.ctypes.data for g in grads])
    _check(lib().yao_batch_run(m, arr(states), arr(circs), parr, arr(hams), _ptr(e), garr))
    return e, [g[:c.nparams] for g, c in zip(grads, circs)]


def header_symbols(path=None):
    """Names of the functions declared in include/yao.h."""
    import re
    path = path or os.path.join(HERE, "..", "include", "yao.h")
    src = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(yao_\w+)\s*\(", src, re.M)))


def plan_selfcheck(circ: Circuit, params, dtype=0, reverse=False, tile_qubits=0):
    """Host run of the circuit's pass plan (qubit layouts, permuted stores, records on tile bits)
    against gate-by-gate application: returns (max amplitude error, number of passes)."""
    p = _params(params)
    err, npass = ctypes.c_double(), ctypes.c_int()
    _check(lib().yao_plan_selfcheck(circ.h, _ptr(p), int(dtype), int(bool(reverse)), int(tile_qubits),
                                    ctypes.byref(err), ctypes.byref(npass)))
    return err.value, npass.value


def jit_selfcheck(circ: Circuit, dtype=0, reverse=False, tile_qubits=0):
    """Generate and compile (hipRTC, host only) the run-time forward (or reverse-sweep) passes of
    the circuit as a device-bound program: returns (number of passes, number compiled)."""
    npass, njit = ctypes.c_int(), ctypes.c_int()
    _check(lib().yao_jit_selfcheck(circ.h, int(dtype), int(bool(reverse)), int(tile_qubits), ctypes.byref(npass),
                                   ctypes.byref(njit)))
    return npass.value, njit.value


def jit_stats():
    """Since the library loaded: dict of programs and passes compiled, failed programs, and
    launches of compiled forward and reverse passes."""
    out = (ctypes.c_longlong * 5)()
    _check(lib().yao_jit_stats(out))
    return {"programs": out[0], "passes": out[1], "failures": out[2], "fwd_launches": out[3], "bwd_launches": out[4]}
