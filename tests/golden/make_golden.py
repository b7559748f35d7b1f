"""Write the stored oracle results that the full-size GPU parity tests compare against.

Only the FP64 oracle (oracle/) computes these values; nothing here touches the GPU path.
Run:  python tests/golden/make_golden.py [vqe20] [fwd25] [rand20] [c4] [b64] [fd20]

  vqe20   20-qubit Rx.Rz.Rx + CNOT-chain ansatz, depth 20, angles seed 2, |0..0>, periodic
          Heisenberg: energy and all 1200 adjoint gradients (the differentiation workload).
  fwd25   25-qubit same ansatz, depth 20, angles seed 1: energy after the forward sweep.
  rand20  20-qubit random circuit (Haar SU(2) layers + CZ pairings), depth 24, seed 5:
          <Z0 Z1> and <X0> of the output (the precision workload's oracle cross-check).
  c4      the uneven batch (1024 circuits, qubits 8..20, depth 4..16, angles seed 1000 + c):
          energy and every adjoint gradient of each circuit with n <= 16 and of 8 circuits per
          n in 17..20 (seeded choice), stored in c4_batch.npz.
  b64     20-qubit ansatz, depth 20, angles seed 2, on 4 seeded random input states: energy and
          the 1200 gradients of each (b64_states.txt); the 64-slot batch test places these
          states on its slots in a seeded pattern.
  fd20    20-qubit ansatz, depth 20, angles seed 2, |0..0>: central differences (h = 1e-4) and
          the shift rule (eq. shiftrule) of the energy for 24 seeded parameters (fd20.txt),
          computed from oracle energies only.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as w  # noqa: E402


def write(name, header, rows):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        for h in header:
            f.write(f"# {h}\n")
        for key, vals in rows:
            f.write(key + " " + " ".join(repr(float(v)) for v in vals) + "\n")
    print("wrote", path)


def vqe20():
    n, depth = 20, 20
    circ = w.hea_circuit(n, depth)
    params = w.angles(2, circ.nparams)
    t0 = time.time()
    e, g, back = oracle.adjoint(w.heisenberg(n), circ, params, w.zero_state(n))
    write("vqe20_adjoint.txt",
          ["FP64 oracle: 20 qubits, Rx.Rz.Rx + open CNOT chain, depth 20, angles "
           "numpy default_rng(2).uniform(0, 2pi, 1200), input |0..0>, periodic Heisenberg",
           f"written by tests/golden/make_golden.py vqe20 ({time.time() - t0:.1f} s, "
           f"{oracle.num_threads()} threads); uncompute error {np.abs(back - w.zero_state(n)).max():.2e}"],
          [("energy", e), ("grad", g[0])])


def fwd25():
    n, depth = 25, 20
    circ = w.hea_circuit(n, depth)
    params = w.angles(1, circ.nparams)
    t0 = time.time()
    e = oracle.energy(w.heisenberg(n), circ, params, w.zero_state(n))
    write("fwd25_energy.txt",
          ["FP64 oracle: 25 qubits, Rx.Rz.Rx + open CNOT chain, depth 20, angles "
           "numpy default_rng(1).uniform(0, 2pi, 1500), input |0..0>, periodic Heisenberg",
           f"written by tests/golden/make_golden.py fwd25 ({time.time() - t0:.1f} s, "
           f"{oracle.num_threads()} threads)"],
          [("energy", e)])


def rand20():
    n, depth = 20, 24
    circ = w.random_circuit(n, depth, seed=5)
    psi = oracle.forward(circ, None, w.zero_state(n))
    zz = w.pauli_sum(n, [(1.0, "ZZ" + "I" * (n - 2))])
    x0 = w.pauli_sum(n, [(1.0, "X" + "I" * (n - 1))])
    write("rand20_observables.txt",
          ["FP64 oracle: 20 qubits, 24 layers of Haar SU(2) on every qubit + CZ on a random "
           "pairing (workloads.random_circuit seed 5), input |0..0>",
           "written by tests/golden/make_golden.py rand20"],
          [("zz01", oracle.expect(zz, psi)[0]), ("x0", oracle.expect(x0, psi)[0]),
           ("amp0", [psi[0, 0].real, psi[0, 0].imag]), ("amp_last", [psi[-1, 0].real, psi[-1, 0].imag])])


def c4_selection(spec):
    """Indices of the uneven batch that the stored values cover."""
    ns = np.array([n for n, _, _ in spec])
    rng = np.random.default_rng(44)
    pick = [i for i in range(len(spec)) if ns[i] <= 16]
    for n in range(17, 21):
        pick += sorted(int(i) for i in rng.choice(np.flatnonzero(ns == n), 8, replace=False))
    return sorted(pick)


def c4():
    spec = w.hetero_batch_spec()
    idx = c4_selection(spec)
    t0 = time.time()
    energy, grads, offs = [], [], [0]
    for i in idx:
        n, d, seed = spec[i]
        circ = w.hea_circuit(n, d)
        e, g, _ = oracle.adjoint(w.heisenberg(n), circ, w.angles(seed, circ.nparams), w.zero_state(n))
        energy.append(e[0])
        grads.append(g[0])
        offs.append(offs[-1] + circ.nparams)
    path = os.path.join(HERE, "c4_batch.npz")
    np.savez_compressed(path, index=np.array(idx, np.int64), energy=np.array(energy),
                        grad=np.concatenate(grads), offset=np.array(offs, np.int64))
    print("wrote", path, f"({len(idx)} circuits, {time.time() - t0:.1f} s)")


B64_SEEDS = (640, 641, 642, 643)


def b64_pattern(B=64):
    """Which of the 4 stored input states each of the B batch slots holds."""
    return np.random.default_rng(64).integers(0, len(B64_SEEDS), B)


def b64():
    n, depth = 20, 20
    circ = w.hea_circuit(n, depth)
    params = w.angles(2, circ.nparams)
    H = w.heisenberg(n)
    rows = []
    t0 = time.time()
    for j, seed in enumerate(B64_SEEDS):
        e, g, _ = oracle.adjoint(H, circ, params, w.random_state(n, 1, seed))
        rows += [(f"energy{j}", e), (f"grad{j}", g[0])]
    write("b64_states.txt",
          ["FP64 oracle: 20 qubits, Rx.Rz.Rx + open CNOT chain, depth 20, angles seed 2, periodic "
           "Heisenberg; input states workloads.random_state(20, 1, seed) for seeds "
           + " ".join(map(str, B64_SEEDS)),
           f"written by tests/golden/make_golden.py b64 ({time.time() - t0:.1f} s)"], rows)


def fd20():
    n, depth = 20, 20
    circ = w.hea_circuit(n, depth)
    params = w.angles(2, circ.nparams)
    H = w.heisenberg(n)
    which = sorted(int(k) for k in np.random.default_rng(24).choice(circ.nparams, 24, replace=False))
    t0 = time.time()
    fd = oracle.fd_grad(H, circ, params, w.zero_state(n), h=1e-4, which=which)
    sh = oracle.shift_grad(H, circ, params, w.zero_state(n), which=which)
    write("fd20.txt",
          ["FP64 oracle energies: 20 qubits, Rx.Rz.Rx + open CNOT chain, depth 20, angles seed 2, "
           "|0..0>, periodic Heisenberg; central differences h = 1e-4 and the shift rule",
           f"written by tests/golden/make_golden.py fd20 ({time.time() - t0:.1f} s)"],
          [("index", which), ("fd", [fd[k][0] for k in which]), ("shift", [sh[k][0] for k in which])])


if __name__ == "__main__":
    todo = sys.argv[1:] or ["vqe20", "rand20", "fwd25", "c4", "b64", "fd20"]
    for name in todo:
        globals()[name]()
