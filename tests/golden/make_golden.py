"""Write the stored oracle results that the full-size GPU parity tests compare against.

Only the FP64 oracle (oracle/) computes these values; nothing here touches the GPU path.
Run:  python tests/golden/make_golden.py [vqe20] [fwd25] [rand20]

  vqe20   20-qubit Rx.Rz.Rx + CNOT-chain ansatz, depth 20, angles seed 2, |0..0>, periodic
          Heisenberg: energy and all 1200 adjoint gradients (the differentiation workload).
  fwd25   25-qubit same ansatz, depth 20, angles seed 1: energy after the forward sweep.
  rand20  20-qubit random circuit (Haar SU(2) layers + CZ pairings), depth 24, seed 5:
          <Z0 Z1> and <X0> of the output (the precision workload's oracle cross-check).
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


if __name__ == "__main__":
    todo = sys.argv[1:] or ["vqe20", "rand20", "fwd25"]
    for name in todo:
        globals()[name]()
