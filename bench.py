"""Benchmark: energy + all gradients of the 20-qubit Heisenberg VQE ansatz on one MI355X.

One step = reset the register to |0...0>, run the circuit, evaluate the periodic Heisenberg
energy, run the reversible adjoint sweep for all 1200 gradients and copy energy and
gradients to the host -- the whole hot path, on synthetic seeded angles.

Prints one JSON line. `value` is amplitude updates per second: per step, every gate of the
circuit counts 2^n * B updates in the forward sweep and 2 * 2^n * B in the reverse sweep
(psi and lambda). `roofline` describes the kernel family with the most GPU time, timed
with HIP events on the library's stream during the timed steps; `cpu_baseline` is the FP64
oracle on a bounded sample of the same workload on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "amplitude-updates/s & HBM GB/s, 20q fwd+grad; batched-adjoint vs plain speedup"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
FAMILIES = {0: "gate", 1: "adjoint", 2: "pass_fwd", 3: "pass_bwd", 4: "expect", 5: "hpsi", 6: "mfma", 7: "batch",
            8: "permute", 9: "qft", 10: "measure", 11: "krylov"}
KERNEL_NAMES = {0: "k_gate1/k_gatek", 1: "k_adjoint", 2: "k_pass_fwd", 3: "k_pass_bwd", 4: "k_expect", 5: "k_hpsi",
                6: "k_dense_mfma", 7: "k_batch", 8: "k_permute", 9: "k_qft_pass", 10: "measure kernels",
                11: "Krylov vector kernels"}


_T0 = time.time()


def log(msg):
    """Progress line on stderr (long measurements, run-time compiles): seconds since start."""
    print(f"bench [{time.time() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def measured_traffic(kernel, summary):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    profiles/<summary> (FETCH_SIZE and WRITE_SIZE per dispatch, calibrated by a cold copy of
    known size), or None when it does not cover the kernel as its source file stands now."""
    import hashlib

    for path in [os.path.join(ROOT, "profiles", summary)]:
        if not os.path.exists(path):
            continue
        fields = {}
        for line in open(path):
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                fields.setdefault(k.strip(), v.strip())
        src = fields.get("source_file")
        if fields.get("kernel") != kernel or not src or "traffic_bytes_per_launch" not in fields:
            continue
        sha = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()[:16]
        if sha == fields.get("source_sha256"):
            return float(fields["traffic_bytes_per_launch"])
    return None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--qubits", type=int, default=20)
    p.add_argument("--depth", type=int, default=20)
    p.add_argument("--batch", type=int, default=1)
    p.add_argument("--dtype", choices=["c64", "c128"], default="c64")
    p.add_argument("--mode", choices=["reversible", "checkpoint", "auto"], default="reversible")
    p.add_argument("--plain-steps", type=int, default=2)
    p.add_argument("--cpu-depth", type=int, default=20, help="depth of the oracle sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-profile", action="store_true")
    p.add_argument("--no-configs", action="store_true", help="skip the 10q/25q/20q-batch-64/30q figures")
    p.add_argument("--case", choices=CASES, help="run one workload --steps times for a profiler, and nothing else")
    p.add_argument("--no-next", action="store_true",
                   help="skip the shift-rule, QFT, permutation, sampling and time-evolution figures")
    p.add_argument("--batch-circuits", type=int, default=1024,
                   help="circuits of the uneven batch measured beside the main step (0: skip)")
    p.add_argument("--batch-steps", type=int, default=5)
    p.add_argument("--fuse-width", type=int, default=-1,
                   help="forward fusion width 0..5 with the autotuner off (-1: autotuned)")
    p.add_argument("--tile-qubits", type=int, default=0, help="tile qubits of the pass kernels (0: default)")
    p.add_argument("--jit", type=int, default=-1,
                   help="run-time compiled passes from this use of a bound program on (0: off; -1: the library "
                        "default, the third use: every timed measurement runs three warm-up calls first)")
    return p.parse_args()


def bench_uneven_batch(yb, w, torch, ncirc, steps):
    """Replays of the graph-recorded uneven batch (qubits 8..20, depth 4..16, complex64) against
    the same circuits run one by one through the per-gate form and through the fused form."""
    import numpy as np

    spec = w.hetero_batch_spec(ncirc)
    states, circs, hams, params = [], [], [], []
    for n, d, seed in spec:
        c = w.hea_circuit(n, d)
        states.append(yb.State(n, 1, yb.C64))
        circs.append(yb.Circuit.from_workload(c))
        hams.append(yb.PauliSum.from_workload(w.heisenberg(n)))
        params.append(w.angles(seed, c.nparams))
    gates = sum(3 * n * d + (n - 1) * d for n, d, _ in spec)
    au = sum(3.0 * (3 * n * d + (n - 1) * d) * (1 << n) for n, d, _ in spec)
    t0 = time.perf_counter()
    yb.batch_run(states, circs, params, hams)  # autotune + record
    torch.cuda.synchronize()
    t_record = time.perf_counter() - t0
    yb.batch_run(states, circs, params, hams)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        e, g = yb.batch_run(states, circs, params, hams)
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t0) * 1e3 / steps
    # A second list (every other circuit) called in turn with the first: each list replays its
    # own recorded graph, so a pair costs about one replay of each.
    half = slice(1, None, 2)
    lists = [(states, circs, params, hams), (states[half], circs[half], params[half], hams[half])]
    yb.batch_run(*lists[1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        yb.batch_run(*lists[1])
    torch.cuda.synchronize()
    half_ms = (time.perf_counter() - t0) * 1e3 / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        for lst in lists:
            yb.batch_run(*lst)
    torch.cuda.synchronize()
    pair_ms = (time.perf_counter() - t0) * 1e3 / steps

    def loop():
        for i in range(ncirc):
            states[i].reset()
            yb.backward(states[i], circs[i], params[i], hams[i])
        torch.cuda.synchronize()

    loop()
    t0 = time.perf_counter()
    loop()
    fused_loop_ms = (time.perf_counter() - t0) * 1e3
    saved = yb.get_options()
    yb.set_options(plain=1, fuse_width=0)
    t0 = time.perf_counter()
    loop()
    plain_ms = (time.perf_counter() - t0) * 1e3
    yb.set_options(plain=0, fuse_width=saved.fuse_width)
    return {"workload": f"{ncirc} circuits, qubits uniform 8..20, depth uniform 4..16, Rx.Rz.Rx + CNOT-chain "
                        "ansatz, periodic Heisenberg energy + all gradients per circuit, complex64",
            "circuits": ncirc, "gates": gates, "ms_per_batch": batch_ms,
            "amplitude_updates_per_s": au / (batch_ms / 1e3), "record_s": t_record,
            "half_list_ms": half_ms, "alternating_pair_ms": pair_ms,
            "fused_loop_ms": fused_loop_ms, "plain_loop_ms": plain_ms,
            "speedup_vs_plain": plain_ms / batch_ms, "speedup_vs_fused_loop": fused_loop_ms / batch_ms,
            "energy_sum": float(np.sum(e))}


def bench_configs(yb, w, torch):
    """The other configurations of the workload table, one figure set each: a 10-qubit
    fwd+grad latency, the 25-qubit forward (fused sweep and one per-gate launch against the HBM
    peak), the same-circuit batch of 64 at 20 qubits, and the 30-qubit precision run
    (complex64 with 5-qubit blocks on the FP32 matrix cores against complex128)."""
    import numpy as np

    def timed(f, reps):
        for _ in range(3):  # warm-up; a program's third use compiles its passes at run time
            f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    out = {}
    saved = yb.get_options()
    try:
        # 10 qubits, depth 5, complex128: fwd + energy + 150 gradients.
        c = w.hea_circuit(10, 5)
        cc, H, p = yb.Circuit.from_workload(c), yb.PauliSum.from_workload(w.heisenberg(10)), w.angles(0, c.nparams)
        s = yb.State(10, 1, yb.C128)

        def c1():
            s.reset()
            yb.backward(s, cc, p, H)
        out["c1_10q_fwd_grad_c128_us"] = round(timed(c1, 50) * 1e3, 1)
        log("config c1 (10 qubits, complex128) done")

        # 25 qubits, depth 20: forward + energy (autotuned fusion), complex64 and complex128;
        # and one Rx launch of the per-gate form (reads and writes the state once).
        c = w.hea_circuit(25, 20)
        cc, H, p = yb.Circuit.from_workload(c), yb.PauliSum.from_workload(w.heisenberg(25)), w.angles(1, c.nparams)
        for dt, name, sb in ((yb.C64, "c64", 8), (yb.C128, "c128", 16)):
            s = yb.State(25, 1, dt)

            def c2():
                s.reset()
                yb.forward(s, cc, p)
            ms = timed(c2, 3)
            e_ms = timed(lambda: yb.expect(s, H), 3)
            yb.set_options(plain=1)
            gate_ms = timed(lambda: s.apply_gate("Rx", (12,), theta=0.3), 20)
            yb.set_options(plain=saved.plain)
            gbs = 2.0 * sb * (1 << 25) / (gate_ms / 1e3) / 1e9
            out[f"c2_25q_fwd_{name}_ms"] = round(ms, 2)
            out[f"c2_25q_energy_{name}_ms"] = round(e_ms, 2)
            out[f"c2_25q_amplitude_updates_per_s_{name}"] = len(c.gates) * float(1 << 25) / (ms / 1e3)
            out[f"c2_25q_per_gate_{name}"] = {"us": round(gate_ms * 1e3, 1), "hbm_gbs": round(gbs, 1),
                                              "hbm_frac": round(gbs / HBM_PEAK_GBS, 3)}
            del s
            log(f"config c2 (25 qubits, {name}) done")

        # 20 qubits, depth 20, the same circuit on a batch of 64 states (512 MiB complex64).
        c = w.hea_circuit(20, 20)
        cc, H, p = yb.Circuit.from_workload(c), yb.PauliSum.from_workload(w.heisenberg(20)), w.angles(2, c.nparams)
        s = yb.State(20, 64, yb.C64)

        def c3():
            s.reset()
            yb.backward(s, cc, p, H)
        ms = timed(c3, 2)
        out["c3_20q_b64_fwd_grad_ms"] = round(ms, 2)
        out["c3_20q_b64_amplitude_updates_per_s"] = 3.0 * len(c.gates) * float(1 << 20) * 64 / (ms / 1e3)
        del s
        log("config c3 (20 qubits, batch 64) done")

        # 30 qubits, depth 24, Haar-random one-qubit layers + CZ pairs: complex64 with 5-qubit
        # blocks on the FP32 matrix cores against complex128 (one-qubit runs merged).
        c = w.random_circuit(30, 24, seed=5)
        cc = yb.Circuit.from_workload(c)
        zz = yb.PauliSum.from_workload(w.pauli_sum(30, [(1.0, "ZZ" + "I" * 28)]))
        t64 = torch.empty(1 << 30, dtype=torch.complex64, device="cuda")
        t128 = torch.empty(1 << 30, dtype=torch.complex128, device="cuda")
        s64, s128 = yb.State(30, 1, yb.C64, tensor=t64), yb.State(30, 1, yb.C128, tensor=t128)
        def f64():
            s64.reset()
            yb.forward(s64, cc, [])
        yb.set_options(autotune=1, mfma=1)
        ms64_tuned = timed(f64, 2)
        log("config c5 (30 qubits) autotuned complex64 done")
        yb.set_options(autotune=0, fuse_width=5, mfma=1)
        ms64 = timed(f64, 2)
        # One more forward with a pair of HIP events around every launch: the matrix-core blocks'
        # share of the HBM and FP32 matrix-core peaks, and the time of the passes between them.
        yb.lib().yao_profile_enable(1)
        f64()
        torch.cuda.synchronize()
        yb.lib().yao_profile_enable(0)
        mfma_prof = profile_family(yb, 6, with_flops=True)
        if mfma_prof:
            mfma_prof["mfma_frac"] = round(mfma_prof["achieved_tflops"] / FP32_PEAK_TFLOPS, 3)
        pass_prof = profile_family(yb, 2)
        w5_split = {"mfma_blocks": mfma_prof,
                    "pass_fwd_ms": round(pass_prof.get("launches", 0) * pass_prof.get("avg_launch_us", 0.0) / 1e3, 1),
                    "pass_fwd_launches": pass_prof.get("launches", 0)}
        log("config c5 (30 qubits) 5-qubit blocks done")
        yb.set_options(autotune=0, fuse_width=1)

        def f128():
            s128.reset()
            yb.forward(s128, cc, [])
        ms128 = timed(f128, 2)
        log("config c5 (30 qubits) complex128 done")
        fid = float(abs(torch.vdot(t128, t64.to(torch.complex128)).item()) ** 2)
        e64, e128 = float(yb.expect(s64, zz)[0]), float(yb.expect(s128, zz)[0])
        out["c5_30q"] = {"gates": len(c.gates), "c64_mfma_w5_ms": round(ms64, 1),
                         "c64_autotuned_ms": round(ms64_tuned, 1), "c64_mfma_w5_split": w5_split,
                         "c128_w1_ms": round(ms128, 1),
                         "fidelity_c64_vs_c128": fid, "z0z1_c64": e64, "z0z1_c128": e128,
                         "z0z1_abs_err": abs(e64 - e128)}
        del s64, s128, t64, t128
    finally:
        yb.set_options(autotune=saved.autotune, fuse_width=saved.fuse_width, mfma=saved.mfma, plain=saved.plain)
    return out


def bench_next_rows(yb, w, torch):
    """Figures of the rows beyond the gradient path: the faithful gradient (shift rule, every
    shifted circuit in one register) against the reversible adjoint at 10 and 20 qubits; the QFT
    kernel and a qubit permutation at 25 qubits against the HBM peak, and the QFT as a gate
    circuit; sampling a million shots from all 24 qubits; Krylov time evolution at 16 and 20
    qubits; and the 20-qubit step in checkpointed mode and in complex128."""
    import numpy as np

    def timed(f, reps):
        for _ in range(3):  # warm-up; a program's third use compiles its passes at run time
            f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    out = {}
    # Faithful gradient vs the reversible adjoint.
    for n, depth, dt, reps in ((10, 5, yb.C128, 3), (20, 20, yb.C64, 1)):
        c = w.hea_circuit(n, depth)
        cc, H, p = yb.Circuit.from_workload(c), yb.PauliSum.from_workload(w.heisenberg(n)), w.angles(2, c.nparams)
        s = yb.State(n, 1, dt)
        shift_ms = timed(lambda: yb.shift_grad(s, cc, p, H), reps)

        def adj():
            s.reset()
            yb.backward(s, cc, p, H)
        adj_ms = timed(adj, 10)
        out[f"f1_shift_{n}q"] = {"params": c.nparams, "circuits": 2 * c.nparams + 1,
                                 "dtype": "c128" if dt == yb.C128 else "c64", "shift_ms": round(shift_ms, 2),
                                 "adjoint_ms": round(adj_ms, 3), "shift_over_adjoint": round(shift_ms / adj_ms, 1)}
        log(f"next row f1 shift rule ({n} qubits) done")
        del s
    # QFT kernel and qubit permutation at 25 qubits.
    n = 25
    for dt, name, es in ((yb.C128, "c128", 16), (yb.C64, "c64", 8)):
        s = yb.State(n, 1, dt)
        locs = list(range(n))
        yb.lib().yao_profile_enable(1)
        qms = timed(lambda: yb.qft(s, locs), 5)
        yb.lib().yao_profile_enable(0)
        prof = profile_family(yb, 9)
        t = yb.State(n, 1, dt)
        perm = list(range(n - 1, -1, -1))
        yb.lib().yao_profile_enable(1)
        pms = timed(lambda: yb.permute_qubits(s, t, perm), 5)
        yb.lib().yao_profile_enable(0)
        pprof = profile_family(yb, 8)
        out[f"f4_qft_25q_{name}"] = {"ms": round(qms, 3), **prof}
        out[f"f4_permute_25q_{name}"] = {"ms": round(pms, 3), **pprof}
        log(f"next row f4 QFT and permutation (25 qubits, {name}) done")
        if dt == yb.C128:
            out["f4_qft_25q_c128"]["traffic_per_launch"] = measured_traffic("k_qft_b1<double, false, 3>",
                                                                            "k_qft_b1_qft25_c128.txt")
            out["f4_permute_25q_c128"]["traffic_per_launch"] = measured_traffic(
                "k_permute_b1<HIP_vector_type<double, 2u>, 8>", "k_permute_b1_perm25_c128.txt")
        else:
            out["f4_qft_25q_c64"]["traffic_per_launch"] = measured_traffic("k_qft_b1<float, false, 4>",
                                                                           "k_qft_b1_qft25_c64.txt")
        if dt == yb.C128:
            qc = yb.Circuit.from_workload(w.qft_circuit(n))
            out["f4_qft_25q_c128"]["gate_circuit_ms"] = round(timed(lambda: yb.forward(s, qc, []), 2), 3)
        del s, t
    # Sampling: all 24 qubits of a state after two ansatz layers, 2^20 shots.
    n = 24
    c = w.hea_circuit(n, 2)
    s = yb.State(n, 1, yb.C128)
    yb.forward(s, yb.Circuit.from_workload(c), w.angles(3, c.nparams))
    u = np.random.default_rng(0).random((1, 1 << 20))
    yb.lib().yao_profile_enable(1)
    mms = timed(lambda: yb.measure(s, list(range(n)), u), 3)
    yb.lib().yao_profile_enable(0)
    out["f2_measure_24q_c128"] = {"shots": 1 << 20, "ms": round(mms, 3), **profile_family(yb, 10)}
    log("next row f2 measurement done")
    del s
    # Time evolution (the 16-qubit size of Listing "Hamiltonian evolution is faster with cache").
    for n in (16, 20):
        H = yb.PauliSum.from_workload(w.heisenberg(n))
        s = yb.State(n, 1, yb.C128)
        psi = w.random_state(n, 1, n)

        def te():
            s.upload(psi)
            return yb.time_evolve(s, H, 0.1)
        steps = te()
        up_ms = timed(lambda: s.upload(psi), 3)
        te_ms = timed(te, 3) - up_ms
        out[f"f3_evolve_{n}q_c128"] = {"t": 0.1, "substeps": steps, "ms": round(te_ms, 3)}
        log(f"next row f3 time evolution ({n} qubits) done")
        del s
    # The headline step in checkpointed mode, and in complex128.
    c = w.hea_circuit(20, 20)
    cc, H, p = yb.Circuit.from_workload(c), yb.PauliSum.from_workload(w.heisenberg(20)), w.angles(2, c.nparams)
    for dt, mode, key in ((yb.C64, yb.GRAD_CHECKPOINT, "c3_20q_checkpoint_c64_ms"),
                          (yb.C128, yb.GRAD_REVERSIBLE, "c3_20q_reversible_c128_ms")):
        s = yb.State(20, 1, dt)

        def st():
            s.reset()
            yb.backward(s, cc, p, H, mode=mode)
        out[key] = round(timed(st, 10), 3)
        del s
    return out


def profile_family(yb, fam, with_flops=False):
    """Launches, mean duration and algorithmic GB/s (and TFLOP/s) of one kernel family since
    profiling was last enabled (HIP events on the library's stream)."""
    import ctypes
    yb.lib().yao_profile_read.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    nl, ms, by, fl = ctypes.c_int(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    yb.lib().yao_profile_read(fam, ctypes.byref(nl), ctypes.byref(ms), ctypes.byref(by), ctypes.byref(fl))
    if not nl.value:
        return {}
    gbs = by.value / (ms.value / 1e3) / 1e9
    r = {"launches": nl.value, "avg_launch_us": round(ms.value * 1e3 / nl.value, 2),
         "algo_bytes_per_launch": by.value / nl.value, "achieved_gbs": round(gbs, 1),
         "hbm_frac": round(gbs / HBM_PEAK_GBS, 3)}
    if with_flops:
        r["algo_flops_per_launch"] = fl.value / nl.value
        r["achieved_tflops"] = round(fl.value / (ms.value / 1e3) / 1e12, 2)
    return r


CASES = ("step20", "step20_b64", "rx25_c128", "rx25_c64", "fwd25_c128", "fwd25_c64", "w5mfma30_c64",
         "qft25_c128", "qft25_c64", "perm25_c128", "measure24_c128", "copy1g", "c4batch")


def run_case(name, reps, jit=-1):
    """One workload, repeated, for profiling runs (rocprofv3 kernel traces and counters): each
    case launches only what it names, after one untimed run, and prints its wall time per rep.
    jit >= 0 overrides the case's compiled-pass setting (0: the generic pass kernels only)."""
    import numpy as np
    import torch

    import workloads as w
    from paper_1912_10877_amd import binding as yb

    torch.cuda.set_device(0)
    yb.init()
    yb.use_torch_stream()
    if name == "copy1g":
        # Calibration of the traffic counters: a copy of known size, 1 GiB read and 1 GiB written
        # per launch (a 27-qubit complex64 register with its two top qubits swapped, so every
        # row of the tile moves whole), rotating over three registers so that each source was
        # last written two launches (2 GiB, 8x the 256 MB Infinity Cache) earlier.
        regs = [yb.State(27, 1, yb.C64) for _ in range(3)]
        perm = list(range(25)) + [26, 25]
        it = [0]

        def f():
            i = it[0] % 3
            yb.permute_qubits(regs[i], regs[(i + 1) % 3], perm)
            it[0] += 1
    elif name in ("step20", "step20_b64"):
        # The headline step with the forward fusion the autotuner picks for it (runs of one-qubit
        # gates merged), fixed so that no timing trial runs under the profiler.
        B = 64 if name == "step20_b64" else 1
        # Compiled passes from the first (untimed) call on, so every profiled step runs them.
        yb.set_options(autotune=0, fuse_width=1, jit=1)
        c = w.hea_circuit(20, 20)
        cc, H, p = yb.Circuit.from_workload(c), yb.PauliSum.from_workload(w.heisenberg(20)), w.angles(2, c.nparams)
        s = yb.State(20, B, yb.C64)

        def f():
            s.reset()
            yb.backward(s, cc, p, H)
    elif name.startswith("rx25"):
        s = yb.State(25, 1, yb.C128 if name.endswith("c128") else yb.C64)
        yb.set_options(plain=1)
        f = lambda: s.apply_gate("Rx", (12,), theta=0.3)
    elif name.startswith("fwd25"):
        c = w.hea_circuit(25, 20)
        cc, p = yb.Circuit.from_workload(c), w.angles(1, c.nparams)
        s = yb.State(25, 1, yb.C128 if name.endswith("c128") else yb.C64)
        yb.set_options(autotune=0, fuse_width=1)

        def f():
            s.reset()
            yb.forward(s, cc, p)
    elif name == "w5mfma30_c64":
        cc = yb.Circuit.from_workload(w.random_circuit(30, 24, seed=5))
        s = yb.State(30, 1, yb.C64)
        yb.set_options(autotune=0, fuse_width=5, mfma=1)

        def f():
            s.reset()
            yb.forward(s, cc, [])
    elif name.startswith("qft25"):
        s = yb.State(25, 1, yb.C128 if name.endswith("c128") else yb.C64)
        f = lambda: yb.qft(s, list(range(25)))
    elif name == "perm25_c128":
        s, t = yb.State(25, 1, yb.C128), yb.State(25, 1, yb.C128)
        perm = list(range(24, -1, -1))
        f = lambda: yb.permute_qubits(s, t, perm)
    elif name == "measure24_c128":
        c = w.hea_circuit(24, 2)
        s = yb.State(24, 1, yb.C128)
        yb.forward(s, yb.Circuit.from_workload(c), w.angles(3, c.nparams))
        u = np.random.default_rng(0).random((1, 1 << 20))
        f = lambda: yb.measure(s, list(range(24)), u)
    elif name == "c4batch":
        # The 1024-circuit uneven batch (complex64), replayed: a kernel trace counts the
        # launches of one replay (from one k_bind_jobs dispatch to the next).
        spec = w.hetero_batch_spec(1024)
        states, circs, hams, params = [], [], [], []
        for n, d, seed in spec:
            c = w.hea_circuit(n, d)
            states.append(yb.State(n, 1, yb.C64))
            circs.append(yb.Circuit.from_workload(c))
            hams.append(yb.PauliSum.from_workload(w.heisenberg(n)))
            params.append(w.angles(seed, c.nparams))
        f = lambda: yb.batch_run(states, circs, params, hams)
    else:
        raise SystemExit(f"unknown case {name}; cases: {', '.join(CASES)}")
    if jit >= 0:
        yb.set_options(jit=jit)
    f()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        f()
    torch.cuda.synchronize()
    print(json.dumps({"case": name, "reps": reps, "ms_per_rep": (time.perf_counter() - t0) * 1e3 / reps}))


def main():
    args = parse()
    if args.case:
        run_case(args.case, args.steps, args.jit)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(sharding the state over GPUs is designed but not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as w
    from paper_1912_10877_amd import binding as yb

    torch.cuda.set_device(0)
    yb.init()
    yb.use_torch_stream()
    if args.fuse_width >= 0:
        yb.set_options(autotune=0, fuse_width=args.fuse_width)
    if args.jit >= 0:
        yb.set_options(jit=args.jit)
    if args.tile_qubits:
        yb.set_options(tile_qubits=args.tile_qubits)
    n, depth, B = args.qubits, args.depth, args.batch
    dtype = yb.C64 if args.dtype == "c64" else yb.C128
    mode = {"reversible": yb.GRAD_REVERSIBLE, "checkpoint": yb.GRAD_CHECKPOINT, "auto": yb.GRAD_AUTO}[args.mode]
    circ_w = w.hea_circuit(n, depth)
    H_w = w.heisenberg(n)
    params = w.angles(2, circ_w.nparams)
    circ = yb.Circuit.from_workload(circ_w)
    H = yb.PauliSum.from_workload(H_w)
    ngates = len(circ_w.gates)
    tensor = torch.empty((1 << n) * B, dtype=torch.complex64 if dtype == yb.C64 else torch.complex128, device="cuda")
    s = yb.State(n, B, dtype, tensor=tensor)

    def step():
        s.reset()
        return yb.backward(s, circ, params, H, mode=mode)

    for _ in range(args.warmup):
        e, g, drift = step()
    torch.cuda.synchronize()
    log("headline warm-up done (run-time compiles included)")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e, g, drift = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {}
    if not args.no_profile:
        # The same K steps again with a pair of HIP events around every launch (on the
        # library's stream): per-kernel durations for the roofline. The events slow the host's
        # launches, so the step time above is taken without them.
        import ctypes
        js0 = yb.jit_stats()
        yb.lib().yao_profile_enable(1)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        yb.lib().yao_profile_enable(0)
        js1 = yb.jit_stats()
        jit_fwd = js1["fwd_launches"] > js0["fwd_launches"]
        jit_bwd = js1["bwd_launches"] > js0["bwd_launches"]
        yb.lib().yao_profile_read.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        for fam in FAMILIES:
            nl, ms, by, fl = ctypes.c_int(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            yb.lib().yao_profile_read(fam, ctypes.byref(nl), ctypes.byref(ms), ctypes.byref(by), ctypes.byref(fl))
            if nl.value:
                prof[fam] = (nl.value, ms.value, by.value, fl.value)
    ms_step = (t1 - t0) * 1e3 / args.steps
    au_step = 3.0 * ngates * (1 << n) * B
    value = au_step / (ms_step / 1e3)

    # Plain per-gate form on the same GPU and dtype, for the speedup.
    plain_ms = None
    if args.plain_steps > 0:
        saved = yb.get_options()
        yb.set_options(plain=1, fuse_width=0)
        step()
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            step()
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - p0) * 1e3 / args.plain_steps
        yb.set_options(plain=0, fuse_width=saved.fuse_width)

    roofline = None
    if prof:
        fam = max(prof, key=lambda f: prof[f][1])
        nl, ms, by, fl = prof[fam]
        gbs = by / (ms / 1e3) / 1e9
        tfl = fl / (ms / 1e3) / 1e12
        peak_alu = FP64_PEAK_TFLOPS if fam in (1, 3) or dtype == yb.C128 else FP32_PEAK_TFLOPS / 2
        if gbs / HBM_PEAK_GBS >= tfl / peak_alu:
            roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}
        else:
            roofline = {"bound": "alu", "achieved": round(tfl, 3), "peak": peak_alu, "unit": "TFLOP/s",
                        "frac": round(tfl / peak_alu, 4), "traffic": None}
        # The pass families run the run-time compiled kernels once a program has compiled.
        kname = KERNEL_NAMES[fam]
        if fam == 3 and jit_bwd:
            kname = "yao_pass_bwd"
        elif fam == 2 and jit_fwd:
            kname = "yao_pass_fwd"
        if dtype == yb.C64 and B == 1 and fam in (2, 3):
            summary = {"k_pass_bwd": "k_pass_bwd_vqe20.txt", "k_pass_fwd": "k_pass_fwd_vqe20.txt",
                       "yao_pass_bwd": "yao_pass_bwd_vqe20.txt", "yao_pass_fwd": "yao_pass_fwd_vqe20.txt"}[kname]
            counted = {"k_pass_bwd": "k_pass_bwd<float, true>", "k_pass_fwd": "k_pass_fwd<float>"}.get(kname, kname)
            roofline["traffic"] = measured_traffic(counted, summary)
        roofline.update({"kernel": kname, "launches_per_step": nl / args.steps,
                         "avg_launch_us": round(ms * 1e3 / nl, 2), "algo_bytes_per_launch": by / nl,
                         "algo_flops_per_launch": fl / nl, "achieved_gbs": round(gbs, 1),
                         "achieved_tflops": round(tfl, 3),
                         "gpu_ms_by_family": {FAMILIES[f]: round(prof[f][1] / args.steps, 4) for f in prof}})

    batch = None
    if args.batch_circuits > 0:
        batch = bench_uneven_batch(yb, w, torch, args.batch_circuits, args.batch_steps)
        log("uneven batch done")

    configs = None
    if not args.no_configs:
        configs = bench_configs(yb, w, torch)
        log("configurations done")
    nxt = None
    if not args.no_next:
        nxt = bench_next_rows(yb, w, torch)
        log("next rows done")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cd = max(1, min(args.cpu_depth, depth))
        sub = w.hea_circuit(n, cd)
        sp = w.angles(2, sub.nparams)
        c0 = time.perf_counter()
        oracle.adjoint(H_w, sub, sp, w.zero_state(n, 1))
        c1 = time.perf_counter()
        au = 3.0 * len(sub.gates) * (1 << n)
        cpu = {"value": au / (c1 - c0), "unit": "amplitude-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"FP64 C oracle, energy + adjoint gradients of the same ansatz at n={n}, depth {cd} "
                         f"({len(sub.gates)} gates, batch 1), {c1 - c0:.2f} s wall"}

    out = {
        "metric": METRIC, "value": value, "unit": "amplitude-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"vqe{n}: {n}-qubit Rx.Rz.Rx + CNOT-chain ansatz, depth {depth}, "
                               f"{circ_w.nparams} params, periodic Heisenberg energy + all gradients, "
                               f"{args.mode} adjoint", "qubits": n, "depth": depth, "batch": B,
                   "params": circ_w.nparams, "gates": ngates, "grad_mode": args.mode,
                   "forward_fusion": "autotuned" if args.fuse_width < 0 else args.fuse_width,
                   "jit": yb.get_options().jit},
        "energy": float(e[0]), "drift": drift, "jit_stats": yb.jit_stats(),
        "plain_ms_per_step": plain_ms,
        "speedup_vs_plain": (plain_ms / ms_step) if plain_ms else None,
        "roofline": roofline, "cpu_baseline": cpu, "uneven_batch": batch, "configs": configs, "next_rows": nxt,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
