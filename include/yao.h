/*
 * yao.h -- C ABI of the MI355X (gfx950) state-vector library.
 *
 * The operations follow the problem statement of Yao (arXiv:1912.10877):
 *   - registers and batched registers: Sec. "Quantum Registers", "Batched Quantum Registers";
 *   - gate instructions instruct!(reg, G, locs, ctrl_locs, ctrl_configs[, theta]):
 *     Sec. "Instructions on Quantum Registers";
 *   - circuits as chains of put/control blocks applied in order: Sec. "Representing
 *     Quantum Circuits";
 *   - expect(H, reg) of a sum of Pauli strings: Sec. "Matrix Representation" (Listing
 *     "Heisenberg Hamiltonian") and Sec. "Forward Mode";
 *   - expect'(H, reg => circuit): reverse mode with uncomputation, eqs. apply-back and
 *     outer-product of Sec. "Reverse Mode".
 *
 * Conventions shared by every call:
 *   - Qubits are 0-based; qubit q is bit q of the amplitude index (the paper's
 *     little-endian readout, 1-based qubits).
 *   - A state of n qubits and batch B is 2^n * B complex numbers, element (i, b) at
 *     offset i*B + b (batch innermost), re/im interleaved: complex64 = 2 x float,
 *     complex128 = 2 x double.
 *   - A k-qubit matrix on locs l_0..l_{k-1} is 2^k x 2^k complex128, row-major,
 *     re/im interleaved (2 * 4^k doubles); locs[j] is bit j of its row/column index.
 *   - A control (c, v) passes when bit c of the amplitude index equals v (v = 0 is
 *     the paper's "inverse control"). ctrl_vals == NULL means all ones.
 *   - Every call returns 0 on success or a negative yao_status. Validation happens on the
 *     host before any launch; a call that fails validation leaves every state unchanged.
 *     yao_last_error() returns the message of the last failure in this thread.
 *   - Device work goes to the stream set with yao_set_stream (default: the null stream)
 *     and is asynchronous, except for calls that return host values (yao_expect,
 *     yao_backward, yao_batch_run, yao_state_download), which synchronise that stream.
 *   - Host arrays passed in are copied during the call; the caller keeps ownership.
 *     Output arrays are caller-allocated host memory.
 *   - The library targets gfx950 only. Calls on a machine without such a device fail
 *     with YAO_ENODEV.
 */
#ifndef YAO_C_ABI_H_
#define YAO_C_ABI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct yao_state yao_state;
typedef struct yao_circuit yao_circuit;
typedef struct yao_pauli_sum yao_pauli_sum;

enum yao_status {
    YAO_OK = 0,
    YAO_EINVAL = -1,   /* invalid argument (message says which) */
    YAO_ENOMEM = -2,   /* device allocation failed */
    YAO_EHIP = -3,     /* HIP runtime error */
    YAO_EDRIFT = -4,   /* reversible uncompute drifted past the bound with fallback disabled */
    YAO_ENODEV = -5    /* no gfx950 device */
};

enum yao_dtype { YAO_C64 = 0, YAO_C128 = 1 };

/* Gate kinds (App. "Builtin blocks"). Rotations are R_G(theta) = exp(-i theta G / 2) with G
 * Hermitian and reflexive (Sec. "Forward Mode"); YAO_ROT takes G as a dense 2^k x 2^k
 * matrix. YAO_SHIFT is diag(1, e^{i theta}) (Listing "inspecting gates"). YAO_DENSE is an
 * arbitrary unitary (matblock). */
enum yao_gate {
    YAO_X = 0, YAO_Y = 1, YAO_Z = 2, YAO_H = 3, YAO_S = 4, YAO_SDAG = 5, YAO_T = 6, YAO_TDAG = 7,
    YAO_RX = 8, YAO_RY = 9, YAO_RZ = 10, YAO_SHIFT = 11, YAO_ROT = 12, YAO_DENSE = 13
};

/* Backward strategies. REVERSIBLE uncomputes the state with inverse gates (constant memory
 * in depth, Sec. "Reverse Mode"). CHECKPOINT cuts the circuit into segments of
 * checkpoint_every gates, keeps the forward state at every segment end and restarts the
 * reverse sweep of each segment from it (memory grows with depth). AUTO runs the reversible
 * sweep (constant memory) and, when the uncomputed input differs from the input by more than
 * drift_tol, restores the input and runs the CHECKPOINT sweep instead; only then are
 * checkpoints allocated. */
enum yao_grad_mode { YAO_GRAD_REVERSIBLE = 0, YAO_GRAD_CHECKPOINT = 1, YAO_GRAD_AUTO = 2 };

/* Execution options (process-wide; set before the calls they should affect).
 *   plain            1: one kernel launch per gate (the per-gate form); 0: fused tile passes.
 *   tile_qubits      qubits per fused tile (0 = chosen by the library or the autotuner).
 *   fuse_width       fusion of forward sweeps (yao_forward, the forward sweep of a
 *                    REVERSIBLE yao_backward, yao_batch_run) when autotune is 0: 0 = none,
 *                    1 = runs of one-qubit gates on one qubit merged into one matrix,
 *                    2..5 = gates folded into dense blocks of up to that many qubits (the
 *                    reverse sweep always takes the gates one by one).
 *   checkpoint_every gates per segment in CHECKPOINT / AUTO mode (0 = max(sqrt(#gates), 4n)).
 *   drift_tol        max |psi_0 uncomputed - psi_0| accepted by AUTO before falling back
 *                    (0 = 1e-5 for complex64 states, 1e-10 for complex128). In REVERSIBLE
 *                    mode a drift_tol > 0 makes yao_backward return YAO_EDRIFT when the
 *                    uncomputed input differs from the input by more than drift_tol (the
 *                    outputs are still written).
 *   mfma             1: dense blocks of 4 or 5 qubits on complex64 states run on FP32
 *                    matrix cores; 0: on the vector units.
 *   autotune         1 (default): the library picks the fusion width of forward sweeps
 *                    per circuit and state shape (and, in yao_batch_run, per qubit count
 *                    together with the tile qubits of both sweeps) by timing the candidates
 *                    on the device the first time it meets them; the state is restored after
 *                    the trials. Which candidate wins depends on timings, so results may
 *                    differ in the last bits between processes. 0: fuse_width and
 *                    tile_qubits are taken as given.
 *   jit              0: off. N >= 1 (default 3): when a device-bound program (a circuit
 *                    whose matrices are bound from the parameters on the device) runs its
 *                    N-th forward sweep on a single-slot state, its passes are compiled at run
 *                    time (hipRTC) into straight-line kernels that read the same op records,
 *                    so later parameter changes need no recompile. Passes outside the
 *                    compiled form (batched states, LDS-applied ops, dense blocks, tiles over
 *                    64 KiB), autotuner trials and graph recording keep the generic kernels; a
 *                    failed compile leaves the program on them. Compiling takes ~0.4 s per
 *                    pass family of ~70 ops, once per program. */
typedef struct {
    int plain;
    int tile_qubits;
    int fuse_width;
    int checkpoint_every;
    double drift_tol;
    int mfma;
    int autotune;
    int jit;
} yao_options;

/* Library ------------------------------------------------------------------------------ */

/* Select the current HIP device, check that it is gfx950, reset options to defaults. */
int yao_init(void);
const char* yao_last_error(void);
/* Bind the stream (a hipStream_t, or NULL for the null stream) that later calls use. */
int yao_set_stream(void* hip_stream);
int yao_synchronize(void);
int yao_set_options(const yao_options* opt);
int yao_get_options(yao_options* opt);

/* States (a1) --------------------------------------------------------------------------- */

/* Allocate a state of n qubits (1 <= n <= 34) and batch >= 1, set to |0...0> in every slot
 * (the paper's zero_state(n; nbatch)). The library owns the memory. */
int yao_state_create(int n, int batch, enum yao_dtype dt, yao_state** out);
/* Wrap caller-owned device memory of 2^n * batch elements (e.g. a torch tensor); the
 * library never frees it. The pointer must stay valid while the state is used. */
int yao_state_wrap(void* dev_ptr, int n, int batch, enum yao_dtype dt, yao_state** out);
int yao_state_destroy(yao_state* s);
/* |0...0> in every batch slot. */
int yao_state_reset(yao_state* s);
/* Copy a host state in the layout above; bytes must equal the state's size. */
int yao_state_upload(yao_state* s, const void* host, size_t bytes);
int yao_state_download(const yao_state* s, void* host, size_t bytes);
/* Device pointer, qubit count, batch and dtype of a state. */
int yao_state_info(const yao_state* s, void** dev_ptr, int* n, int* batch, int* dtype);

/* Gate instructions (a2, a3, a4) --------------------------------------------------------- */

/* Apply a k-qubit matrix U (1 <= k <= 5) on locs, with nctrl controls (instruct! with a
 * general matrix). Errors: YAO_EINVAL for a loc or control out of range, repeated qubits,
 * a control on a target, k out of range. U is rounded once to the state's precision. */
int yao_apply(yao_state* s, const double* U, int k, const int* locs, int nctrl, const int* ctrls,
              const int* ctrl_vals);
/* Apply a named gate; theta is used by the parametric kinds, G by YAO_ROT (generator) and
 * YAO_DENSE (matrix), k is the number of locs (1 for every kind but YAO_ROT/YAO_DENSE). */
int yao_apply_gate(yao_state* s, enum yao_gate g, double theta, const double* G, const int* locs, int k,
                   int nctrl, const int* ctrls, const int* ctrl_vals);

/* Observables (a5, a6) --------------------------------------------------------------- */

/* H = sum_t coef[t] P_t on n qubits; P_t has X on the bits set only in xmask[t], Z on the
 * bits set only in zmask[t], Y on the bits set in both. */
int yao_pauli_sum_create(int n, int nterms, const double* coef, const uint64_t* xmask, const uint64_t* zmask,
                         yao_pauli_sum** out);
int yao_pauli_sum_destroy(yao_pauli_sum* h);
/* energy[b] = Re <psi_b|H|psi_b> for every batch slot, accumulated in FP64. Synchronises. */
int yao_expect(const yao_state* s, const yao_pauli_sum* h, double* energy);
/* yao_expect for callers that cannot allocate device memory (code under graph capture, tight
 * serving loops, harnesses that forbid hipMalloc). Same result as yao_expect (one read of the
 * state per X-mask group of the terms), but the term tables and every partial sum live in a
 * static device array of 2 MiB that each GPU holds from the library's load until the process
 * ends; no hipMalloc, hipFree or other allocating call is made. Limits: at most 4096 terms and
 * batch * min(2^n * batch_block / 256, 1024) <= 131072 partial sums (batch <= 128 for n >= 10);
 * YAO_EINVAL beyond them. All calls on one GPU share the array, which keeps the last call's
 * contents (every value a call reads is written earlier in that call): calls that overlap on
 * one GPU, from several threads or streams, race. Synchronises the bound stream. */
int yao_expect_noalloc(const yao_state* s, const yao_pauli_sum* h, double* energy);
/* out = H psi (the adjoint seed of the reverse mode) and, if energy != NULL,
 * energy[b] = Re <psi_b|H psi_b> from the same pass. out must match s in n, batch, dtype. */
int yao_hpsi(const yao_state* s, const yao_pauli_sum* h, yao_state* out, double* energy);

/* re[b] + i im[b] = <a_b|b_b> for every batch slot, accumulated in FP64 (the overlap behind
 * the fidelity |<a|b>|^2 of App. "Gate Learning"). a and b must have equal n and batch; their
 * dtypes may differ. Synchronises. */
int yao_inner(const yao_state* a, const yao_state* b, double* re, double* im);

/* Qubit management and the QFT (f4) ------------------------------------------------------- */

/* dst = src with qubit q moved to index bit perm[q] (perm: a permutation of 0..n-1); the
 * building block of focus! / relax! (Sec. "Active qubits and environment qubits"). src and dst
 * must match in n, batch and dtype; dst == src permutes in place (through a library buffer of
 * the state's size). Batch * element bytes <= 16 KiB. */
int yao_permute_qubits(const yao_state* src, yao_state* dst, const int* perm);
/* focus!(reg, locs): qubit locs[j] becomes qubit j (the active qubits, in the given order) and
 * the other qubits follow in ascending order; relax! with the same locs undoes it. In place;
 * 1 <= k <= n distinct locs. */
int yao_focus(yao_state* s, const int* locs, int k);
int yao_relax(yao_state* s, const int* locs, int k);
/* QFT on the k qubits locs (locs[j] = bit j of the transform's index x), in place (App.
 * "Extending QBIR: emulating QFT circuit"): out[y] = 2^{-k/2} sum_x exp(2 pi i rev_k(x) y / 2^k)
 * psi[x], which is the QFT circuit of Listing "QFT circuit" on those qubits (no final swaps),
 * i.e. the paper's emulation by reversing the qubit order and applying the unitary inverse
 * DFT. inverse = 1 applies the adjoint. Computed by in-place radix-2 stages in LDS tiles (a
 * few passes over the state), not by gates. Batch * element bytes <= 16 KiB. */
int yao_qft(yao_state* s, const int* locs, int k, int inverse);

/* Faithful gradient (f1) ------------------------------------------------------------------ */

/* The gradient by the shift rule (Sec. "Forward Mode: Faithful Quantum Gradients", eq.
 * shiftrule), as an experiment would measure it: for every parametrised gate occurrence, the
 * energies with that gate's angle moved by +pi/2 and by -pi/2 give (E+ - E-) / 2, added to the
 * gradient of its parameter (a parameter shared by several gates gets the sum over its gates).
 * Exact for rotations exp(-i theta G / 2) with G reflexive and for phase shifts; for controlled
 * rotations it is the rule's value, not the derivative. All 2K + 1 circuits (K occurrences, plus
 * the unshifted one) run as one register of n + s qubits whose top s bits select the circuit
 * (in chunks when it would exceed a quarter of the free device memory): one forward sweep
 * through the fused passes, one expectation pass with a sum per circuit. s is the input state
 * (batch 1, unchanged); energy[0] receives the unshifted energy, grad[p] the gradients.
 * Synchronises. */
int yao_shift_grad(const yao_state* s, const yao_circuit* c, const double* params, const yao_pauli_sum* h,
                   double* energy, double* grad);

/* Time evolution (f3) --------------------------------------------------------------------- */

/* psi_b <- exp(-i H t) psi_b for every slot (time_evolve of Sec. "Matrix Representation"), by
 * the Krylov (Lanczos) method: H is applied to the register krylov_dim times per substep (the
 * H psi tile passes; 0 = 30 vectors, at most 64), the projected tridiagonal problem is
 * exponentiated on the host, and the substep is halved until the error estimate
 * |psi| beta_m |(exp(-i tau T) e_1)_m| <= tol (0 = 1e-12 for complex128, 1e-6 for complex64).
 * Needs krylov_dim + 2 state-sized library buffers. nsteps (may be NULL) receives the number of
 * substeps. Synchronises. */
int yao_time_evolve(yao_state* s, const yao_pauli_sum* h, double t, double tol, int krylov_dim, int* nsteps);

/* Measurement (f2) ---------------------------------------------------------------------- */

/* Outcomes of the k qubits locs are x = sum_j bit(locs[j]) 2^j (1 <= k <= min(n, 30)); every
 * batch slot is measured on its own (Sec. "Batched Quantum Registers"). Probabilities are summed
 * in FP64 in a fixed order, so results repeat bit for bit. Batch * element bytes <= 16 KiB.
 *
 * probs[b * 2^k + x] = sum of |psi_b[i]|^2 over the indices i whose locs read x. Synchronises. */
int yao_probs(const yao_state* s, const int* locs, int k, double* probs);
/* measure(reg; nshots) (Listing "instruct! and measure"): shot j of slot b is the smallest x
 * with C_b(x) > u[b * nshots + j] * C_b(2^k - 1), C_b the cumulative sums of the probabilities in
 * the order of x (inverse-CDF sampling). The caller supplies the uniform numbers u in [0, 1)
 * (YAO_EINVAL otherwise); out[b * nshots + j] receives x. The state is unchanged. Synchronises. */
int yao_measure(const yao_state* s, const int* locs, int k, int nshots, const double* u, uint64_t* out);
/* measure!: one shot per slot from u[b] as in yao_measure, then slot b is projected onto its
 * outcome and renormalised (amplitudes whose locs read x_b divided by sqrt(p_b), the others
 * set to 0). out[b] = x_b; prob[b] = p_b if prob != NULL. Synchronises. */
int yao_measure_collapse(yao_state* s, const int* locs, int k, const double* u, uint64_t* out, double* prob);

/* Circuits ---------------------------------------------------------------------------- */

int yao_circuit_create(int n, yao_circuit** out);
int yao_circuit_destroy(yao_circuit* c);
/* Append a gate. param_index >= 0 takes the angle from params[param_index] at run time
 * (several gates may share one); -1 uses theta_fixed. G as for yao_apply_gate. */
int yao_circuit_push(yao_circuit* c, enum yao_gate g, int param_index, double theta_fixed, const double* G,
                     const int* locs, int k, int nctrl, const int* ctrls, const int* ctrl_vals);
/* 1 + the largest param_index pushed. */
int yao_circuit_nparams(const yao_circuit* c, int* out);

/* Forward and backward (a7, a8) ------------------------------------------------------- */

/* psi <- circuit(params) psi (apply!(reg, circuit)). */
int yao_forward(yao_state* s, const yao_circuit* c, const double* params);
/* expect'(H, reg => circuit): runs the circuit on s (which holds the input and ends
 * holding the output state), energy[b] = <psi_b|H|psi_b> and the gradient of every
 * parameter: grad[b * nparams + p] if reduce_batch == 0, else grad[p] summed over the
 * batch (the paper's batched gradient). If drift != NULL it receives
 * max |psi_0 uncomputed - psi_0| of the reversible sweep (REVERSIBLE and AUTO, also when AUTO
 * fell back) or 0 (CHECKPOINT). Synchronises. */
int yao_backward(yao_state* s, const yao_circuit* c, const double* params, const yao_pauli_sum* h,
                 enum yao_grad_mode mode, int reduce_batch, double* energy, double* grad, double* drift);

/* Number of YAO_GRAD_AUTO backward calls since the library loaded whose reversible sweep
 * drifted past drift_tol and fell back to the checkpointed sweep (process-wide). */
int yao_auto_fallbacks(long* count);

/* Batches of independent circuits (a9) --------------------------------------------------- */

/* Energy and gradient of ncirc independent circuits, each on its own single-slot state
 * (n may differ between circuits) starting from |0...0>; energy[c] and grad[c] (length
 * nparams of circuit c) are host arrays. Every state must have batch 1, at least 5 qubits
 * and the dtype of states[0]. The first call with a given list of circuits, states and
 * observables records the whole batch (resets, forward sweeps, H psi, reverse sweeps and
 * gradient sums of every circuit, spread over several streams) into one HIP graph; calls
 * with the same lists upload the new parameters in one copy and replay that graph. A
 * circuit changed by yao_circuit_push since is recorded anew. states[c] ends holding
 * circuit c's output state. The graph is replayed on the bound stream. Synchronises. */
int yao_batch_run(int ncirc, yao_state* const* states, const yao_circuit* const* circs,
                  const double* const* params, const yao_pauli_sum* const* h, double* energy,
                  double* const* grad);

/* Profiling ---------------------------------------------------------------------------- */

/* Kernel families whose launches the profiler can time. */
enum yao_kernel_family {
    YAO_KF_GATE = 0,      /* per-gate forward kernels */
    YAO_KF_ADJOINT = 1,   /* per-gate reverse-sweep kernels */
    YAO_KF_PASS_FWD = 2,  /* fused forward tile passes */
    YAO_KF_PASS_BWD = 3,  /* fused reverse-sweep tile passes */
    YAO_KF_EXPECT = 4,    /* Pauli-sum expectation */
    YAO_KF_HPSI = 5,      /* H psi (adjoint seed) */
    YAO_KF_MFMA = 6,      /* dense 4/5-qubit blocks on matrix cores */
    YAO_KF_BATCH = 7,     /* persistent batch kernel */
    YAO_KF_PERMUTE = 8,   /* qubit permutations (focus! / relax!) */
    YAO_KF_QFT = 9,       /* QFT passes */
    YAO_KF_MEASURE = 10,  /* outcome probabilities, cumulative sums, sampling, collapse */
    YAO_KF_KRYLOV = 11,   /* vector updates of the Krylov time evolution */
    YAO_KF_COUNT = 12
};
/* on = 1 clears earlier records and starts bracketing every launch with a pair of HIP
 * events on the bound stream; on = 0 stops. */
int yao_profile_enable(int on);
/* Totals for one family since profiling was enabled: number of launches, summed GPU time
 * between each launch's events (ms), and the algorithmic bytes and flops those launches
 * were credited with (bytes: each state element read or written once per launch; flops:
 * real arithmetic of the gate applications). Synchronises. */
int yao_profile_read(int family, int* launches, double* total_ms, double* algo_bytes, double* algo_flops);

/* Planner check (host only) ----------------------------------------------------------- */

/* Runs the pass plan of circuit c (forward, or the reverse sweep U^dagger in reverse gate order
 * when reverse = 1) for a state of dtype dt and batch 1 over tiles of tile_qubits qubits (0:
 * default) on the host, the way the pass kernels run it: tiles gathered from the index bits
 * the plan's qubit layout gives each pass, every op applied from its device record on tile
 * bits, tiles stored back through the pass's bit permutation. The start state is a seeded
 * Gaussian vector; *max_err receives the largest amplitude difference from applying the
 * gates one by one (Sec. "Representing Quantum Circuits": the chain as matrix product) and
 * *npasses the number of passes. params: nparams host doubles (or null when there are none).
 * At most 20 qubits; no GPU is used. */
int yao_plan_selfcheck(const yao_circuit* c, const double* params, enum yao_dtype dt, int reverse, int tile_qubits,
                       double* max_err, int* npasses);
/* Generates the run-time compiled forward passes (reverse = 0) or reverse-sweep passes with
 * gradients (reverse = 1; see yao_options.jit) of circuit c, held as a device-bound program of
 * a single-slot state of dtype dt over tiles of tile_qubits qubits (0: default), and compiles
 * them for gfx950 with hipRTC, without loading them (no GPU is used).
 * *npasses receives the plan's pass count and *njit how many of them compile to straight-line
 * kernels. Errors: YAO_EINVAL when c cannot be bound on the device or is too small for tile
 * passes; YAO_EHIP with the compiler log when the generated source does not compile. */
int yao_jit_selfcheck(const yao_circuit* c, enum yao_dtype dt, int reverse, int tile_qubits, int* npasses,
                      int* njit);
/* Counters of the run-time compiled passes since the library was loaded, into out[0 .. 4]:
 * programs compiled, passes compiled, programs whose compile or load failed (they keep the
 * generic kernels; the reason is printed once to stderr), launches of compiled forward passes
 * and launches of compiled reverse passes. */
int yao_jit_stats(long long* out);

#ifdef __cplusplus
}
#endif

#endif /* YAO_C_ABI_H_ */
