// Host runtime of the gfx950 state-vector library: errors, stream, workspace, gate matrices
// and the launchers of every kernel family.
#pragma once

#include "common.h"

namespace yao {

// ---------------------------------------------------------------------------- errors
int set_error(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
#define YAO_HIP(call)                                   \
    do {                                                \
        hipError_t _e = (call);                         \
        if (_e != hipSuccess) return hip_fail(_e, #call); \
    } while (0)
#define YAO_TRY(call)          \
    do {                       \
        int _r = (call);       \
        if (_r != 0) return _r; \
    } while (0)

hipStream_t stream();
const yao_options& options();
int ensure_device();

// ---------------------------------------------------------------------------- workspace
// Named device scratch slots that grow on demand and live until the library unloads.
enum WsSlot {
    WS_PSI0 = 0,    // copy of the input state (drift check)
    WS_PSI64,       // complex128 state of the backward sweep
    WS_LAM,         // adjoint state
    WS_PARTIAL,     // per-block partial sums
    WS_PARTIAL2,    // second-level sums
    WS_MAT,         // gate matrices and pass programs (forward sweeps)
    WS_MAT2,        // pass programs of reverse sweeps
    WS_CKPT,        // checkpoints
    WS_SEG,         // segment states of the checkpointed backward
    WS_TUNE,        // copy of a state while schedules are timed on it
    WS_PARAMS,      // circuit parameters for the device-side binding of programs
    WS_MISC,
    WS_PERM,        // out-of-place target of an in-place qubit permutation
    WS_MEAS,        // outcome probabilities, cumulative sums and sampled outcomes
    WS_KRYLOV,      // Krylov vectors of the time evolution
    WS_SHIFT,       // the shifted-circuit register of the faithful gradient
    WS_QFTTW,       // the QFT's table of roots of unity (filled once)
    WS_COUNT
};
void* workspace(int slot, size_t bytes);
// Pinned host staging buffer for results (grows on demand).
void* host_staging(size_t bytes);
// Pinned host buffer per workspace slot, for uploads that must not block the host (grows on
// demand; growing first waits for the stream, so no queued copy still reads the old one).
void* pinned(int slot, size_t bytes);
// Copy a small host block (<= 64 KiB) into the next slot of a device ring and return the slot.
// The copy is queued on the current stream, so kernels queued after it see the data; slots
// are reused round-robin after 256 uploads.
// Refused (YAO_EINVAL) while set_recording(true) is in force: launches recorded into a graph
// take their constants by value or from buffers that the graph owns.
void* ring_upload(const void* host, size_t bytes);
void set_recording(bool on);
bool recording();
// Copy a host block into workspace slot `slot` (grown as needed), ordered on the stream.
void* upload_to(int slot, const void* host, size_t bytes);

// ---------------------------------------------------------------------------- matrices
// A dense 2^k x 2^k complex matrix in FP64, row-major; row/col bit j <-> locs[j].
struct HostMat {
    int k = 0;
    std::vector<double> re, im;
    int dim() const { return 1 << k; }
    void resize(int kk)
    {
        k = kk;
        re.assign(size_t(1) << (2 * k), 0.0);
        im.assign(size_t(1) << (2 * k), 0.0);
    }
};
bool is_param_kind(int kind);
// U(theta) of a gate; returns false on an unknown kind.
bool gate_matrix(const GateRec& g, double theta, HostMat& U);
// (dU/dtheta) U^dagger, so that dE/dtheta = 2 Re <lambda_{k+1}| M |psi_{k+1}> on the gate's
// controlled subspace.
bool gate_grad_matrix(const GateRec& g, double theta, HostMat& M);
HostMat dagger(const HostMat& U);
void dagger_into(const HostMat& U, HostMat& D);
HostMat matmul(const HostMat& A, const HostMat& B);

// Matrix classes that pick a kernel specialisation (App. "sparse matrices": diagonal,
// permutation-with-phases, dense).
enum MatClass { MC_DENSE = 0, MC_DIAG = 1, MC_DIAG1 = 2, MC_ANTI = 3 };
int classify(const HostMat& U);

// ---------------------------------------------------------------------------- launchers
struct CtrlSpec {
    uint64_t mask = 0, val = 0;
};
CtrlSpec make_ctrl(int nctrl, const int* ctrls, const int* cvals);

int launch_reset(yao_state* s);
// |0...0> into nz single-slot states of n qubits (device array of their data pointers), and
// those states widened to complex128 into dst (nz consecutive blocks of 2^n elements).
int launch_fill_basis_z(void* const* ptrs, int nz, int dtype, int n);
int launch_convert_z(const void* const* src, int nz, int dtype, double* dst, int n);
int launch_fill_basis(void* data, int dtype, int n, int B);
// One gate on a state of either precision (per-gate form).
// k >= 2 matrices come from dev_mat (re block then im block, rounded to the state's real
// type) or, when dev_mat is null, from a ring upload.
int launch_gate(void* data, int dtype, int n, int B, const HostMat& U, const int* locs, CtrlSpec c,
                const void* dev_mat = nullptr);
// Device form of a k >= 2 matrix as launch_gate reads it from dev_mat for this state (the FP32
// real form of the matrix-core path, else re block then im block in the state's real type),
// appended to pool (8-byte words); returns its offset in words.
size_t encode_gate_matrix(int dtype, int n, int B, const HostMat& U, std::vector<double>& pool);
// energy[b] (host) = Re <psi|H|psi>.
int launch_expect(const void* data, int dtype, int n, int B, yao_pauli_sum* h, double* energy_host);
// out = H psi; energy[b] (host, may be null) from the same pass. out_dtype may differ.
int launch_hpsi(const void* data, int dtype, void* out, int out_dtype, int n, int B, yao_pauli_sum* h,
                double* energy_host);
// The same with the energy left on the device and no synchronisation (graph-capturable).
// Doubles of partials that launch_hpsi_dev needs for this observable and state shape (builds
// the observable's pass tables on first use; call it outside graph capture).
size_t hpsi_partial_doubles(const yao_pauli_sum* h, int n, int B, int dtype);
// Observables in tile passes (states of >= 5 qubits): H psi into out (nullptr: energy only),
// energy partials partial[b * W + column].
bool obs_passes_ok(const yao_pauli_sum* h, int n, int B, int dtype);
size_t obs_partial_doubles(const yao_pauli_sum* h, int n, int B, int dtype);
// Qubits of each observable pass's tile (the non-tile qubits index the tiles, ascending).
int obs_tile_qubits(const yao_pauli_sum* h, int n, int B, int dtype);
int launch_obs_passes(const void* psi, int dtype, void* out, int out_dtype, int n, int B, const yao_pauli_sum* h,
                      double* partial, int* W);
void drop_obs_plans(const yao_pauli_sum* h);
int launch_hpsi_dev(const void* data, int dtype, void* out, int out_dtype, int n, int B, const yao_pauli_sum* h,
                    double* partial, double* energy_dev);
// Precision conversion / copies between states of equal shape.
int launch_convert(const void* src, int src_dtype, void* dst, int dst_dtype, size_t elems);
// <a_b|b_b> per batch slot (host results), FP64 accumulation.
int launch_inner(const void* a, int a_dtype, const void* b, int b_dtype, int n, int B, double* re, double* im);
// max |a - b| over the elements (host result).
int launch_maxdiff(const void* a, int a_dtype, const void* b, int b_dtype, size_t elems, double* out);

// One reverse step of the per-gate backward: grad partials of gate g (if M != null) with
// psi_{k+1}, lambda_{k+1}, then psi <- Ud psi, lambda <- Ud lambda. psi is complex128,
// lambda is lam_dtype. partial receives [B][nblk] doubles; nblk is returned via *nblk.
// k >= 2 matrices come from dev_mats (Ud re, Ud im, M re, M im; 4^k doubles each) or a ring upload.
int launch_adjoint_step(double* psi, void* lam, int lam_dtype, int n, int B, const HostMat& Ud, const HostMat* M,
                        const int* locs, CtrlSpec c, const double* dev_mats, double* partial, int* nblk);
int adjoint_nblk(int n, int k, int B);
// The same with the per-slot partial rows pstride apart (pstride >= the launch's block count).
int launch_adjoint_step_strided(double* psi, void* lam, int lam_dtype, int n, int B, const HostMat& Ud,
                                const HostMat* M, const int* locs, CtrlSpec c, const double* dev_mats, double* partial,
                                int pstride);
// sums[r] = sum_j partial[r * nblk + j] for r < rows (device), sequential per row.
int launch_row_sums(const double* partial, int rows, int nblk, double* sums);

// Pauli tables
// Device tables of a Pauli sum (pauli_upload): terms grouped by X mask x. Term t of a group
// adds c_t i^{ny} (-1)^{|(j ^ x) & z|} psi[j ^ x] to (H psi)[j].
struct PGroup {
    uint64_t x;
    int t0, t1;
};
struct PTerm {
    double c;
    uint64_t z;
    int ny;
    int pad;
};
// Group the terms by X mask into h->host_groups / h->host_terms (PGroup / PTerm records).
void pauli_group_host(yao_pauli_sum* h);
int pauli_upload(yao_pauli_sum* h);
// Expectation through the one-read-per-X-mask-group kernel into caller-given device buffers:
// groups / terms hold the PGroup / PTerm tables, partial B * expect_grid_x(n, B) doubles,
// sums[b] receives the energy of slot b. Nothing is allocated and nothing synchronises.
int expect_grid_x(int n, int B);
int launch_expect_into(const void* data, int dtype, int n, int B, const void* groups, int ngroups, const void* terms,
                       double* partial, double* sums);

// Qubit permutation (qubit q -> index bit perm[q]) from in to out (distinct buffers), and the
// QFT (or its inverse) on the qubits locs in place (kernels_qubits.hip). Batch * element bytes
// must stay <= 16 KiB.
int launch_permute(const void* in, void* out, int dtype, int n, int B, const int* perm);
int launch_qft(void* data, int dtype, int n, int B, const int* locs, int k, bool inverse);
int qft_passes(int dtype, int n, int B, const int* locs, int k);

// Faithful gradient by the shift rule, every shifted circuit in one register (shift.hip):
// energy (host, 1 value) and grad (host, c->nparams values) of the batch-1 state st.
int shift_grad(const yao_state* st, const yao_circuit* c, const double* params, yao_pauli_sum* h, double* energy,
               double* grad);
// psi <- exp(-i H t) psi per slot by the Lanczos method (krylov.hip); nsteps: substeps taken.
int time_evolve(yao_state* s, yao_pauli_sum* h, double t, double tol, int krylov_dim, int* nsteps);

// Measurement (kernels_measure.hip). prob: B * 2^k doubles [b][x]; launch_cdf scans p into q
// per chunk of 2048 outcomes and writes the chunks' exclusive offsets to tot
// (cdf_tot_doubles(k, B)); launch_sample draws nshots outcomes per slot from u (device,
// [B][nshots]) with q and tot as launch_cdf left them; launch_collapse projects s onto the outcomes x (device, [B]) and writes dep, scale
// and prob (device, B each). locs_dev: the k locs in device memory.
int launch_outcome_probs(const yao_state* s, const int* locs, int k, double* prob);
int launch_cdf(const double* p, double* q, int k, int B, double* tot);
size_t cdf_tot_doubles(int k, int B);
int launch_sample(const double* cdf, const double* tot, int k, int B, int nshots, const double* u, uint64_t* out);
int launch_collapse(yao_state* s, const double* probs, const int* locs_dev, const int* locs, int k, const uint64_t* x,
                    uint64_t* dep, double* scale, double* prob);

// Dense 4/5-qubit gates on complex64 states through the FP32 matrix cores.
bool mfma_supported(int k, int n, int B);
void mfma_encode(const HostMat& U, float* out);  // 3 * 4^k floats
int launch_dense_mfma(float2* psi, int n, int B, const HostMat& U, const int* locs, CtrlSpec c,
                      const void* dev_mat = nullptr);

// ---------------------------------------------------------------------------- profiler
// prof_begin records a start event for a launch of `family` when profiling is on (returns
// -1 otherwise); prof_end records the matching end event and credits bytes / flops.
int prof_begin(int family);
void prof_end(int idx, double bytes, double flops);
int prof_enable(bool on);
// While suspended (graph capture), prof_begin records nothing.
void prof_suspend(bool on);
int prof_read(int family, int* launches, double* total_ms, double* bytes, double* flops);

}  // namespace yao
