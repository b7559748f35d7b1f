// Fused tile passes: a pass loads a tile of 2^t elements (c batch bits and t-c chosen
// qubits) into LDS, applies every gate whose targets lie in the tile -- in register groups of
// 3 or 4 tile bits per thread -- and writes the tile back. Controls outside the tile are
// constant over a tile and become a per-tile predicate.
#pragma once

#include "runtime.h"

namespace yao {

constexpr int kRegBitsFwd = 4;    // register bits per group in the forward: 16 elements per thread
constexpr int kRegBitsBwd = 3;    // backward: 8 elements of psi and 8 of lambda per thread
constexpr int kMaxRegBits = 4;
constexpr int kMaxTileBits = 13;  // 2^13 complex64 = 64 KiB of LDS
constexpr int kMaxFusedK = 3;     // reverse passes: wider gates run as standalone launches
constexpr int kMaxDenseK = 4;     // forward passes: gates up to 4 qubits as dense register blocks
constexpr int kMaxGroupSlots = 32;  // gradient-carrying gates per register group (at most)
constexpr int kMaxPassOps = 4096;   // op records of a pass (read in place through the scalar cache)
constexpr int kMaxPassDense = 8;    // dense blocks of a forward pass (their matrices are staged too)

// Entries of gradient partials per register group of a reverse pass: one per 16-lane row and
// batch slot of the tile (row sums), or one per thread in tiles of fewer than 16 threads.
__host__ __device__ __forceinline__ int grad_entries(int nthr, int c)
{
    return nthr >= 16 ? (nthr >> 4) << c : nthr;
}

// Gradient-carrying ops per register group of a reverse pass, so that the two partial buffers
// fit in the LDS a tile of 2^t elements of psi (FP64) and lambda (lam_bytes each) leaves.
inline int reverse_slot_limit(int t, int c, int lam_bytes)
{
    const long avail = 160L * 1024 - ((long)(16 + lam_bytes) << t);
    const long per = 2L * (long)sizeof(double) * grad_entries(1 << (t - kRegBitsBwd), c);
    const long s = avail > 0 ? avail / per : 0;
    return (int)(s < 1 ? 1 : (s > kMaxGroupSlots ? kMaxGroupSlots : s));
}

// Structure classes of a one-qubit matrix inside a pass.
enum OpType : int {
    OT_SWAP = 0,   // X
    OT_DIAG = 1,   // diag(d0, d1)
    OT_REAL = 2,   // every entry real (Ry, H)
    OT_RX = 3,     // [[c, -i s], [-i s, c]] with c, s real
    OT_DENSE = 4,
    OT_LDSK = 5    // k = 2 or 3 dense matrix applied in LDS
};

// Gradient generators: M = (dU/dtheta) U^dagger restricted to the op's subspace.
enum GenType : int { GEN_NONE = 0, GEN_X = 1, GEN_Y = 2, GEN_Z = 3, GEN_P1 = 4, GEN_DENSE = 5 };

// Code paths of one-qubit ops, chosen on the host: var = class * R + register position (R =
// register bits). Forward classes: 0 Rx-like, 1 diagonal, 2 dense (all without controls),
// 3 swap with controls inside the tile, 4 anything else. Reverse classes: 0 Rx-like with an
// X generator, 1 diagonal with a Z generator (both without controls, with a gradient),
// 2 swap with controls inside the tile and no gradient, 3 anything else.
constexpr int kFwdGenericClass = 4;
constexpr int kBwdGenericClass = 3;

// Device op record (one gate inside a pass), 128 bytes: everything a one-qubit op needs comes
// in one scalar fetch, so the next op's record can be fetched while the current one computes.
struct POp {
    int type;       // OpType
    int k;
    int gen;        // GenType (backward only)
    int rpos;       // register position (0..register bits - 1) of a one-qubit target
    int slot;       // gradient slot (-1 none)
    int mat;        // offset in doubles into the matrix pool: U (re, im) then M (re, im)
    uint32_t cmask, cval;  // controls on tile bits
    uint64_t omask, oval;  // controls on qubits outside the tile
    double u[8];    // one-qubit matrix (forward U, backward U^dagger): re[4] then im[4]; in
                    // forward programs of complex64 states the same entries as float[8]; for
                    // reverse ops of the Z-generator diagonal class (var / 3 == 1) entry 3
                    // holds d1 / d0 instead of d1 (split_diag_phase)
    int tpos[3];    // tile-bit positions of the targets of a k = 2, 3 op, in locs order
    int var;        // code path of a one-qubit op (see op_variant)
};
static_assert(sizeof(POp) == 128, "op record layout");

// diag(d0, d1) as d0 * diag(1, d1 / d0): entry 3 of u (re[4] then im[4]) becomes d1 / d0.
__host__ __device__ inline void split_diag_phase(double* u)
{
    const double n = u[0] * u[0] + u[4] * u[4];
    const double rr = (u[3] * u[0] + u[7] * u[4]) / n, ri = (u[7] * u[0] - u[3] * u[4]) / n;
    u[3] = rr;
    u[7] = ri;
}

struct PGroupDesc {
    int rpos[kMaxRegBits];  // tile-bit positions of the register bits, ascending
    int lds;             // 1: a single OT_LDSK op applied in LDS; 2: a single dense block, a
                         // 16 x 16 matrix on the register bits (index bit j <-> rpos[j])
    int op0, nops;
    int nslot;           // ops with a gradient in this group
    int slots[kMaxGroupSlots];  // their gradient slots, in op order
};

struct PassDesc {
    int group0, ngroups;
    int standalone;      // >= 0: a gate applied by its own launch (k > kMaxFusedK)
    int tile_qubits[kMaxTileBits];
    int ntq;             // number of tile qubits (t - c)
};

// Host plan of one direction of one circuit.
struct HostOp {
    int gate;            // index into the circuit
    uint64_t tmask, qmask;
};
struct HostGroup {
    std::vector<int> ops;   // indices into plan ops
    uint64_t rbits = 0;     // register tile-bit mask
    bool lds = false;       // one k = 2, 3 gate applied in LDS (reverse passes)
    bool dense = false;     // one k = 2..4 gate as a 16 x 16 matrix on the register bits (forward)
};
// Qubit layout: inside a plan the state may be held with its qubits permuted, qubit q at
// amplitude-index bit phys[q]. A pass loads its tile from the index bits tile_qubits and may
// store it back permuted among those same bits (store_src), which lets the next pass find the
// qubits it needs on the low, contiguous index bits. Every plan starts and ends with qubit q
// on bit q.
struct HostPass {
    std::vector<int> tile_qubits;   // index bits of the tile, ascending
    std::vector<HostGroup> groups;
    int standalone = -1;            // op index for a standalone launch
    std::vector<int> phys;          // layout at the start of the pass (empty: identity)
    std::vector<int> store_src;     // t entries: tile bit i of the stored tile comes from tile
                                    // bit store_src[i] of the tile in LDS (empty: identity)
};
struct Plan {
    int n = 0, B = 1, c = 0, t = 0;
    int reg_bits = kRegBitsFwd;
    int g0 = 0, g1 = 0;  // gate range
    bool reverse = false;
    bool valid = true;   // false: the layout could not be put back (never expected)
    int max_slots = kMaxGroupSlots;  // gradient-carrying ops per register group
    std::vector<HostOp> ops;        // in application order (reverse order of gates if reverse)
    std::vector<HostPass> passes;
};

// Build the pass structure of gates [g0, g1); taken in circuit order, or reversed for the
// backward.
// max_ops: at most that many ops per pass.
// max_slots: at most that many gradient-carrying ops per register group.
Plan make_plan(const yao_circuit* c, int g0, int g1, int B, int t, int cbits, int low_fixed, bool reverse,
               int reg_bits, int max_ops = kMaxPassOps, int max_slots = kMaxGroupSlots);
// Choose tile geometry for a state (tile qubits from the options, 0 = default).
void tile_geometry(int n, int B, int dtype, bool backward, int* t, int* cbits, int* low_fixed);
// The same for an explicit number of tile qubits (<= 0: default).
void tile_geometry_tq(int n, int B, int dtype, bool backward, int tq, int* t, int* cbits, int* low_fixed);

// Parameter binding on the device: op record `op` (index in the program's records) takes the
// one-qubit matrix U = U_{nf-1} ... U_0 of factors f0 .. f0 + nf - 1, each a gate kind with
// its angle from params[param] (param >= 0) or theta. mode 0: U as float[8] (forward,
// complex64), 1: U as double[8] (forward, complex128), 2: U^dagger as double[8] (reverse).
struct BindRec {
    int op, f0, nf, mode;
};
struct BindFac {
    int kind, param;
    double theta;
};
static_assert(sizeof(BindRec) == 16 && sizeof(BindFac) == 16, "bind table layout");

// Device program of one plan for given parameters (built on the host, copied in one block).
struct Program {
    std::vector<POp> ops;
    std::vector<PGroupDesc> groups;
    std::vector<double> mats;
    std::vector<int> pass_group0;   // per pass
    std::vector<int> pass_op0;      // first op record of the pass; group op0 is relative to it
    std::vector<int> pass_nops;
    std::vector<double> pass_flops; // algorithmic flops per element of the state, per pass
    std::vector<int> pass_mat;      // standalone passes: offset in doubles of their matrices in mats
    std::vector<int> pass_dmat0;    // first double of the pass's dense block matrices in mats
    std::vector<int> pass_dmat_words;  // their size in 16-byte words (0: none)
    std::vector<int> slot_of_gate;  // gradient slot per gate (-1)
    int nslots = 0;
    // Built without parameters: the matrices that depend on them are left to k_bind.
    std::vector<BindRec> binds;
    std::vector<BindFac> facs;
    bool bindable = true;  // false: some parameter-dependent matrix cannot be bound on the device
};
struct DevProgram {
    POp* ops;
    PGroupDesc* groups;
    double* mats;
};
// One circuit of a launch over several circuits of one structure (grid z): its state (psi),
// adjoint state or H psi output (lam), program records (ops: the program's first record; the
// pass's offset is added by the kernel) and partial sums.
struct ZSlot {
    void* psi;
    void* lam;
    const POp* ops;
    double* partial;
};
// While set (nz > 0), pass and observable launches run over the nz circuits of zs (device
// memory) instead of their own pointers; the rest of a launch (plan, groups, matrices, tiles)
// is shared. launch_hpsi_dev then also sums the energies of all nz circuits (partials nz * B
// rows apart by the observable's partial size, energies to consecutive entries).
void set_zbatch(const ZSlot* zs, int nz);
const ZSlot* zbatch_slots();
int zbatch_count();
// lam_bytes: bytes per element of the adjoint state (reverse plans size their register groups'
// gradient buffers by it).
const Plan& get_plan(const yao_circuit* c, int g0, int g1, int B, int t, int cb, int L, bool reverse,
                     int lam_bytes = 16);
// A plan with the given register bits, pass size and group slots (cached like get_plan's).
const Plan& get_plan_ex(const yao_circuit* c, int g0, int g1, int B, int t, int cb, int L, bool reverse, int reg_bits,
                        int max_ops, int max_slots = kMaxGroupSlots);
// dtype: the state's (forward) or the adjoint state's (backward) precision. With params null
// the program is built for binding on the device (Program::binds); when c is the structure of a
// fused circuit (fused_shape), parts and orig describe its multi-gate placeholders.
struct FusedPart;
int build_program(const Plan& P, const yao_circuit* c, const double* params, bool bwd, int dtype, Program& prog,
                  const std::vector<FusedPart>* parts = nullptr, const yao_circuit* orig = nullptr);
// Fill the bound matrices of a device program (see BindRec) for the device array params.
int launch_bind(POp* ops, const BindRec* binds, int nbinds, const BindFac* facs, const double* params);
size_t program_blob_bytes(const Program& prog);
void pack_program(const Program& prog, char* host, char* dev, DevProgram& d);
// Launch the passes of a plan whose program is already in device memory (no host sync, no
// copies: capturable in a graph). bp: the bound program prog belongs to, whose run-time
// compiled passes (if any) are used.
struct BoundProgram;
int launch_forward_passes(const Plan& P, const Program& prog, const DevProgram& d, void* data, int dtype, int n, int B,
                          const yao_circuit* c, const double* params, const BoundProgram* bp = nullptr);
int launch_backward_passes(const Plan& P, const Program& prog, const DevProgram& d, const yao_circuit* c,
                           const double* params, double* psi, void* lam, int lam_dtype, int n, int B, double* gpartial,
                           int W, const BoundProgram* bp = nullptr);

// Drivers.
int forward_fused(void* data, int dtype, int n, int B, const yao_circuit* c, const double* params);
// Forward sweep at fusion width `width` (0: none) over tiles of tq qubits (<= 0: default);
// dparams: c's parameters already on the device, or null.
int forward_sweep(void* data, int dtype, int n, int B, const yao_circuit* c, const double* params, int width, int tq,
                  const double* dparams);
// Device-bound programs (built once per plan; see BindRec).
// One circuit of a batch whose whole state fits one tile, run start to end by one workgroup
// (k_small_circuit): forward program, then H psi and the energy, then the reverse program
// with its gradients. Both programs are one pass over the tile holding qubits 0 .. n-1 in
// order, with 3 register bits and FP64 matrices.
struct SmallCircuit {
    const POp* fops;
    const PGroupDesc* fgroups;
    const double* fmats;
    const POp* rops;
    const PGroupDesc* rgroups;
    const double* rmats;
    const PGroup* hgroups;
    const PTerm* hterms;
    void* state;     // psi_N is written here (complex64 or complex128)
    double* energy;  // <psi_N|H|psi_N>
    double* grad;    // one value per gradient slot of the reverse program
    int nfg, nrg, nhg, n;
    int c64;         // state precision: 1 complex64, 0 complex128
    int pad[3];
};
// One program to bind (k_bind over its records) in a launch that binds many.
struct BindJob {
    POp* ops;
    const BindRec* binds;
    const BindFac* facs;
    const double* params;
    int nb, pad;
};
int launch_bind_jobs(const BindJob* jobs, int njobs, int max_nb);
// count circuits of n qubits each, one workgroup apiece.
int launch_small_circuits(const SmallCircuit* items, int count, int n);
constexpr int kSmallMaxQubits = 12;  // psi and lambda in FP64: 32 B x 2^12 = 128 KiB of LDS

struct JitPasses;
struct BoundProgram {
    const yao_circuit* circ = nullptr;
    Program prog;
    char* dev = nullptr;
    DevProgram d{};
    BindRec* dbinds = nullptr;
    BindFac* dfacs = nullptr;
    bool ok = false;  // false: the program needs the host for some matrix
    // Run-time compiled passes (jit.cpp): uses so far, the module once compiled, and whether
    // compiling failed (then the generic kernels for good).
    mutable int uses = 0;
    mutable JitPasses* jit = nullptr;
    mutable bool jit_failed = false;
};
// The run-time compiled passes of a bound program (compiled on its options().jit-th use),
// or nullptr. jit_has: pass p has a compiled kernel. jit_launch_forward runs it on psi with
// the program's records (op_first: the pass's first record), over the current z batch.
const JitPasses* jit_passes(const BoundProgram* bp, const Plan& P, bool bwd, int dtype, int n, int B);
bool jit_has(const JitPasses* J, int p);
int jit_launch_forward(const JitPasses* J, int p, void* psi, const POp* ops, int op_first, double bytes,
                       double flops);
void jit_free(JitPasses* J);
// Programs compiled, passes compiled, programs that failed to compile or load, launches of
// compiled forward passes, of compiled reverse passes.
void jit_stats(long long* out);
// Host only: generate and compile (no module load) the run-time forward (or reverse) passes of
// circuit c as a bound program; *njit of *npasses passes are compiled.
int jit_selfcheck(const yao_circuit* c, int dtype, int reverse, int tile_qubits, int* npasses, int* njit);
int jit_launch_backward(const JitPasses* J, int p, double* psi, void* lam, const POp* ops, int op_first,
                        const double* mats, double* gpartial, int pstride, double bytes, double flops);
// Nested: while any suspension is active nothing is compiled (autotuner trials).
void jit_suspend(bool on);
const BoundProgram* bound_program(const Plan& P, const yao_circuit* c, bool bwd, int dtype,
                                  const std::vector<FusedPart>* parts, const yao_circuit* orig);
const double* upload_params(const double* params, int nparams);
int bind_program(const BoundProgram* b, const double* dparams);
void drop_bound(const yao_circuit* c);
// Gates [g0, g1) only.
int forward_fused_range(void* data, int dtype, int n, int B, const yao_circuit* c, const double* params, int g0,
                        int g1);
int backward_fused(yao_state* s, const yao_circuit* c, const double* params, yao_pauli_sum* h, int mode,
                   bool reduce_batch, double* energy, double* grad, double* drift);
// AUTO sweeps that fell back to the checkpointed form since the library loaded.
long auto_fallbacks();
// Tiles need more qubits than register bits.
bool fused_supported(int n, int B);

}  // namespace yao
