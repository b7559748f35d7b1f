// Fused tile-pass kernels: forward sweep and reversible adjoint sweep.
//
// One workgroup owns one tile: 2^t elements = Bc = 2^c consecutive batch slots (lowest tile
// bits) x the 2^(t-c) amplitudes spanned by the pass's tile qubits, with every other qubit
// fixed by the tile id. The tile is staged in LDS (XOR-swizzled), then processed in register
// groups: each of the 2^(t-RB) threads holds the 2^RB elements that differ only in the
// group's RB register bits, so a one-qubit gate on a register bit is pure ALU work on pairs of
// registers. Gates of 2 or 3 qubits are applied directly in LDS. The backward kernel holds psi
// (complex128: the FP64 uncompute) and lambda (widened to FP64 in registers) and, per gate,
// first adds 2 Re <lambda|M|psi> over the tile (eq. outer-product reduced to the parameter),
// then applies U^dagger to both (eq. apply-back). Per-thread gradient partials go to LDS and
// are reduced once per register group, in a fixed order.
//
// The pass's op records are copied to LDS together with the tile; LDS reads complete in
// order, so the record of the next op is fetched while the current op computes.
#include <algorithm>
#include <map>
#include <tuple>
#include <mutex>
#include <vector>

#include "fused.h"

namespace yao {

namespace {
struct ZBatch {
    const ZSlot* zs = nullptr;
    int nz = 0;
};
ZBatch g_zbatch;
}  // namespace

void set_zbatch(const ZSlot* zs, int nz)
{
    g_zbatch.zs = nz > 0 ? zs : nullptr;
    g_zbatch.nz = nz > 0 ? nz : 0;
}

int zbatch_count()
{
    return g_zbatch.zs ? g_zbatch.nz : 1;
}

const ZSlot* zbatch_slots()
{
    return g_zbatch.zs;
}

namespace {

struct PassArgs {
    void* psi;
    void* lam;
    const POp* ops;         // the pass's records: ops[0 .. nops)
    const PGroupDesc* groups;  // the pass's groups: groups[0 .. ngroups), op0 relative to ops
    const double* mats;
    double* gpartial;       // [slot][B][pstride]
    int n, B, c, t;
    int ngroups, nops;
    int ntq, nnt;
    int ntiles;
    int pstride;
    int tile_qubits[kMaxTileBits];
    int nontile_qubits[40];
    uint64_t rofs[1 << kMaxRegBits];  // element offset (x B) of load register r from the thread's first
    const uint4* dmats;     // the pass's dense block matrices (forward), staged in LDS
    int ndm;                // their size in 16-byte words
    // Store permutation: stored tile element e = th + r * nthr comes from LDS tile element
    // store_thread_bits(th) | sreg[r] (thread bit i of e moves to tile bit ssrc[i]).
    int ssrc[kMaxTileBits];
    uint32_t sreg[1 << kMaxRegBits];
    int mslots;             // reverse passes: gradient-carrying ops per register group (at most)
    // Launches over several circuits of one structure (grid z): circuit z's state, adjoint
    // state, records (ops: program base, plus op_first) and partial sums; null: one circuit.
    const ZSlot* zs;
    int op_first;
};

// The per-circuit pointers of a launch (the circuit's own, or its z slot's).
__device__ __forceinline__ void* z_psi(const PassArgs& a)
{
    return a.zs ? a.zs[blockIdx.z].psi : a.psi;
}
__device__ __forceinline__ void* z_lam(const PassArgs& a)
{
    return a.zs ? a.zs[blockIdx.z].lam : a.lam;
}
__device__ __forceinline__ const POp* z_ops(const PassArgs& a)
{
    return a.zs ? a.zs[blockIdx.z].ops + a.op_first : a.ops;
}
__device__ __forceinline__ double* z_partial(const PassArgs& a, double* p)
{
    return a.zs ? a.zs[blockIdx.z].partial : p;
}

__device__ __forceinline__ uint32_t swz(uint32_t e)
{
    return e ^ (((e >> 4) ^ (e >> 8)) & 15u);
}

template <typename V, typename RR> __device__ __forceinline__ V mkv(RR a, RR b)
{
    V v;
    v.x = a;
    v.y = b;
    return v;
}

__device__ __forceinline__ int sc(int v)
{
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ uint64_t sc64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Control fields of an op record, made wave-uniform (scalar registers).
struct OpCtl {
    int type, gen, rpos, slot, mat, var;
    uint32_t cmask, cval;
    uint64_t omask, oval;
};
// Control fields and the one-qubit matrix of an op, wave-uniform. The matrix is read in the
// precision MR: the host stores float entries (u viewed as float[8]) in programs for complex64
// forward sweeps, double entries otherwise.
template <typename MR> struct OpS {
    OpCtl c;
    MR m[8];  // re[4], im[4]
};
// Op records and group descriptors are read in place through the scalar cache: a pointer in
// the constant address space tells the compiler that the kernel never writes them, so
// wave-uniform reads become scalar loads straight into SGPRs (the records are written by the
// host or by the bind kernel before the pass is launched).
#define YAO_CONST __attribute__((address_space(4)))
template <typename T> __device__ __forceinline__ const YAO_CONST T* cptr(const T* p)
{
    return (const YAO_CONST T*)p;
}
__device__ __forceinline__ OpCtl op_ctl_c(const YAO_CONST POp* r)
{
    OpCtl o;
    o.type = r->type;
    o.gen = r->gen;
    o.rpos = r->rpos;
    o.slot = r->slot;
    o.mat = r->mat;
    o.var = r->var;
    o.cmask = r->cmask;
    o.cval = r->cval;
    o.omask = r->omask;
    o.oval = r->oval;
    return o;
}
template <typename MR> __device__ __forceinline__ OpS<MR> load_op_c(const YAO_CONST POp* r)
{
    OpS<MR> o;
    o.c = op_ctl_c(r);
    if constexpr (sizeof(MR) == 4) {
        const YAO_CONST float* f = (const YAO_CONST float*)r->u;
#pragma unroll
        for (int q = 0; q < 8; ++q) o.m[q] = f[q];
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) o.m[q] = r->u[q];
    }
    return o;
}

__device__ __forceinline__ void fold_outer_controls(OpCtl& c, uint64_t base)
{
    if ((base & c.omask) != c.oval) {
        c.cmask = 0x80000000u;
        c.cval = 0x80000000u;
    }
}

// ------------------------------------------------------------------------------ in-place updates
// The common one-qubit updates are written as inline assembly whose results are tied to the
// registers of their inputs. A register group's amplitudes stay in fixed registers from op to
// op; computed as plain expressions, each op variant would leave its results in fresh
// registers and every op would end with a copy of all of them. Scalar operands are the op's
// matrix entries (SGPRs); each VALU instruction reads at most one of them.
#define YAO_IP_FNS(T, V, SFX, MOV)                                                                       \
    /* (a, b) <- (c a + i s b, i s a + c b) */                                                          \
    __device__ __forceinline__ void rx_ip(V& a, V& b, T cc, T ss)                                      \
    {                                                                                                   \
        T t0, t1;                                                                                       \
        asm("v_mul_" SFX " %[t0], %[s], %[by]\n\t"                                                    \
            "v_mul_" SFX " %[t1], %[s], %[ax]\n\t"                                                    \
            "v_fma_" SFX " %[ax], %[c], %[ax], -%[t0]\n\t"                                            \
            "v_fma_" SFX " %[by], %[c], %[by], %[t1]\n\t"                                             \
            "v_mul_" SFX " %[t0], %[s], %[bx]\n\t"                                                    \
            "v_mul_" SFX " %[t1], %[s], %[ay]\n\t"                                                    \
            "v_fma_" SFX " %[ay], %[c], %[ay], %[t0]\n\t"                                             \
            "v_fma_" SFX " %[bx], %[c], %[bx], -%[t1]"                                                  \
            : [ax] "+v"(a.x), [ay] "+v"(a.y), [bx] "+v"(b.x), [by] "+v"(b.y), [t0] "=&v"(t0),            \
              [t1] "=&v"(t1)                                                                            \
            : [c] "s"(cc), [s] "s"(ss));                                                                \
    }                                                                                                   \
    /* a <- (r + i m) a */                                                                              \
    __device__ __forceinline__ void diag_ip(V& a, T r, T m)                                            \
    {                                                                                                   \
        T t0, t1;                                                                                       \
        asm("v_mul_" SFX " %[t0], %[m], %[ay]\n\t"                                                    \
            "v_mul_" SFX " %[t1], %[m], %[ax]\n\t"                                                    \
            "v_fma_" SFX " %[ax], %[r], %[ax], -%[t0]\n\t"                                            \
            "v_fma_" SFX " %[ay], %[r], %[ay], %[t1]"                                                   \
            : [ax] "+v"(a.x), [ay] "+v"(a.y), [t0] "=&v"(t0), [t1] "=&v"(t1)                             \
            : [r] "s"(r), [m] "s"(m));                                                                  \
    }                                                                                                   \
    /* (a, b) <- U (a, b) for U = mr + i mi, row-major; four interleaved FMA chains, the last */  \
    /* of which ends in b.y itself */                                                                 \
    __device__ __forceinline__ void dense_ip(V& a, V& b, const T* mr, const T* mi)                     \
    {                                                                                                   \
        T t0, t1, t2, t3;                                                                               \
        asm("v_mul_" SFX " %[t0], %[r0], %[ax]\n\t"                                                   \
            "v_mul_" SFX " %[t1], %[r0], %[ay]\n\t"                                                   \
            "v_mul_" SFX " %[t2], %[r2], %[ax]\n\t"                                                   \
            "v_mul_" SFX " %[t3], %[r2], %[ay]\n\t"                                                   \
            "v_fma_" SFX " %[t0], -%[i0], %[ay], %[t0]\n\t"                                           \
            "v_fma_" SFX " %[t1], %[i0], %[ax], %[t1]\n\t"                                            \
            "v_fma_" SFX " %[t2], -%[i2], %[ay], %[t2]\n\t"                                           \
            "v_fma_" SFX " %[t3], %[i2], %[ax], %[t3]\n\t"                                            \
            "v_fma_" SFX " %[t0], %[r1], %[bx], %[t0]\n\t"                                            \
            "v_fma_" SFX " %[t1], %[i1], %[bx], %[t1]\n\t"                                            \
            "v_fma_" SFX " %[t2], %[r3], %[bx], %[t2]\n\t"                                            \
            "v_fma_" SFX " %[t3], %[i3], %[bx], %[t3]\n\t"                                            \
            "v_fma_" SFX " %[t0], -%[i1], %[by], %[t0]\n\t"                                           \
            "v_fma_" SFX " %[t1], %[r1], %[by], %[t1]\n\t"                                            \
            "v_fma_" SFX " %[t2], -%[i3], %[by], %[t2]\n\t"                                           \
            "v_fma_" SFX " %[by], %[r3], %[by], %[t3]\n\t"                                            \
            MOV " %[ax], %[t0]\n\t"                                                                   \
            MOV " %[ay], %[t1]\n\t"                                                                   \
            MOV " %[bx], %[t2]"                                                                         \
            : [ax] "+v"(a.x), [ay] "+v"(a.y), [bx] "+v"(b.x), [by] "+v"(b.y), [t0] "=&v"(t0),            \
              [t1] "=&v"(t1), [t2] "=&v"(t2), [t3] "=&v"(t3)                                            \
            : [r0] "s"(mr[0]), [r1] "s"(mr[1]), [r2] "s"(mr[2]), [r3] "s"(mr[3]), [i0] "s"(mi[0]),       \
              [i1] "s"(mi[1]), [i2] "s"(mi[2]), [i3] "s"(mi[3]));                                        \
    }
#define YAO_IP_CTL_FNS(T, V, SFX, MOV)                                                                   \
    /* (a, b) <- U (a, b) in the lanes of the mask m (a ballot), unchanged elsewhere */                \
    __device__ __forceinline__ void dense_ctl_ip(V& a, V& b, const T* mr, const T* mi, uint64_t m)     \
    {                                                                                                   \
        T t0, t1, t2, t3;                                                                               \
        uint64_t sv;                                                                                    \
        asm volatile("v_mul_" SFX " %[t0], %[r0], %[ax]\n\t"                                          \
                     "v_mul_" SFX " %[t1], %[r0], %[ay]\n\t"                                          \
                     "v_mul_" SFX " %[t2], %[r2], %[ax]\n\t"                                          \
                     "v_mul_" SFX " %[t3], %[r2], %[ay]\n\t"                                          \
                     "v_fma_" SFX " %[t0], -%[i0], %[ay], %[t0]\n\t"                                  \
                     "v_fma_" SFX " %[t1], %[i0], %[ax], %[t1]\n\t"                                   \
                     "v_fma_" SFX " %[t2], -%[i2], %[ay], %[t2]\n\t"                                  \
                     "v_fma_" SFX " %[t3], %[i2], %[ax], %[t3]\n\t"                                   \
                     "v_fma_" SFX " %[t0], %[r1], %[bx], %[t0]\n\t"                                   \
                     "v_fma_" SFX " %[t1], %[i1], %[bx], %[t1]\n\t"                                   \
                     "v_fma_" SFX " %[t2], %[r3], %[bx], %[t2]\n\t"                                   \
                     "v_fma_" SFX " %[t3], %[i3], %[bx], %[t3]\n\t"                                   \
                     "v_fma_" SFX " %[t0], -%[i1], %[by], %[t0]\n\t"                                  \
                     "v_fma_" SFX " %[t1], %[r1], %[by], %[t1]\n\t"                                   \
                     "v_fma_" SFX " %[t2], -%[i3], %[by], %[t2]\n\t"                                  \
                     "v_fma_" SFX " %[t3], %[r3], %[by], %[t3]\n\t"                                   \
                     "s_mov_b64 %[sv], exec\n\t"                                                      \
                     "s_mov_b64 exec, %[m]\n\t"                                                       \
                     MOV " %[ax], %[t0]\n\t"                                                          \
                     MOV " %[ay], %[t1]\n\t"                                                          \
                     MOV " %[bx], %[t2]\n\t"                                                          \
                     MOV " %[by], %[t3]\n\t"                                                          \
                     "s_mov_b64 exec, %[sv]"                                                            \
                     : [ax] "+v"(a.x), [ay] "+v"(a.y), [bx] "+v"(b.x), [by] "+v"(b.y), [t0] "=&v"(t0),   \
                       [t1] "=&v"(t1), [t2] "=&v"(t2), [t3] "=&v"(t3), [sv] "=&s"(sv)                   \
                     : [r0] "s"(mr[0]), [r1] "s"(mr[1]), [r2] "s"(mr[2]), [r3] "s"(mr[3]),              \
                       [i0] "s"(mi[0]), [i1] "s"(mi[1]), [i2] "s"(mi[2]), [i3] "s"(mi[3]), [m] "s"(m));  \
    }
YAO_IP_CTL_FNS(float, float2, "f32", "v_mov_b32")
YAO_IP_CTL_FNS(double, double2, "f64", "v_mov_b64")
#undef YAO_IP_CTL_FNS
YAO_IP_FNS(float, float2, "f32", "v_mov_b32")
YAO_IP_FNS(double, double2, "f64", "v_mov_b64")
#undef YAO_IP_FNS

// Swap a and b in the lanes of the mask m (a ballot, so a subset of the active lanes): exec is
// narrowed to m for the moves and restored.
__device__ __forceinline__ void cswap_ip(float2& a, float2& b, uint64_t m)
{
    uint64_t sv;
    asm volatile("s_mov_b64 %[sv], exec\n\t"
                 "s_mov_b64 exec, %[m]\n\t"
                 "v_swap_b32 %[ax], %[bx]\n\t"
                 "v_swap_b32 %[ay], %[by]\n\t"
                 "s_mov_b64 exec, %[sv]"
                 : [ax] "+v"(a.x), [ay] "+v"(a.y), [bx] "+v"(b.x), [by] "+v"(b.y), [sv] "=&s"(sv)
                 : [m] "s"(m));
}
__device__ __forceinline__ void cswap_ip(double2& a, double2& b, uint64_t m)
{
    uint64_t sv;
    double t;
    asm volatile("s_mov_b64 %[sv], exec\n\t"
                 "s_mov_b64 exec, %[m]\n\t"
                 "v_mov_b64 %[t], %[ax]\n\t"
                 "v_mov_b64 %[ax], %[bx]\n\t"
                 "v_mov_b64 %[bx], %[t]\n\t"
                 "v_mov_b64 %[t], %[ay]\n\t"
                 "v_mov_b64 %[ay], %[by]\n\t"
                 "v_mov_b64 %[by], %[t]\n\t"
                 "s_mov_b64 exec, %[sv]"
                 : [ax] "+v"(a.x), [ay] "+v"(a.y), [bx] "+v"(b.x), [by] "+v"(b.y), [t] "=&v"(t), [sv] "=&s"(sv)
                 : [m] "s"(m));
}
__device__ __forceinline__ void cswap_ip(double2& a, double2& b, double2& c, double2& d, uint64_t m)
{
    uint64_t sv;
    double t;
    asm volatile("s_mov_b64 %[sv], exec\n\t"
                 "s_mov_b64 exec, %[m]\n\t"
                 "v_mov_b64 %[t], %[ax]\n\t"
                 "v_mov_b64 %[ax], %[bx]\n\t"
                 "v_mov_b64 %[bx], %[t]\n\t"
                 "v_mov_b64 %[t], %[ay]\n\t"
                 "v_mov_b64 %[ay], %[by]\n\t"
                 "v_mov_b64 %[by], %[t]\n\t"
                 "v_mov_b64 %[t], %[cx]\n\t"
                 "v_mov_b64 %[cx], %[dx]\n\t"
                 "v_mov_b64 %[dx], %[t]\n\t"
                 "v_mov_b64 %[t], %[cy]\n\t"
                 "v_mov_b64 %[cy], %[dy]\n\t"
                 "v_mov_b64 %[dy], %[t]\n\t"
                 "s_mov_b64 exec, %[sv]"
                 : [ax] "+v"(a.x), [ay] "+v"(a.y), [bx] "+v"(b.x), [by] "+v"(b.y), [cx] "+v"(c.x),
                   [cy] "+v"(c.y), [dx] "+v"(d.x), [dy] "+v"(d.y), [t] "=&v"(t), [sv] "=&s"(sv)
                 : [m] "s"(m));
}

// diag(1, d) on a register bit: the reverse passes' Z-generator diagonal ops, whose first entry
// is carried as a phase of the whole tile.
constexpr int kDiagHigh = 100;

// An uncontrolled one-qubit op of structure TYPE (OT_RX, OT_DIAG, kDiagHigh or OT_DENSE) on
// register bit J.
template <int J, int TYPE, typename RR, typename V, int N>
__device__ __forceinline__ void pairs_ip(V (&x)[N], const RR* mr, const RR* mi)
{
#pragma unroll
    for (int a = 0; a < N; ++a) {
        if (a & (1 << J)) continue;
        V& p = x[a];
        V& q = x[a + (1 << J)];
        if constexpr (TYPE == OT_RX) {
            rx_ip(p, q, mr[0], mi[1]);
        } else if constexpr (TYPE == OT_DIAG) {
            diag_ip(p, mr[0], mi[0]);
            diag_ip(q, mr[3], mi[3]);
        } else if constexpr (TYPE == kDiagHigh) {
            diag_ip(q, mr[3], mi[3]);
        } else {
            dense_ip(p, q, mr, mi);
        }
    }
}

// Any one-qubit op on register bit J (as a dense 2 x 2 matrix) where the pair's tile index
// matches the tile-bit controls (every pair when cmask is 0); the backward form updates psi
// and lambda with the same matrix.
template <int J, typename RR, typename V, int N>
__device__ __forceinline__ void pairs_dense_ctl_ip(V (&x)[N], const RR* mr, const RR* mi, uint32_t ethr,
                                                   const uint32_t (&er)[N], uint32_t cmask, uint32_t cval)
{
#pragma unroll
    for (int a = 0; a < N; ++a) {
        if (a & (1 << J)) continue;
        const uint64_t m = __builtin_amdgcn_ballot_w64(((ethr | er[a]) & cmask) == cval);
        dense_ctl_ip(x[a], x[a + (1 << J)], mr, mi, m);
    }
}
template <int J, int N>
__device__ __forceinline__ void pairs_dense_ctl_ip(double2 (&x)[N], double2 (&y)[N], const double* mr,
                                                   const double* mi, uint32_t ethr, const uint32_t (&er)[N],
                                                   uint32_t cmask, uint32_t cval)
{
#pragma unroll
    for (int a = 0; a < N; ++a) {
        if (a & (1 << J)) continue;
        const uint64_t m = __builtin_amdgcn_ballot_w64(((ethr | er[a]) & cmask) == cval);
        dense_ctl_ip(x[a], x[a + (1 << J)], mr, mi, m);
        dense_ctl_ip(y[a], y[a + (1 << J)], mr, mi, m);
    }
}

// A SWAP of the pair on register bit J where the pair's tile index matches the tile-bit controls.
template <int J, typename V, int N>
__device__ __forceinline__ void pairs_cswap_ip(V (&x)[N], uint32_t ethr, const uint32_t (&er)[N], uint32_t cmask,
                                               uint32_t cval)
{
    if ((cmask & ~er[N - 1]) == 0) {
        // Controls on register bits only (er[N - 1] holds them all): a pair is swapped in
        // every lane or in none, so the pairs that fail them cost nothing.
#pragma unroll
        for (int a = 0; a < N; ++a) {
            if (a & (1 << J)) continue;
            if ((er[a] & cmask) == cval) cswap_ip(x[a], x[a + (1 << J)], __builtin_amdgcn_read_exec());
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
        if (a & (1 << J)) continue;
        const uint64_t m = __builtin_amdgcn_ballot_w64(((ethr | er[a]) & cmask) == cval);
        cswap_ip(x[a], x[a + (1 << J)], m);
    }
}
template <int J, int N>
__device__ __forceinline__ void pairs_cswap_ip(double2 (&x)[N], double2 (&y)[N], uint32_t ethr,
                                               const uint32_t (&er)[N], uint32_t cmask, uint32_t cval)
{
    if ((cmask & ~er[N - 1]) == 0) {
        // Controls on register bits only, as above.
#pragma unroll
        for (int a = 0; a < N; ++a) {
            if (a & (1 << J)) continue;
            if ((er[a] & cmask) == cval)
                cswap_ip(x[a], x[a + (1 << J)], y[a], y[a + (1 << J)], __builtin_amdgcn_read_exec());
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
        if (a & (1 << J)) continue;
        const uint64_t m = __builtin_amdgcn_ballot_w64(((ethr | er[a]) & cmask) == cval);
        cswap_ip(x[a], x[a + (1 << J)], y[a], y[a + (1 << J)], m);
    }
}

// 2 Re( conj(l0) (M p)_0 + conj(l1) (M p)_1 ) for the generator class GEN.
template <int GEN>
__device__ __forceinline__ double grad_pair(const double* mr, const double* mi, const double2& p0, const double2& p1,
                                            const double2& l0, const double2& l1)
{
    if constexpr (GEN == GEN_X) {  // M = -(i/2) X: Im(conj(l0) p1 + conj(l1) p0)
        return fma(l0.x, p1.y, fma(-l0.y, p1.x, fma(l1.x, p0.y, -l1.y * p0.x)));
    } else if constexpr (GEN == GEN_Y) {  // M = -(i/2) Y = [[0, -1/2], [1/2, 0]]
        return fma(l1.x, p0.x, fma(l1.y, p0.y, fma(-l0.x, p1.x, -l0.y * p1.y)));
    } else if constexpr (GEN == GEN_Z) {  // M = diag(-i/2, i/2)
        return fma(l0.x, p0.y, fma(-l0.y, p0.x, fma(-l1.x, p1.y, l1.y * p1.x)));
    } else if constexpr (GEN == GEN_P1) {  // M = diag(0, i)
        return -2.0 * fma(l1.x, p1.y, -l1.y * p1.x);
    } else {
        double m0x = mr[0] * p0.x - mi[0] * p0.y + mr[1] * p1.x - mi[1] * p1.y;
        double m0y = mr[0] * p0.y + mi[0] * p0.x + mr[1] * p1.y + mi[1] * p1.x;
        double m1x = mr[2] * p0.x - mi[2] * p0.y + mr[3] * p1.x - mi[3] * p1.y;
        double m1y = mr[2] * p0.y + mi[2] * p0.x + mr[3] * p1.y + mi[3] * p1.x;
        return 2.0 * (l0.x * m0x + l0.y * m0y + l1.x * m1x + l1.y * m1y);
    }
}

template <int J, bool CTRL, int GEN, int N>
__device__ __forceinline__ double pairs_grad(const double2 (&x)[N], const double2 (&y)[N], const double* mr,
                                             const double* mi, uint32_t ethr, const uint32_t (&er)[N], uint32_t cmask,
                                             uint32_t cval)
{
    double g = 0;
    bool first = true;  // resolved at compile time when CTRL is false
#pragma unroll
    for (int a = 0; a < N; ++a) {
        if (a & (1 << J)) continue;
        const double v = grad_pair<GEN>(mr, mi, x[a], x[a + (1 << J)], y[a], y[a + (1 << J)]);
        if (CTRL) g += (((ethr | er[a]) & cmask) == cval) ? v : 0.0;  // a select
        else g = first ? v : g + v;
        first = false;
    }
    return g;
}

template <int J, bool CTRL, int N>
__device__ __forceinline__ double op_grad(const double2 (&x)[N], const double2 (&y)[N], int gen, const double* mr,
                                          const double* mi, uint32_t ethr, const uint32_t (&er)[N], uint32_t cmask,
                                          uint32_t cval)
{
    switch (gen) {
    case GEN_X: return pairs_grad<J, CTRL, GEN_X>(x, y, mr, mi, ethr, er, cmask, cval);
    case GEN_Y: return pairs_grad<J, CTRL, GEN_Y>(x, y, mr, mi, ethr, er, cmask, cval);
    case GEN_Z: return pairs_grad<J, CTRL, GEN_Z>(x, y, mr, mi, ethr, er, cmask, cval);
    case GEN_P1: return pairs_grad<J, CTRL, GEN_P1>(x, y, mr, mi, ethr, er, cmask, cval);
    default: return pairs_grad<J, CTRL, GEN_DENSE>(x, y, mr, mi, ethr, er, cmask, cval);
    }
}

// ------------------------------------------------------------------------------ tile helpers
struct TileCtx {
    uint64_t base;   // amplitude index bits outside the tile
    uint64_t dth;    // this thread's deposited qubit bits for the load/store mapping
    uint64_t toff;   // element offset of the thread's register 0: (base | dth) * B + bidx
    int b0, bl;      // first batch slot of the tile, this thread's slot offset
    int bidx;        // batch slot this thread loads: b0 + bl, clamped to the last slot
    bool bvalid;     // b0 + bl < B: only then does the thread store
};

// Load/store mapping: element e = th + r * nthr; the low c bits of th are the batch slot, the
// next t - RB - c bits of th and then the RB bits of r are the tile qubits in ascending order.
template <int RB> __device__ __forceinline__ TileCtx tile_ctx(const PassArgs& a, int th)
{
    TileCtx tc;
    uint64_t base = 0;
    const uint64_t tid = blockIdx.x;
#pragma unroll
    for (int j = 0; j < 40; ++j)
        if (j < a.nnt) base |= ((tid >> j) & uint64_t(1)) << a.nontile_qubits[j];
    tc.base = base;
    const int c = a.c, t = a.t;
    uint64_t dth = 0;
    const uint32_t q = (uint32_t)th >> c;
#pragma unroll
    for (int j = 0; j < kMaxTileBits; ++j)
        if (j < t - RB - c) dth |= (uint64_t)((q >> j) & 1u) << a.tile_qubits[j];
    tc.dth = dth;
    tc.b0 = blockIdx.y << c;
    tc.bl = th & ((1 << c) - 1);
    tc.bvalid = tc.b0 + tc.bl < a.B;
    tc.bidx = tc.bvalid ? tc.b0 + tc.bl : a.B - 1;
    tc.toff = (base | dth) * (uint64_t)a.B + (uint64_t)tc.bidx;
    return tc;
}

// LDS tile bits of the thread part (the low nb bits of th) of a stored element.
__device__ __forceinline__ uint32_t store_thread_bits(const PassArgs& a, int th, int nb)
{
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < kMaxTileBits; ++i)
        if (i < nb) v |= (((uint32_t)th >> i) & 1u) << a.ssrc[i];
    return v;
}

// The register bits of the load mapping are tile qubits whose offsets are the same for every
// thread: the host passes them per register.
template <int RB> __device__ __forceinline__ uint64_t tile_off(const PassArgs& a, const TileCtx& tc, int r)
{
    return tc.toff + a.rofs[r];
}

// Tile index of register element r in a register group, split into the per-thread part
// (ethr) and the per-register part (er[r], the same for every thread).
template <int RB>
__device__ __forceinline__ void group_index(const int (&rpos)[kMaxRegBits], int t, int th, uint32_t& ethr,
                                            uint32_t (&er)[1 << RB])
{
    uint32_t rmask = 0;
#pragma unroll
    for (int j = 0; j < RB; ++j) rmask |= 1u << rpos[j];
    uint32_t v = 0;
    int k = 0;
    for (int b = 0; b < t; ++b) {
        if ((rmask >> b) & 1u) continue;
        v |= (((uint32_t)th >> k) & 1u) << b;
        ++k;
    }
    ethr = v;
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        uint32_t e = 0;
#pragma unroll
        for (int j = 0; j < RB; ++j) e |= ((uint32_t)(r >> j) & 1u) << rpos[j];
        er[r] = e;
    }
}

// The dense block matrices of a forward pass are copied to LDS in 16-byte words; the first
// kDmRegs words of every thread are loaded together with the tile (one wait for both), with
// indices clamped so that every load is in bounds.
static_assert(sizeof(POp) % 16 == 0 && sizeof(PGroupDesc) % 16 == 0, "16-byte records");
constexpr int kDmRegs = 4;
// With no dense matrices the words are read from the first op record (every forward pass has
// one) and dropped, so the registers are always defined.
__device__ __forceinline__ void dm_load(const PassArgs& a, int th, int nthr, uint4 (&w)[kDmRegs])
{
    const uint4* src = a.ndm > 0 ? a.dmats : (const uint4*)a.ops;
    const int last = a.ndm > 0 ? a.ndm - 1 : 0;
#pragma unroll
    for (int k = 0; k < kDmRegs; ++k) w[k] = src[min(th + k * nthr, last)];
}
__device__ __forceinline__ void dm_store(const PassArgs& a, uint4* ldm, int th, int nthr, const uint4 (&w)[kDmRegs])
{
    // Unconditional: a clamped index writes the word it loaded, so duplicates are identical.
#pragma unroll
    for (int k = 0; k < kDmRegs; ++k) ldm[min(th + k * nthr, a.ndm - 1)] = w[k];
    for (int i = th + kDmRegs * nthr; i < a.ndm; i += nthr) ldm[i] = a.dmats[i];
}

struct GroupCtl {
    int lds, op0, nops;
    int rpos[kMaxRegBits];
};
__device__ __forceinline__ GroupCtl group_ctl_c(const YAO_CONST PGroupDesc* g)
{
    GroupCtl o;
    o.lds = g->lds;
    o.op0 = g->op0;
    o.nops = g->nops;
#pragma unroll
    for (int j = 0; j < kMaxRegBits; ++j) o.rpos[j] = g->rpos[j];
    return o;
}

// ------------------------------------------------------------------------------ gradient sums
// v from lane (lane op CTRL) of the same DPP row, both 32-bit halves. The patterns used here
// read inside the row only, so every source lane is valid.
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum of v over the lanes of a 16-lane row that share this lane's low c bits (its batch slot
// of the tile); lanes 0 .. 2^c - 1 of the row end with the sums of slots 0 .. 2^c - 1. Every
// lane of the row must be active.
__device__ __forceinline__ double row_sum(double v, int c)
{
    if (c < 1) v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]: lane ^ 1
    if (c < 2) v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]: lane ^ 2
    if (c < 3) v += dpp_f64<0x124>(v);  // row_ror 4
    v += dpp_f64<0x128>(v);             // row_ror 8
    return v;
}

// Reduce partials red[s * E + e] for gradient s < S (entry e holds batch slot e mod 2^c) to
// one value per (gradient, batch slot b0 + j of the tile) and store it in gpartial at
// ((slot_of(s) * B + b0 + j) * pstride + col). The order of the sums is fixed.
template <typename SlotOf>
__device__ __forceinline__ void reduce_partials(double* __restrict__ gpartial, int B, int pstride, int c,
                                                const double* red, SlotOf slot_of, int S, int E, int nthr, int th,
                                                int col, int b0)
{
    const int Bc = 1 << c;
    if (nthr >= 16) {
        for (int task = th; task < S * 16; task += nthr) {
            const int s = task >> 4, j = task & 15;
            double v = 0;
            for (int e = j; e < E; e += 16) v += red[s * E + e];
            for (int off = 8; off >= Bc; off >>= 1) v += __shfl_xor(v, off, 16);
            if (j < Bc && b0 + j < B) gpartial[((uint64_t)slot_of(s) * B + b0 + j) * pstride + col] = v;
        }
    } else {
        for (int task = th; task < S * Bc; task += nthr) {
            const int s = task / Bc, bb = task % Bc;
            double v = 0;
            for (int e = bb; e < E; e += Bc) v += red[s * E + e];
            if (b0 + bb < B) gpartial[((uint64_t)slot_of(s) * B + b0 + bb) * pstride + col] = v;
        }
    }
}

// Sorted target positions and member offsets of a K-qubit op inside the tile.
template <int K> struct LdsGeom {
    int sorted[K];
    uint32_t off[1 << K];
};

template <int K> __device__ __forceinline__ LdsGeom<K> lds_geom(const int* tpos)
{
    LdsGeom<K> g;
#pragma unroll
    for (int i = 0; i < K; ++i) g.sorted[i] = tpos[i];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = i + 1; j < K; ++j)
            if (g.sorted[j] < g.sorted[i]) {
                int tmp = g.sorted[i];
                g.sorted[i] = g.sorted[j];
                g.sorted[j] = tmp;
            }
#pragma unroll
    for (int s = 0; s < (1 << K); ++s) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((s >> j) & 1) o |= 1u << tpos[j];
        g.off[s] = o;
    }
    return g;
}

template <int K> __device__ __forceinline__ uint32_t lds_base(uint32_t gidx, const LdsGeom<K>& g)
{
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint32_t lo = gidx & ((1u << g.sorted[i]) - 1);
        gidx = ((gidx >> g.sorted[i]) << (g.sorted[i] + 1)) | lo;
    }
    return gidx;
}

template <typename RP, int K>
__device__ __noinline__ void lds_op_fwd(vec2_t<RP>* lp, const YAO_CONST POp* rec, const double* m, int t, int th,
                                        int nthr)
{
    using VP = vec2_t<RP>;
    constexpr int D = 1 << K, DD = D * D;
    int tpos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) tpos[j] = sc(rec->tpos[j]);
    const uint32_t cmask = (uint32_t)sc((int)rec->cmask), cval = (uint32_t)sc((int)rec->cval);
    const LdsGeom<K> g = lds_geom<K>(tpos);
    for (int gidx = th; gidx < (1 << (t - K)); gidx += nthr) {
        const uint32_t eb = lds_base<K>((uint32_t)gidx, g);
        if ((eb & cmask) != cval) continue;
        VP v[D];
#pragma unroll
        for (int s = 0; s < D; ++s) v[s] = lp[swz(eb | g.off[s])];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            RP x = 0, y = 0;
#pragma unroll
            for (int s = 0; s < D; ++s) {
                const RP ur = (RP)m[r * D + s], ui = (RP)m[DD + r * D + s];
                x = fma(ur, v[s].x, fma(-ui, v[s].y, x));
                y = fma(ur, v[s].y, fma(ui, v[s].x, y));
            }
            lp[swz(eb | g.off[r])] = mkv<VP, RP>(x, y);
        }
    }
}

template <typename RL, int K>
__device__ __noinline__ double lds_op_bwd(double2* lp, vec2_t<RL>* ll, const YAO_CONST POp* rec, const double* m, int t, int th,
                                          int nthr)
{
    using VL = vec2_t<RL>;
    constexpr int D = 1 << K, DD = D * D;
    int tpos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) tpos[j] = sc(rec->tpos[j]);
    const uint32_t cmask = (uint32_t)sc((int)rec->cmask), cval = (uint32_t)sc((int)rec->cval);
    const bool grad = sc(rec->slot) >= 0;
    const LdsGeom<K> g = lds_geom<K>(tpos);
    const double* Mr = m + 2 * DD;
    const double* Mi = m + 3 * DD;
    double acc = 0;
    for (int gidx = th; gidx < (1 << (t - K)); gidx += nthr) {
        const uint32_t eb = lds_base<K>((uint32_t)gidx, g);
        if ((eb & cmask) != cval) continue;
        double2 p[D], l[D];
#pragma unroll
        for (int s = 0; s < D; ++s) {
            p[s] = lp[swz(eb | g.off[s])];
            const VL w = ll[swz(eb | g.off[s])];
            l[s] = make_double2((double)w.x, (double)w.y);
        }
        if (grad) {
#pragma unroll
            for (int r = 0; r < D; ++r) {
                double x = 0, y = 0;
#pragma unroll
                for (int s = 0; s < D; ++s) {
                    x += Mr[r * D + s] * p[s].x - Mi[r * D + s] * p[s].y;
                    y += Mr[r * D + s] * p[s].y + Mi[r * D + s] * p[s].x;
                }
                acc += 2.0 * (l[r].x * x + l[r].y * y);
            }
        }
#pragma unroll
        for (int r = 0; r < D; ++r) {
            double x = 0, y = 0, u = 0, w = 0;
#pragma unroll
            for (int s = 0; s < D; ++s) {
                const double ur = m[r * D + s], ui = m[DD + r * D + s];
                x += ur * p[s].x - ui * p[s].y;
                y += ur * p[s].y + ui * p[s].x;
                u += ur * l[s].x - ui * l[s].y;
                w += ur * l[s].y + ui * l[s].x;
            }
            lp[swz(eb | g.off[r])] = make_double2(x, y);
            ll[swz(eb | g.off[r])] = mkv<VL, RL>((RL)u, (RL)w);
        }
    }
    return acc;
}

// y = M x for the 16 register elements of a thread. M sits in LDS column-major: column c is
// re[16] then im[16] in the precision RR; every lane reads the same address (broadcast).
template <typename RR, typename V>
__device__ __forceinline__ void dense16_apply(V (&x)[16], const RR* M)
{
    RR yr[16], yi[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) yr[r] = yi[r] = (RR)0;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const RR* col = M + c * 32;
        const RR xr = x[c].x, xi = x[c].y;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const RR mr = col[r], mi = col[16 + r];
            yr[r] = fma(mr, xr, yr[r]);
            yi[r] = fma(mr, xi, yi[r]);
            yr[r] = fma(-mi, xi, yr[r]);
            yi[r] = fma(mi, xr, yi[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = mkv<V, RR>(yr[r], yi[r]);
}

typedef float v4f __attribute__((ext_vector_type(4)));

// A dense block on the FP32 matrix cores, for complex64 tiles of >= 64 columns (one column per
// thread of the group). The block's 4 bits p[0..3] (ascending) index the 16 amplitudes of a
// column; the other t - 4 tile bits number the columns. Taking 16 columns as the B operand
// [Re x; Im x] (32 x 16), the update is the real GEMM [[Re M, -Im M], [Im M, Re M]] x B with
// v_mfma_f32_16x16x4f32 (A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k,
// D[4 (l / 16) + v][l % 16] in accumulator v of lane l). Each wave takes 64 columns; the
// amplitudes are read from and written back to the LDS tile in that layout, so no barrier
// is needed inside the block. Mf holds the 16 A fragments of 64 lanes each.
__device__ __forceinline__ uint32_t insert_zeros4(uint32_t c, const int (&p)[kMaxRegBits])
{
#pragma unroll
    for (int j = 0; j < 4; ++j) c = ((c >> p[j]) << (p[j] + 1)) | (c & ((1u << p[j]) - 1));
    return c;
}
__device__ __forceinline__ uint32_t deposit4(uint32_t b, const int (&p)[kMaxRegBits])
{
    uint32_t e = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) e |= ((b >> j) & 1u) << p[j];
    return e;
}
__device__ __forceinline__ void dense16_mfma(float2* lp, const float2* M, const int (&p)[kMaxRegBits], int th,
                                             uint32_t cmask, uint32_t cval)
{
    const int lane = th & 63, wave = th >> 6;
    const int q = lane >> 4, cl = lane & 15;
    // A fragments of the real form: row 16 rt + cl, column 4 kc + q, from the complex matrix
    // M (row-major, 16 x 16): Re, -Im in the upper half, Im, Re in the lower one.
    float a[16];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
        const float2 m = M[cl * 16 + 4 * kc + q];
        a[kc] = m.x;
        a[4 + kc] = -m.y;
        a[8 + kc] = m.y;
        a[12 + kc] = m.x;
    }
    uint32_t bin[4], bout[4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
        bin[s2] = deposit4((uint32_t)(q + 4 * s2), p);
        bout[s2] = deposit4((uint32_t)(4 * q + s2), p);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const uint32_t ec = insert_zeros4((uint32_t)(wave * 64 + ct * 16 + cl), p);
        float2 xv[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) xv[s2] = lp[swz(ec | bin[s2])];
        v4f acc0 = v4f{0.f, 0.f, 0.f, 0.f}, acc1 = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 8; ++kc) {
            const float bv = kc < 4 ? xv[kc].x : xv[kc - 4].y;
            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kc], bv, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[8 + kc], bv, acc1, 0, 0, 0);
        }
        if ((ec & cmask) == cval) {
#pragma unroll
            for (int v = 0; v < 4; ++v) lp[swz(ec | bout[v])] = make_float2(acc0[v], acc1[v]);
        }
    }
}

// ------------------------------------------------------------------------------ forward kernel
template <typename RP>
__global__ __launch_bounds__(512, sizeof(RP) == 4 ? 3 : 1) void k_pass_fwd(PassArgs a)
{
    constexpr int RB = kRegBitsFwd, N = 1 << RB;
    using VP = vec2_t<RP>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = a.t;
    const int nthr = 1 << (t - RB);
    const int th = threadIdx.x;
    // LDS: tile | dense block matrices (2 * 256 RP each), sized for this pass.
    VP* lp = (VP*)smem;
    uint4* ldm = (uint4*)(smem + (sizeof(VP) << t));
    const YAO_CONST POp* gops = cptr(z_ops(a));
    const YAO_CONST PGroupDesc* ggrp = cptr(a.groups);
    const TileCtx tc = tile_ctx<RB>(a, th);
    VP* gp = (VP*)z_psi(a);
    // Every load is in bounds (slots past B read the last slot and are never stored), so all
    // of them are issued before the first wait.
    {
        uint4 w[kDmRegs];
        dm_load(a, th, nthr, w);
        // The tile goes straight to LDS before the matrices' remaining words: a register copy
        // of it held across that loop stayed in scratch memory.
#pragma unroll
        for (int r = 0; r < N; ++r) lp[swz((uint32_t)th + (uint32_t)r * nthr)] = gp[tile_off<RB>(a, tc, r)];
        if (a.ndm) dm_store(a, ldm, th, nthr, w);
    }
    __syncthreads();

    for (int gi = 0; gi < a.ngroups; ++gi) {
        const GroupCtl G = group_ctl_c(ggrp + gi);
        if (G.lds == 2) {
            // One dense block on the register bits; its remaining controls are on tile bits
            // outside them (the same for all 16 elements of a thread) or outside the tile.
            OpCtl op = op_ctl_c(gops + G.op0);
            fold_outer_controls(op, tc.base);
            if constexpr (sizeof(RP) == 4) {
                // Complex64 plans hold dense blocks only for tiles of >= 64 columns.
                dense16_mfma(lp, (const float2*)ldm + op.mat * 256, G.rpos, th, op.cmask, op.cval);
            } else {
                uint32_t ethr, er[N];
                group_index<RB>(G.rpos, t, th, ethr, er);
                VP x[N];
#pragma unroll
                for (int r = 0; r < N; ++r) x[r] = lp[swz(ethr | er[r])];
                if ((ethr & op.cmask) == op.cval) dense16_apply<RP>(x, (const RP*)ldm + op.mat * 512);
#pragma unroll
                for (int r = 0; r < N; ++r) lp[swz(ethr | er[r])] = x[r];
            }
            __syncthreads();
            continue;
        }
        if (G.lds) {
            const YAO_CONST POp* rec = gops + G.op0;
            const uint64_t omask = rec->omask, oval = rec->oval;
            if ((tc.base & omask) == oval) {
                const double* m = a.mats + rec->mat;
                if (rec->k == 2) lds_op_fwd<RP, 2>(lp, rec, m, t, th, nthr);
                else lds_op_fwd<RP, 3>(lp, rec, m, t, th, nthr);
            }
            __syncthreads();
            continue;
        }
        uint32_t ethr, er[N];
        group_index<RB>(G.rpos, t, th, ethr, er);
        VP x[N];
#pragma unroll
        for (int r = 0; r < N; ++r) x[r] = lp[swz(ethr | er[r])];
        // One op: the common classes (see op_variant: no controls outside the tile, and none
        // at all but for the controlled SWAP) have in-place code of their own, picked by one
        // switch on the variant the host chose; the rest take the masked dense update.
        auto apply = [&](const OpS<RP>& o) __attribute__((always_inline)) {
            const RP* mr = o.m;
            const RP* mi = o.m + 4;
#define YAO_FWD_CASE(J)                                                  \
    case J: {                                                            \
        OpCtl op = o.c;                                                  \
        fold_outer_controls(op, tc.base);                                \
        pairs_dense_ctl_ip<J>(x, mr, mi, ethr, er, op.cmask, op.cval);   \
        break;                                                           \
    }
#define YAO_FWD_FAST(J)                                                                            \
    case 0 * kRegBitsFwd + J: pairs_ip<J, OT_RX>(x, mr, mi); break;                                 \
    case 1 * kRegBitsFwd + J: pairs_ip<J, OT_DIAG>(x, mr, mi); break;                               \
    case 2 * kRegBitsFwd + J: pairs_ip<J, OT_DENSE>(x, mr, mi); break;                              \
    case 3 * kRegBitsFwd + J: pairs_cswap_ip<J>(x, ethr, er, o.c.cmask, o.c.cval); break;
            switch (o.c.var) {
                YAO_FWD_FAST(0) YAO_FWD_FAST(1) YAO_FWD_FAST(2) YAO_FWD_FAST(3)
            default:
                switch (o.c.rpos) { YAO_FWD_CASE(0) YAO_FWD_CASE(1) YAO_FWD_CASE(2) default: YAO_FWD_CASE(3) }
                break;
            }
#undef YAO_FWD_FAST
#undef YAO_FWD_CASE
        };
        // Two record buffers in turn: the record of the next op is loaded (scalar loads) while
        // the current one computes, and is waited for only at the end of it. The record one
        // past a group's last op is always readable (it lies inside the program's buffer) and
        // is never used.
        // Scalar loads return out of order, so each buffer's wait is placed (and fenced from
        // the scheduler) before the other buffer's loads are issued; otherwise it would also
        // wait for the prefetch.
        const YAO_CONST POp* rec = gops + G.op0;
        OpS<RP> A = load_op_c<RP>(rec);
        for (int oi = 0; oi < G.nops; oi += 2) {
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): A (and the LDS reads) arrived
            __builtin_amdgcn_sched_barrier(0);
            const OpS<RP> B = load_op_c<RP>(rec + oi + 1);
            apply(A);
            if (oi + 1 >= G.nops) break;
            __builtin_amdgcn_s_waitcnt(0xC07F);  // B arrived
            __builtin_amdgcn_sched_barrier(0);
            A = load_op_c<RP>(rec + oi + 2);
            apply(B);
        }
#pragma unroll
        for (int r = 0; r < N; ++r) lp[swz(ethr | er[r])] = x[r];
        __syncthreads();
    }

    if (tc.bvalid) {
        const uint32_t sth = store_thread_bits(a, th, t - RB);
#pragma unroll
        for (int r = 0; r < N; ++r) gp[tile_off<RB>(a, tc, r)] = lp[swz(sth | a.sreg[r])];
    }
}

// ------------------------------------------------------------------------------ backward kernel

// Where the gradient partials of a reverse sweep go: reduce_partials' gpartial, B, pstride
// and, for this tile, the column and the first batch slot.
struct GradOut {
    double* gpartial;
    int B, pstride, col, b0;
};

// The register groups and LDS ops of a reverse pass over the tile in LDS: psi (lp, FP64) and
// lambda (ll, in RL), with every gradient partial reduced per group into go. tbase holds the
// qubits outside the tile (for controls there); red0 holds two buffers of mslots * E
// partials (a group's partials are reduced after the barrier that ends it, while the next
// group fills the other buffer). C0: tiles of one batch slot (c = 0).
template <typename RL, bool C0>
__device__ __forceinline__ double2 reverse_groups(double2* lp, vec2_t<RL>* ll, double* red0, const YAO_CONST POp* gops,
                                               const YAO_CONST PGroupDesc* ggrp, const PGroupDesc* groups,
                                               int ngroups, const double* mats, uint64_t tbase, int t, int c,
                                               int nthr, int th, int mslots, const GradOut& go)
{
    constexpr int RB = kRegBitsBwd, N = 1 << RB;
    using VL = vec2_t<RL>;
    const bool rows = nthr >= 16;
    // Product of the first diagonal entries of the uncontrolled Z-generator ops applied so far:
    // those ops apply diag(1, d1 / d0) to both states and leave d0, a phase common to every
    // element of every tile, to the caller (gradients do not see a phase psi and lambda share).
    double2 phase = make_double2(1.0, 0.0);
    const int E = grad_entries(nthr, c);
    const int ent = rows ? (th >> 4) * (1 << c) + (th & 15) : th;
    const bool stores = rows ? (th & 15) < (1 << c) : true;
    int buf = 0;
    for (int gi = 0; gi < ngroups; ++gi) {
        const GroupCtl G = group_ctl_c(ggrp + gi);
        double* red = red0 + buf * (mslots * E);
        int nslot = 0;
        if (G.lds) {
            const YAO_CONST POp* rec = gops + G.op0;
            const uint64_t omask = rec->omask, oval = rec->oval;
            double g = 0;
            if ((tbase & omask) == oval) {
                const double* m = mats + rec->mat;
                if (rec->k == 2) g = lds_op_bwd<RL, 2>(lp, ll, rec, m, t, th, nthr);
                else g = lds_op_bwd<RL, 3>(lp, ll, rec, m, t, th, nthr);
            }
            if (rec->slot >= 0) {
                if (rows) g = row_sum(g, c);
                if (stores) red[ent] = g;
                nslot = 1;
            }
        } else {
            uint32_t ethr, er[N];
            group_index<RB>(G.rpos, t, th, ethr, er);
            double2 x[N], y[N];
#pragma unroll
            for (int r = 0; r < N; ++r) {
                const uint32_t p = swz(ethr | er[r]);
                x[r] = lp[p];
                const VL w = ll[p];
                y[r] = make_double2((double)w.x, (double)w.y);
            }
            // One op (see the forward kernel): its gradient partial first, from psi and lambda
            // before the update, then U^dagger on both.
            auto apply = [&](const OpS<double>& o) __attribute__((always_inline)) {
                const double* m = o.m;
                double g = 0;
#define YAO_BWD_CASE(J)                                                                                 \
    case J: {                                                                                           \
        OpCtl op = o.c;                                                                                 \
        fold_outer_controls(op, tbase);                                                                 \
        const double* gm = mats + op.mat + 8; /* M of a dense generator */                             \
        if (op.slot >= 0) {                                                                             \
            if (op.cmask) g = op_grad<J, true>(x, y, op.gen, gm, gm + 4, ethr, er, op.cmask, op.cval);  \
            else g = op_grad<J, false>(x, y, op.gen, gm, gm + 4, ethr, er, 0u, 0u);                     \
        }                                                                                               \
        pairs_dense_ctl_ip<J>(x, y, m, m + 4, ethr, er, op.cmask, op.cval);                             \
        break;                                                                                          \
    }
#define YAO_BWD_FAST(J)                                                          \
    case 0 * kRegBitsBwd + J:                                                    \
        g = pairs_grad<J, false, GEN_X>(x, y, m, m + 4, ethr, er, 0u, 0u);         \
        pairs_ip<J, OT_RX>(x, m, m + 4);                                         \
        pairs_ip<J, OT_RX>(y, m, m + 4);                                         \
        break;                                                                   \
    case 1 * kRegBitsBwd + J: {                                                  \
        g = pairs_grad<J, false, GEN_Z>(x, y, m, m + 4, ethr, er, 0u, 0u);         \
        pairs_ip<J, kDiagHigh>(x, m, m + 4);                                     \
        pairs_ip<J, kDiagHigh>(y, m, m + 4);                                     \
        const double pr = phase.x * m[0] - phase.y * m[4];                       \
        phase.y = phase.x * m[4] + phase.y * m[0];                               \
        phase.x = pr;                                                            \
        break;                                                                   \
    }                                                                            \
    case 2 * kRegBitsBwd + J:                                                    \
        pairs_cswap_ip<J>(x, y, ethr, er, o.c.cmask, o.c.cval);                  \
        break;
                switch (o.c.var) {
                    YAO_BWD_FAST(0) YAO_BWD_FAST(1) YAO_BWD_FAST(2)
                default:
                    switch (o.c.rpos) { YAO_BWD_CASE(0) YAO_BWD_CASE(1) default: YAO_BWD_CASE(2) }
                    break;
                }
#undef YAO_BWD_FAST
#undef YAO_BWD_CASE
                if (o.c.slot >= 0) {
                    if (rows) g = row_sum(g, c);
                    if (stores) red[nslot * E + ent] = g;
                    ++nslot;
                }
            };
            // Two record buffers in turn, as in the forward kernel.
            const YAO_CONST POp* rec = gops + G.op0;
            OpS<double> A = load_op_c<double>(rec);
            for (int oi = 0; oi < G.nops; oi += 2) {
                __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), as in the forward kernel
                __builtin_amdgcn_sched_barrier(0);
                const OpS<double> B = load_op_c<double>(rec + oi + 1);
                apply(A);
                if (oi + 1 >= G.nops) break;
                __builtin_amdgcn_s_waitcnt(0xC07F);
                __builtin_amdgcn_sched_barrier(0);
                A = load_op_c<double>(rec + oi + 2);
                apply(B);
            }
#pragma unroll
            for (int r = 0; r < N; ++r) {
                const uint32_t p = swz(ethr | er[r]);
                lp[p] = x[r];
                ll[p] = mkv<VL, RL>((RL)y[r].x, (RL)y[r].y);
            }
        }
        __syncthreads();
        if (nslot > 0) {
            const int* slots = groups[gi].slots;
            reduce_partials(go.gpartial, go.B, go.pstride, c, red, [&](int s) { return slots[s]; }, nslot, E, nthr,
                            th, go.col, go.b0);
            buf ^= 1;
        }
    }
    return phase;
}

// C0: tiles of one batch slot (c = 0), where every row-sum step applies. At most 168 VGPRs, so
// that three 256-thread tiles of 2^11 elements (48 KiB of LDS each) fit on one CU.
template <typename RL, bool C0>
__global__ __launch_bounds__(512, 3) void k_pass_bwd(PassArgs a)
{
    constexpr int RB = kRegBitsBwd, N = 1 << RB;
    using VL = vec2_t<RL>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = a.t;
    const int nthr = 1 << (t - RB);
    const int th = threadIdx.x;
    const int c = C0 ? 0 : a.c;
    // LDS: psi | lambda | gradient partials.
    double2* lp = (double2*)smem;
    VL* ll = (VL*)(smem + ((size_t)16 << t));
    double* red0 = (double*)(smem + ((size_t)(16 + sizeof(VL)) << t));
    const TileCtx tc = tile_ctx<RB>(a, th);
    double2* gp = (double2*)z_psi(a);
    VL* gl = (VL*)z_lam(a);
    // Straight from global memory to LDS: a staging array here stayed in scratch memory
    // (a store and a reload per element through the cache hierarchy).
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const uint64_t off = tile_off<RB>(a, tc, r);
        const uint32_t e = swz((uint32_t)th + (uint32_t)r * nthr);
        lp[e] = gp[off];
        ll[e] = gl[off];
    }
    __syncthreads();

    const GradOut go{z_partial(a, a.gpartial), a.B, a.pstride, (int)blockIdx.x, (int)blockIdx.y << c};
    const double2 ph = reverse_groups<RL, C0>(lp, ll, red0, cptr(z_ops(a)), cptr(a.groups), a.groups, a.ngroups,
                                              a.mats, tc.base, t, c, nthr, th, a.mslots, go);

    if (tc.bvalid) {
        const uint32_t sth = store_thread_bits(a, th, t - RB);
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const uint64_t off = tile_off<RB>(a, tc, r);
            const uint32_t e = swz(sth | a.sreg[r]);
            const double2 v = lp[e];
            const VL w = ll[e];
            const double wx = (double)w.x, wy = (double)w.y;
            gp[off] = make_double2(ph.x * v.x - ph.y * v.y, ph.x * v.y + ph.y * v.x);
            gl[off] = mkv<VL, RL>((RL)(ph.x * wx - ph.y * wy), (RL)(ph.x * wy + ph.y * wx));
        }
    }
}

// ------------------------------------------------------------------------------ small circuits
// The register groups and LDS ops of a forward pass with 3 register bits and FP64 matrices
// over a tile in LDS that holds every qubit (no controls outside it, no dense blocks).
__device__ __forceinline__ void forward_groups3(double2* lp, const YAO_CONST POp* gops,
                                                const YAO_CONST PGroupDesc* ggrp, int ngroups, const double* mats,
                                                int t, int nthr, int th)
{
    constexpr int RB = 3, N = 1 << RB;
    for (int gi = 0; gi < ngroups; ++gi) {
        const GroupCtl G = group_ctl_c(ggrp + gi);
        if (G.lds) {
            const YAO_CONST POp* rec = gops + G.op0;
            const double* m = mats + rec->mat;
            if (rec->k == 2) lds_op_fwd<double, 2>(lp, rec, m, t, th, nthr);
            else lds_op_fwd<double, 3>(lp, rec, m, t, th, nthr);
            __syncthreads();
            continue;
        }
        uint32_t ethr, er[N];
        group_index<RB>(G.rpos, t, th, ethr, er);
        double2 x[N];
#pragma unroll
        for (int r = 0; r < N; ++r) x[r] = lp[swz(ethr | er[r])];
        // The forward classes of op_variant on 3 register bits (see the forward kernel).
        auto apply = [&](const OpS<double>& o) __attribute__((always_inline)) {
            const double* mr = o.m;
            const double* mi = o.m + 4;
#define YAO_SF_CASE(J) \
    case J: pairs_dense_ctl_ip<J>(x, mr, mi, ethr, er, o.c.cmask, o.c.cval); break;
#define YAO_SF_FAST(J)                                                               \
    case 0 * RB + J: pairs_ip<J, OT_RX>(x, mr, mi); break;                           \
    case 1 * RB + J: pairs_ip<J, OT_DIAG>(x, mr, mi); break;                         \
    case 2 * RB + J: pairs_ip<J, OT_DENSE>(x, mr, mi); break;                        \
    case 3 * RB + J: pairs_cswap_ip<J>(x, ethr, er, o.c.cmask, o.c.cval); break;
            switch (o.c.var) {
                YAO_SF_FAST(0) YAO_SF_FAST(1) YAO_SF_FAST(2)
            default:
                switch (o.c.rpos) { YAO_SF_CASE(0) YAO_SF_CASE(1) default: YAO_SF_CASE(2) }
                break;
            }
#undef YAO_SF_FAST
#undef YAO_SF_CASE
        };
        const YAO_CONST POp* rec = gops + G.op0;
        OpS<double> A = load_op_c<double>(rec);
        for (int oi = 0; oi < G.nops; oi += 2) {
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), as in the forward kernel
            __builtin_amdgcn_sched_barrier(0);
            const OpS<double> B = load_op_c<double>(rec + oi + 1);
            apply(A);
            if (oi + 1 >= G.nops) break;
            __builtin_amdgcn_s_waitcnt(0xC07F);
            __builtin_amdgcn_sched_barrier(0);
            A = load_op_c<double>(rec + oi + 2);
            apply(B);
        }
#pragma unroll
        for (int r = 0; r < N; ++r) lp[swz(ethr | er[r])] = x[r];
        __syncthreads();
    }
}

// One workgroup per circuit of a batch whose state fits one tile (eq. apply-back and the
// outer-product gradient as in the reverse passes, all in LDS): psi = |0..0>, the forward
// program, psi_N to the state, lambda = H psi and the energy, then the reverse program with
// its gradients. LDS: psi (FP64) | lambda (FP64) | gradient partials.
__global__ __launch_bounds__(512, 1) void k_small_circuit(const SmallCircuit* items)
{
    constexpr int RB = 3, N = 1 << RB;
    extern __shared__ __align__(16) unsigned char smem[];
    const YAO_CONST SmallCircuit* it = cptr(items) + blockIdx.x;
    const int t = it->n;
    const int nthr = 1 << (t - RB);
    const int th = threadIdx.x;
    double2* lp = (double2*)smem;
    double2* ll = lp + (size_t(1) << t);
    double* red0 = (double*)(ll + (size_t(1) << t));
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const uint32_t e = (uint32_t)th + (uint32_t)r * nthr;
        lp[swz(e)] = make_double2(e == 0 ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    forward_groups3(lp, cptr(it->fops), cptr(it->fgroups), it->nfg, it->fmats, t, nthr, th);

    // Tile element e is basis state e (the tile holds qubits 0 .. n-1 in order).
    const YAO_CONST PGroup* hg = cptr(it->hgroups);
    const YAO_CONST PTerm* ht = cptr(it->hterms);
    const int nhg = it->nhg;
    const bool c64 = it->c64 != 0;
    double acc = 0;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const uint32_t e = (uint32_t)th + (uint32_t)r * nthr;
        const double2 a = lp[swz(e)];
        if (c64) ((float2*)it->state)[e] = make_float2((float)a.x, (float)a.y);
        else ((double2*)it->state)[e] = a;
        double orr = 0, oi = 0;
        for (int g = 0; g < nhg; ++g) {
            const uint32_t src = e ^ (uint32_t)hg[g].x;
            const double2 p = lp[swz(src)];
            double cr = 0, ci = 0;  // sum of c i^ny (-1)^{|src & z|}
            for (int k = hg[g].t0; k < hg[g].t1; ++k) {
                const double cc = (__popcll((uint64_t)src & ht[k].z) & 1) ? -ht[k].c : ht[k].c;
                switch (ht[k].ny & 3) {
                case 0: cr += cc; break;
                case 1: ci += cc; break;
                case 2: cr -= cc; break;
                default: ci -= cc; break;
                }
            }
            orr += cr * p.x - ci * p.y;
            oi += cr * p.y + ci * p.x;
        }
        ll[swz(e)] = make_double2(orr, oi);
        acc += a.x * orr + a.y * oi;
    }
    red0[th] = acc;
    __syncthreads();
    if (th == 0) {
        double sum = 0;
        for (int i = 0; i < nthr; ++i) sum += red0[i];
        *it->energy = sum;
    }
    __syncthreads();
    const GradOut go{it->grad, 1, 1, 0, 0};
    reverse_groups<double, true>(lp, ll, red0, cptr(it->rops), cptr(it->rgroups), it->rgroups, it->nrg, it->rmats, 0,
                                 t, 0, nthr, th, kMaxGroupSlots, go);
}

size_t small_circuit_lds_bytes(int n)
{
    const int nthr = 1 << (n - 3);
    return ((size_t)32 << n) + sizeof(double) * 2 * kMaxGroupSlots * (size_t)grad_entries(nthr, 0);
}

// ------------------------------------------------------------------------------ observables
// H psi and <psi|H|psi> in tile passes: the X-mask groups of the Pauli sum are split into
// passes whose masks lie inside one tile qubit set; a pass reads each tile of psi into LDS once
// and adds, for every element j of the tile and group g, c_t i^{ny} (-1)^{|(j ^ x) & z|}
// psi[j ^ x] over the group's terms (eq. expectation). Partners stay inside the tile, so the
// state is read once per pass instead of once per group.
constexpr int kObsRegBits = 3;  // elements per thread: 8
constexpr int kObsMaxTile = 12;
struct ObsGroupT {
    uint32_t x;  // X mask in tile-bit coordinates
    int t0, t1;  // terms
    int pad;
};
struct ObsTermT {
    double c;
    uint64_t zout;  // Z mask on qubits outside the tile (qubit coordinates)
    uint32_t zin;   // Z mask on the tile (tile-bit coordinates)
    int ny;         // number of Y factors
};

// One pass: groups[0 .. ng) over every tile. With OUT, (H psi) of these groups is written to
// a.lam (accumulate: added to what earlier passes wrote there). The pass's part of
// <psi|H|psi> per batch slot and tile goes to partial[b * W + pcol0 + tile].
template <typename RP, typename RO, bool OUT>
__global__ __launch_bounds__(512) void k_obs_pass(PassArgs a, const ObsGroupT* __restrict__ groups, int ng,
                                                  const ObsTermT* __restrict__ terms, int accumulate,
                                                  double* __restrict__ partial, int pcol0, int W)
{
    constexpr int RB = kObsRegBits, N = 1 << RB;
    using VP = vec2_t<RP>;
    using VO = vec2_t<RO>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = a.t, c = a.c;
    const int nthr = 1 << (t - RB);
    const int th = threadIdx.x;
    VP* lp = (VP*)smem;
    double* red = (double*)(smem + (sizeof(VP) << t));
    const TileCtx tc = tile_ctx<RB>(a, th);
    const VP* gp = (const VP*)z_psi(a);
    // Straight from global memory to LDS (a staging array stayed in scratch memory).
#pragma unroll
    for (int r = 0; r < N; ++r) lp[swz((uint32_t)th + (uint32_t)r * nthr)] = gp[tile_off<RB>(a, tc, r)];
    __syncthreads();
    const YAO_CONST ObsGroupT* gq = cptr(groups);
    const YAO_CONST ObsTermT* tq = cptr(terms);
    VO* go = (VO*)z_lam(a);
    partial = z_partial(a, partial);
    // Table entries are read once per thread (scalar loads) and applied to the thread's 16
    // elements: group by group, term by term.
    double orr[N], oi[N];
#pragma unroll
    for (int r = 0; r < N; ++r) orr[r] = oi[r] = 0;
    for (int g = 0; g < ng; ++g) {
        const uint32_t x = gq[g].x;
        const int t0 = gq[g].t0, t1 = gq[g].t1;
        VP p[N];
#pragma unroll
        for (int r = 0; r < N; ++r) p[r] = lp[swz(((uint32_t)th + (uint32_t)r * nthr) ^ x)];
        for (int k = t0; k < t1; ++k) {
            const uint32_t zin = tq[k].zin;
            const int ny = tq[k].ny;
            // i^ny and the sign of the Z bits outside the tile, folded into the coefficient.
            double cb = (__popcll(tc.base & tq[k].zout) & 1) ? -tq[k].c : tq[k].c;
            if (ny & 2) cb = -cb;
            if (ny & 1) {
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    const uint32_t src = ((uint32_t)th + (uint32_t)r * nthr) ^ x;
                    const double cc = (__popc(src & zin) & 1) ? -cb : cb;
                    orr[r] = fma(-cc, (double)p[r].y, orr[r]);
                    oi[r] = fma(cc, (double)p[r].x, oi[r]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    const uint32_t src = ((uint32_t)th + (uint32_t)r * nthr) ^ x;
                    const double cc = (__popc(src & zin) & 1) ? -cb : cb;
                    orr[r] = fma(cc, (double)p[r].x, orr[r]);
                    oi[r] = fma(cc, (double)p[r].y, oi[r]);
                }
            }
        }
    }
    double acc = 0;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const VP ae = lp[swz((uint32_t)th + (uint32_t)r * nthr)];
        acc += (double)ae.x * orr[r] + (double)ae.y * oi[r];
        if constexpr (OUT) {
            if (tc.bvalid) {
                const uint64_t off = tile_off<RB>(a, tc, r);
                double wr = orr[r], wi = oi[r];
                if (accumulate) {
                    const VO prev = go[off];
                    wr += (double)prev.x;
                    wi += (double)prev.y;
                }
                go[off] = mkv<VO, RO>((RO)wr, (RO)wi);
            }
        }
    }
    // Per batch slot of the tile: row sums, then the rows in order.
    const int Bc = 1 << c;
    const int E = grad_entries(nthr, c);
    if (nthr >= 16) {
        acc = row_sum(acc, c);
        if ((th & 15) < Bc) red[(th >> 4) * Bc + (th & 15)] = acc;
    } else {
        red[th] = acc;
    }
    __syncthreads();
    if (th < Bc) {
        double sum = 0;
        for (int k = th; k < E; k += Bc) sum += red[k];
        const int b = (int)(blockIdx.y << c) + th;
        if (b < a.B) partial[(uint64_t)b * W + pcol0 + blockIdx.x] = sum;
    }
}

// Raise each pass kernel's dynamic LDS limit to the CU's 160 KiB, once per kernel.
template <typename K> int set_lds_limit(K kernel)
{
    static std::mutex mu;
    static std::vector<const void*> done;
    std::lock_guard<std::mutex> lk(mu);
    for (const void* k : done)
        if (k == (const void*)kernel) return 0;
    YAO_HIP(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    done.push_back((const void*)kernel);
    return 0;
}

// One-qubit matrix of a gate kind at angle th: rotations exp(-i th S / 2), shift(th) =
// diag(1, e^{i th}), and the fixed Pauli, Hadamard, S and T gates (the same definitions as the
// host's gate matrices).
__device__ void gate2(int kind, double th, double (&r)[4], double (&i)[4])
{
    const double h = 0.70710678118654752440;
    for (int e = 0; e < 4; ++e) r[e] = i[e] = 0.0;
    double sn, cs;
    switch (kind) {
    case YAO_X: r[1] = r[2] = 1.0; break;
    case YAO_Y: i[1] = -1.0; i[2] = 1.0; break;
    case YAO_Z: r[0] = 1.0; r[3] = -1.0; break;
    case YAO_H: r[0] = r[1] = r[2] = h; r[3] = -h; break;
    case YAO_S: r[0] = 1.0; i[3] = 1.0; break;
    case YAO_SDAG: r[0] = 1.0; i[3] = -1.0; break;
    case YAO_T: r[0] = 1.0; r[3] = h; i[3] = h; break;
    case YAO_TDAG: r[0] = 1.0; r[3] = h; i[3] = -h; break;
    case YAO_SHIFT: sincos(th, &sn, &cs); r[0] = 1.0; r[3] = cs; i[3] = sn; break;
    case YAO_RX: sincos(0.5 * th, &sn, &cs); r[0] = r[3] = cs; i[1] = i[2] = -sn; break;
    case YAO_RY: sincos(0.5 * th, &sn, &cs); r[0] = r[3] = cs; r[1] = -sn; r[2] = sn; break;
    case YAO_RZ: sincos(0.5 * th, &sn, &cs); r[0] = r[3] = cs; i[0] = -sn; i[3] = sn; break;
    default: r[0] = r[3] = 1.0; break;
    }
}

// Parameter binding: one thread per bound record multiplies its factors (in application
// order) and writes the matrix into the record (see BindRec).
// The matrix of one bound record: the product of its factors (gate kind and angle), written
// as U (forward, float or double) or U^dagger (reverse) into the record.
__device__ void bind_one(POp* __restrict__ ops, const BindRec br, const BindFac* __restrict__ facs,
                         const double* __restrict__ params)
{
    double ar[4] = {1.0, 0.0, 0.0, 1.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
    for (int f = 0; f < br.nf; ++f) {
        const BindFac x = facs[br.f0 + f];
        double gr[4], gi[4];
        gate2(x.kind, x.param >= 0 ? params[x.param] : x.theta, gr, gi);
        double nr[4], ni[4];
        for (int row = 0; row < 2; ++row)
            for (int col = 0; col < 2; ++col) {
                const int o = 2 * row + col;
                nr[o] = gr[2 * row] * ar[col] - gi[2 * row] * ai[col] + gr[2 * row + 1] * ar[2 + col] -
                        gi[2 * row + 1] * ai[2 + col];
                ni[o] = gr[2 * row] * ai[col] + gi[2 * row] * ar[col] + gr[2 * row + 1] * ai[2 + col] +
                        gi[2 * row + 1] * ar[2 + col];
            }
        for (int e = 0; e < 4; ++e) {
            ar[e] = nr[e];
            ai[e] = ni[e];
        }
    }
    if (br.mode == 2) {  // U^dagger
        double t = ar[1];
        ar[1] = ar[2];
        ar[2] = t;
        t = ai[1];
        ai[1] = -ai[2];
        ai[2] = -t;
        ai[0] = -ai[0];
        ai[3] = -ai[3];
    }
    POp& op = ops[br.op];
    if (br.mode == 0) {
        float* u = (float*)op.u;
        for (int e = 0; e < 4; ++e) {
            u[e] = (float)ar[e];
            u[4 + e] = (float)ai[e];
        }
    } else {
        for (int e = 0; e < 4; ++e) {
            op.u[e] = ar[e];
            op.u[4 + e] = ai[e];
        }
        if (br.mode == 2 && op.var / kRegBitsBwd == 1) split_diag_phase(op.u);
    }
}

__global__ void k_bind(POp* __restrict__ ops, const BindRec* __restrict__ binds, int nb,
                       const BindFac* __restrict__ facs, const double* __restrict__ params)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    bind_one(ops, binds[b], facs, params);
}

// Many programs at once: job blockIdx.y, record blockIdx.x * blockDim.x + threadIdx.x.
__global__ void k_bind_jobs(const BindJob* __restrict__ jobs)
{
    const BindJob j = jobs[blockIdx.y];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= j.nb) return;
    bind_one(j.ops, j.binds[b], j.facs, j.params);
}

}  // namespace

int launch_bind_jobs(const BindJob* jobs, int njobs, int max_nb)
{
    if (njobs <= 0 || max_nb <= 0) return 0;
    if (njobs > 65535) return set_error(YAO_EINVAL, "%d bind jobs in one launch", njobs);
    k_bind_jobs<<<dim3((max_nb + 255) / 256, njobs), 256, 0, stream()>>>(jobs);
    YAO_HIP(hipGetLastError());
    return 0;
}

int launch_small_circuits(const SmallCircuit* items, int count, int n)
{
    if (count <= 0) return 0;
    if (n < 5 || n > kSmallMaxQubits) return set_error(YAO_EINVAL, "small-circuit kernel takes 5..%d qubits, not %d",
                                                       kSmallMaxQubits, n);
    YAO_TRY(set_lds_limit(k_small_circuit));
    k_small_circuit<<<count, 1 << (n - 3), small_circuit_lds_bytes(n), stream()>>>(items);
    YAO_HIP(hipGetLastError());
    return 0;
}

int launch_bind(POp* ops, const BindRec* binds, int nbinds, const BindFac* facs, const double* params)
{
    if (nbinds <= 0) return 0;
    k_bind<<<(nbinds + 255) / 256, 256, 0, stream()>>>(ops, binds, nbinds, facs, params);
    YAO_HIP(hipGetLastError());
    return 0;
}

// Raise the dynamic LDS limit of every pass kernel ahead of a graph capture.
int prepare_pass_kernels()
{
    YAO_TRY(set_lds_limit(k_pass_fwd<float>));
    YAO_TRY(set_lds_limit(k_pass_fwd<double>));
    YAO_TRY(set_lds_limit(k_pass_bwd<float, true>));
    YAO_TRY(set_lds_limit(k_pass_bwd<float, false>));
    YAO_TRY(set_lds_limit(k_pass_bwd<double, true>));
    YAO_TRY(set_lds_limit(k_pass_bwd<double, false>));
    YAO_TRY(set_lds_limit(k_small_circuit));
    return 0;
}

size_t pass_lds_bytes(bool bwd, int t, int c, int psi_bytes, int lam_bytes, int dm_words, int mslots)
{
    if (!bwd) return ((size_t)psi_bytes << t) + 16 * (size_t)dm_words;
    const int nthr = 1 << (t - kRegBitsBwd);
    return ((size_t)(16 + lam_bytes) << t) + sizeof(double) * 2 * mslots * (size_t)grad_entries(nthr, c);
}

// The tile geometry of a pass: tile qubits (ascending), the qubits outside the tile, and the
// per-register offsets of the load mapping for RB register bits.
static void tile_args(PassArgs& a, int n, int B, int c, int t, const std::vector<int>& tile_qubits, int RB,
                      const std::vector<int>& store_src = {})
{
    // Store permutation (identity when store_src is empty).
    for (int i = 0; i < t; ++i) {
        const int src = store_src.empty() ? i : store_src[i];
        if (i < t - RB) a.ssrc[i] = src;
    }
    for (int r = 0; r < (1 << RB); ++r) {
        uint32_t v = 0;
        for (int j = 0; j < RB; ++j)
            if ((r >> j) & 1) v |= 1u << (store_src.empty() ? t - RB + j : store_src[t - RB + j]);
        a.sreg[r] = v;
    }
    a.n = n;
    a.B = B;
    a.c = c;
    a.t = t;
    a.ntq = (int)tile_qubits.size();
    uint64_t T = 0;
    for (int j = 0; j < a.ntq; ++j) {
        a.tile_qubits[j] = tile_qubits[j];
        T |= uint64_t(1) << tile_qubits[j];
    }
    a.nnt = 0;
    for (int q = 0; q < n; ++q)
        if (!((T >> q) & 1)) a.nontile_qubits[a.nnt++] = q;
    const int j0 = t - RB - c;
    for (int r = 0; r < (1 << RB); ++r) {
        uint64_t d = 0;
        for (int rb = 0; rb < RB; ++rb)
            if ((r >> rb) & 1) d |= uint64_t(1) << tile_qubits[j0 + rb];
        a.rofs[r] = d * (uint64_t)B;
    }
    a.ntiles = 1 << a.nnt;
}

int launch_pass(bool bwd, int psi_dtype, int lam_dtype, void* psi, void* lam, const POp* ops, const PGroupDesc* groups,
                const double* mats, double* gpartial, int pstride, int mslots, int n, int B, int c, int t, int group0,
                int ngroups, const std::vector<int>& tile_qubits, const std::vector<int>& store_src, double flops,
                int op_first, int nops, const double* dmats, int dm_words)
{
    if (bwd && (mslots < 1 || mslots > kMaxGroupSlots))
        return set_error(YAO_EINVAL, "%d gradient slots per register group (1 .. %d)", mslots, kMaxGroupSlots);
    if (!store_src.empty() && (int)store_src.size() != t)
        return set_error(YAO_EINVAL, "store permutation of %zu bits for a tile of %d", store_src.size(), t);
    if (!store_src.empty()) {
        uint32_t seen = 0;
        for (int v : store_src) {
            if (v < 0 || v >= t || ((seen >> v) & 1)) return set_error(YAO_EINVAL, "store permutation is not one");
            seen |= 1u << v;
        }
        for (int b = 0; b < c; ++b)
            if (store_src[b] != b) return set_error(YAO_EINVAL, "store permutation moves a batch bit");
    }
    if (nops > kMaxPassOps || ngroups > kMaxPassOps)
        return set_error(YAO_EINVAL, "pass of %d ops exceeds %d", nops, kMaxPassOps);
    const int dm_max = bwd ? 0 : kMaxPassDense * 256;  // 4 KiB per block in every layout
    if (dm_words < 0 || dm_words > dm_max)
        return set_error(YAO_EINVAL, "pass carries %d words of dense matrices (at most %d)", dm_words, dm_max);
    PassArgs a;
    memset(&a, 0, sizeof(a));
    a.psi = psi;
    a.lam = lam;
    a.ops = ops + op_first;
    a.groups = groups + group0;
    a.mats = mats;
    a.gpartial = gpartial;
    a.dmats = (const uint4*)dmats;
    a.ndm = dm_words;
    a.ngroups = ngroups;
    a.nops = nops;
    a.mslots = mslots;
    a.zs = g_zbatch.zs;
    a.op_first = op_first;
    tile_args(a, n, B, c, t, tile_qubits, bwd ? kRegBitsBwd : kRegBitsFwd, store_src);
    a.pstride = pstride > a.ntiles ? pstride : a.ntiles;
    const int Bc = 1 << c;
    const int RBk = bwd ? kRegBitsBwd : kRegBitsFwd;
    // The kernels are compiled for at most 512 threads per block (one tile, 2^(t - RB) threads).
    if (t - RBk < 0 || t - RBk > 9) return set_error(YAO_EINVAL, "tile of 2^%d does not fit 1 .. 512 threads", t);
    const int nz = g_zbatch.zs ? g_zbatch.nz : 1;
    dim3 grid(a.ntiles, (B + Bc - 1) / Bc, nz);
    dim3 block(1 << (t - RBk));
    const int pb = bwd ? 16 : (psi_dtype == YAO_C64 ? 8 : 16);
    const int lb = bwd ? (lam_dtype == YAO_C64 ? 8 : 16) : 0;
    const size_t lds = pass_lds_bytes(bwd, t, c, pb, lb, bwd ? 0 : dm_words, mslots);
    if (lds > 160 * 1024) return set_error(YAO_EINVAL, "tile of 2^%d needs %zu bytes of LDS", t, lds);
    hipStream_t st = stream();
    const int pi = prof_begin(bwd ? YAO_KF_PASS_BWD : YAO_KF_PASS_FWD);
    if (!bwd) {
        if (psi_dtype == YAO_C64) {
            YAO_TRY(set_lds_limit(k_pass_fwd<float>));
            k_pass_fwd<float><<<grid, block, lds, st>>>(a);
        } else {
            YAO_TRY(set_lds_limit(k_pass_fwd<double>));
            k_pass_fwd<double><<<grid, block, lds, st>>>(a);
        }
    } else {
        if (lam_dtype == YAO_C64) {
            if (c == 0) {
                YAO_TRY(set_lds_limit(k_pass_bwd<float, true>));
                k_pass_bwd<float, true><<<grid, block, lds, st>>>(a);
            } else {
                YAO_TRY(set_lds_limit(k_pass_bwd<float, false>));
                k_pass_bwd<float, false><<<grid, block, lds, st>>>(a);
            }
        } else {
            if (c == 0) {
                YAO_TRY(set_lds_limit(k_pass_bwd<double, true>));
                k_pass_bwd<double, true><<<grid, block, lds, st>>>(a);
            } else {
                YAO_TRY(set_lds_limit(k_pass_bwd<double, false>));
                k_pass_bwd<double, false><<<grid, block, lds, st>>>(a);
            }
        }
    }
    prof_end(pi, 2.0 * (double)(uint64_t(1) << n) * B * (pb + lb) * nz, flops * nz);
    YAO_HIP(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------------- observable passes
namespace {

struct ObsPass {
    std::vector<int> tile_qubits;
    int g0 = 0, g1 = 0;  // groups of the pass in the device table
};
struct ObsPlan {
    bool ok = false;  // false: an X mask is wider than a tile (the observable takes the
                      // per-group kernels)
    int c = 0, t = 0;
    std::vector<ObsPass> passes;
    ObsGroupT* dgroups = nullptr;
    ObsTermT* dterms = nullptr;
};
using ObsKey = std::tuple<const yao_pauli_sum*, int, int, int>;  // h, n, B, dtype
std::map<ObsKey, ObsPlan*> g_obs;
std::mutex g_obs_mu;

// Group the terms by X mask, then put each group in the first pass whose tile qubits can take
// its mask (first fit, over tiles of t - c qubits that keep the lowest qubits for contiguous
// rows), and fill every pass's tile with the lowest unused qubits.
ObsPlan* obs_plan(const yao_pauli_sum* h, int n, int B, int dtype)
{
    std::lock_guard<std::mutex> lk(g_obs_mu);
    const ObsKey key{h, n, B, dtype};
    auto it = g_obs.find(key);
    if (it != g_obs.end()) return it->second;
    const int lb = ilog2_ceil((uint64_t)B);
    const int c = lb < 3 ? lb : 3;
    const int tq = std::min(n, kObsMaxTile - c);
    const int L = std::max(0, std::min((dtype == YAO_C64 ? 4 : 3) - c, tq));
    std::vector<uint64_t> xs;
    for (size_t k = 0; k < h->coef.size(); ++k) {
        bool seen = false;
        for (uint64_t x : xs) seen |= x == h->x[k];
        if (!seen) xs.push_back(h->x[k]);
    }
    const uint64_t low = L > 0 ? ((uint64_t(1) << L) - 1) : 0;
    ObsPlan* P = new ObsPlan;
    P->c = c;
    P->t = c + tq;
    for (uint64_t x : xs)
        if (__builtin_popcountll(x) > tq) {
            g_obs[key] = P;
            return P;
        }
    std::vector<uint64_t> T;                // qubits of each pass
    std::vector<std::vector<uint64_t>> gx;  // X masks of each pass
    for (uint64_t x : xs) {
        size_t p = 0;
        while (p < T.size() && __builtin_popcountll(T[p] | x) > tq) ++p;
        if (p == T.size()) {
            // A mask too wide for a tile with the low qubits fixed drops them.
            T.push_back(__builtin_popcountll(low | x) <= tq ? low : 0);
            gx.emplace_back();
        }
        T[p] |= x;
        gx[p].push_back(x);
    }
    std::vector<ObsGroupT> hg;
    std::vector<ObsTermT> ht;
    for (size_t p = 0; p < T.size(); ++p) {
        uint64_t Tp = T[p];
        for (int q = 0; q < n && __builtin_popcountll(Tp) < tq; ++q) Tp |= uint64_t(1) << q;
        ObsPass ps;
        for (int q = 0; q < n; ++q)
            if ((Tp >> q) & 1) ps.tile_qubits.push_back(q);
        auto to_tile = [&](uint64_t m) {
            uint32_t r = 0;
            for (size_t j = 0; j < ps.tile_qubits.size(); ++j)
                if ((m >> ps.tile_qubits[j]) & 1) r |= 1u << (c + (int)j);
            return r;
        };
        ps.g0 = (int)hg.size();
        for (uint64_t x : gx[p]) {
            ObsGroupT g;
            g.x = to_tile(x);
            g.t0 = (int)ht.size();
            for (size_t k = 0; k < h->coef.size(); ++k) {
                if (h->x[k] != x) continue;
                ObsTermT tt;
                tt.c = h->coef[k];
                tt.zin = to_tile(h->z[k]);
                tt.zout = h->z[k] & ~Tp;
                tt.ny = __builtin_popcountll(h->x[k] & h->z[k]);
                ht.push_back(tt);
            }
            g.t1 = (int)ht.size();
            g.pad = 0;
            hg.push_back(g);
        }
        ps.g1 = (int)hg.size();
        P->passes.push_back(ps);
    }
    if (hipMalloc((void**)&P->dgroups, sizeof(ObsGroupT) * (hg.size() + 1)) != hipSuccess ||
        hipMalloc((void**)&P->dterms, sizeof(ObsTermT) * (ht.size() + 1)) != hipSuccess ||
        hipMemcpy(P->dgroups, hg.data(), sizeof(ObsGroupT) * hg.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P->dterms, ht.data(), sizeof(ObsTermT) * ht.size(), hipMemcpyHostToDevice) != hipSuccess) {
        if (P->dgroups) (void)hipFree(P->dgroups);
        if (P->dterms) (void)hipFree(P->dterms);
        delete P;
        set_error(YAO_ENOMEM, "observable pass tables");
        return nullptr;
    }
    P->ok = true;
    g_obs[key] = P;
    return P;
}

template <typename RP, typename RO, bool OUT> int obs_launch_one(const PassArgs& a, dim3 grid, int nthr, size_t lds,
                                                                 const ObsPlan* P, const ObsPass& ps, int accumulate,
                                                                 double* partial, int pcol0, int W)
{
    YAO_TRY(set_lds_limit(k_obs_pass<RP, RO, OUT>));
    k_obs_pass<RP, RO, OUT><<<grid, nthr, lds, stream()>>>(a, P->dgroups + ps.g0, ps.g1 - ps.g0, P->dterms, accumulate,
                                                           partial, pcol0, W);
    YAO_HIP(hipGetLastError());
    return 0;
}

}  // namespace

bool obs_passes_ok(const yao_pauli_sum* h, int n, int B, int dtype)
{
    if (n < kObsRegBits + 1) return false;
    const ObsPlan* P = obs_plan(h, n, B, dtype);
    return P && P->ok;
}

int obs_tile_qubits(const yao_pauli_sum* h, int n, int B, int dtype)
{
    const ObsPlan* P = obs_plan(h, n, B, dtype);
    return P && P->ok ? P->t - P->c : 0;
}

size_t obs_partial_doubles(const yao_pauli_sum* h, int n, int B, int dtype)
{
    const ObsPlan* P = obs_plan(h, n, B, dtype);
    if (!P || !P->ok) return 0;
    return (size_t)B * P->passes.size() * (size_t(1) << (n - (P->t - P->c)));
}

// H psi into out (out == nullptr: the energy only) and the pass/tile partials of the energy
// in partial[b * W + column]; *W receives the row length.
int launch_obs_passes(const void* psi, int dtype, void* out, int out_dtype, int n, int B, const yao_pauli_sum* h,
                      double* partial, int* W)
{
    const ObsPlan* P = obs_plan(h, n, B, dtype);
    if (!P) return YAO_ENOMEM;
    if (!P->ok) return set_error(YAO_EINVAL, "observable has an X mask wider than a tile");
    const int t = P->t, c = P->c;
    const int nthr = 1 << (t - kObsRegBits);
    const int ntiles = 1 << (n - (t - c));
    *W = (int)P->passes.size() * ntiles;
    const int Bc = 1 << c;
    const dim3 grid(ntiles, (B + Bc - 1) / Bc, g_zbatch.zs ? g_zbatch.nz : 1);
    const size_t lds = ((size_t)(dtype == YAO_C64 ? 8 : 16) << t) + sizeof(double) * (size_t)grad_entries(nthr, c);
    for (size_t p = 0; p < P->passes.size(); ++p) {
        const ObsPass& ps = P->passes[p];
        PassArgs a;
        memset(&a, 0, sizeof(a));
        a.psi = const_cast<void*>(psi);
        a.lam = out;
        a.zs = g_zbatch.zs;
        tile_args(a, n, B, c, t, ps.tile_qubits, kObsRegBits);
        const int acc = p > 0 ? 1 : 0, col = (int)p * ntiles;
        if (!out) {
            if (dtype == YAO_C64) YAO_TRY((obs_launch_one<float, float, false>(a, grid, nthr, lds, P, ps, 0, partial, col, *W)));
            else YAO_TRY((obs_launch_one<double, double, false>(a, grid, nthr, lds, P, ps, 0, partial, col, *W)));
        } else if (dtype == YAO_C64 && out_dtype == YAO_C64) {
            YAO_TRY((obs_launch_one<float, float, true>(a, grid, nthr, lds, P, ps, acc, partial, col, *W)));
        } else if (dtype == YAO_C64) {
            YAO_TRY((obs_launch_one<float, double, true>(a, grid, nthr, lds, P, ps, acc, partial, col, *W)));
        } else if (out_dtype == YAO_C64) {
            YAO_TRY((obs_launch_one<double, float, true>(a, grid, nthr, lds, P, ps, acc, partial, col, *W)));
        } else {
            YAO_TRY((obs_launch_one<double, double, true>(a, grid, nthr, lds, P, ps, acc, partial, col, *W)));
        }
    }
    return 0;
}

void drop_obs_plans(const yao_pauli_sum* h)
{
    std::lock_guard<std::mutex> lk(g_obs_mu);
    for (auto it = g_obs.begin(); it != g_obs.end();) {
        if (std::get<0>(it->first) == h) {
            (void)hipDeviceSynchronize();
            if (it->second->dgroups) (void)hipFree(it->second->dgroups);
            if (it->second->dterms) (void)hipFree(it->second->dterms);
            delete it->second;
            it = g_obs.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace yao
