// Fused tile-pass kernels: forward sweep and reversible adjoint sweep.
//
// One workgroup owns one tile: 2^t elements = Bc = 2^c consecutive batch slots (lowest tile
// bits) x the 2^(t-c) amplitudes spanned by the pass's tile qubits, with every other qubit
// fixed by the tile id. The tile is staged in LDS (XOR-swizzled), then processed in register
// groups: each of the 2^(t-kRegBits) threads holds the 2^kRegBits elements that differ only in
// the group's register bits, so a one-qubit gate on a register bit is pure ALU work on pairs
// of registers. Gates of 2 or 3 qubits are applied directly in LDS. The backward kernel holds
// psi (complex128, the FP64 uncompute) and lambda side by side and, per gate, first adds
// 2 Re <lambda|M|psi> over the tile (eq. outer-product reduced to the parameter) and then
// applies U^dagger to both (eq. apply-back).
#include "fused.h"

namespace yao {

namespace {

constexpr int R = 1 << kRegBits;

struct PassArgs {
    void* psi;
    void* lam;
    const POp* ops;
    const PGroupDesc* groups;
    const double* mats;
    double* gpartial;       // [slot][B][ntiles]
    int n, B, c, t;
    int group0, ngroups;
    int ntq, nnt;
    int ntiles;
    int pstride;            // row stride of gpartial (>= ntiles)
    int tile_qubits[kMaxTileBits];
    int nontile_qubits[40];
};

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

// out = m0 * a + m1 * b (complex), in real type RR.
template <typename RR, typename V>
__device__ __forceinline__ V lin2(RR m0r, RR m0i, RR m1r, RR m1i, const V& a, const V& b)
{
    RR x = m0r * a.x;
    x = fma(-m0i, a.y, x);
    x = fma(m1r, b.x, x);
    x = fma(-m1i, b.y, x);
    RR y = m0r * a.y;
    y = fma(m0i, a.x, y);
    y = fma(m1r, b.y, y);
    y = fma(m1i, b.x, y);
    return mkv<V, RR>(x, y);
}

// Apply a one-qubit matrix of structure TYPE to the pair (a, b); m = {re[4], im[4]}.
template <int TYPE, typename RR, typename V>
__device__ __forceinline__ void apply_pair(const RR* mr, const RR* mi, V& a, V& b)
{
    if constexpr (TYPE == OT_SWAP) {
        V t = a;
        a = b;
        b = t;
    } else if constexpr (TYPE == OT_ANTI) {
        V na = mkv<V, RR>(mr[1] * b.x - mi[1] * b.y, mr[1] * b.y + mi[1] * b.x);
        V nb = mkv<V, RR>(mr[2] * a.x - mi[2] * a.y, mr[2] * a.y + mi[2] * a.x);
        a = na;
        b = nb;
    } else if constexpr (TYPE == OT_DIAG1) {
        b = mkv<V, RR>(mr[3] * b.x - mi[3] * b.y, mr[3] * b.y + mi[3] * b.x);
    } else if constexpr (TYPE == OT_DIAG) {
        a = mkv<V, RR>(mr[0] * a.x - mi[0] * a.y, mr[0] * a.y + mi[0] * a.x);
        b = mkv<V, RR>(mr[3] * b.x - mi[3] * b.y, mr[3] * b.y + mi[3] * b.x);
    } else if constexpr (TYPE == OT_REAL) {
        V na = mkv<V, RR>(fma(mr[0], a.x, mr[1] * b.x), fma(mr[0], a.y, mr[1] * b.y));
        V nb = mkv<V, RR>(fma(mr[2], a.x, mr[3] * b.x), fma(mr[2], a.y, mr[3] * b.y));
        a = na;
        b = nb;
    } else if constexpr (TYPE == OT_RX) {
        // [[c, i s'], [i s', c]] with c = mr[0], s' = mi[1] = mi[2]
        const RR cc = mr[0], ss = mi[1];
        V na = mkv<V, RR>(fma(cc, a.x, -ss * b.y), fma(cc, a.y, ss * b.x));
        V nb = mkv<V, RR>(fma(cc, b.x, -ss * a.y), fma(cc, b.y, ss * a.x));
        a = na;
        b = nb;
    } else {
        V na = lin2<RR>(mr[0], mi[0], mr[1], mi[1], a, b);
        V nb = lin2<RR>(mr[2], mi[2], mr[3], mi[3], a, b);
        a = na;
        b = nb;
    }
}

// 2 Re( conj(l0) (M p)_0 + conj(l1) (M p)_1 ) for the generator class GEN.
template <int GEN, typename VL>
__device__ __forceinline__ double grad_pair(const double* mr, const double* mi, const double2& p0, const double2& p1,
                                            const VL& l0, const VL& l1)
{
    const double l0x = l0.x, l0y = l0.y, l1x = l1.x, l1y = l1.y;
    if constexpr (GEN == GEN_X) {  // M = -(i/2) X: Im(conj(l0) p1 + conj(l1) p0)
        return l0x * p1.y - l0y * p1.x + l1x * p0.y - l1y * p0.x;
    } else if constexpr (GEN == GEN_Y) {  // M = -(i/2) Y = [[0, -1/2], [1/2, 0]]
        return l1x * p0.x + l1y * p0.y - l0x * p1.x - l0y * p1.y;
    } else if constexpr (GEN == GEN_Z) {  // M = diag(-i/2, i/2)
        return (l0x * p0.y - l0y * p0.x) - (l1x * p1.y - l1y * p1.x);
    } else if constexpr (GEN == GEN_P1) {  // M = diag(0, i)
        return -2.0 * (l1x * p1.y - l1y * p1.x);
    } else {
        double m0x = mr[0] * p0.x - mi[0] * p0.y + mr[1] * p1.x - mi[1] * p1.y;
        double m0y = mr[0] * p0.y + mi[0] * p0.x + mr[1] * p1.y + mi[1] * p1.x;
        double m1x = mr[2] * p0.x - mi[2] * p0.y + mr[3] * p1.x - mi[3] * p1.y;
        double m1y = mr[2] * p0.y + mi[2] * p0.x + mr[3] * p1.y + mi[3] * p1.x;
        return 2.0 * (l0x * m0x + l0y * m0y + l1x * m1x + l1y * m1y);
    }
}

// One one-qubit op of structure TYPE on register bit J of every thread's R elements.
template <int J, bool CTRL, int TYPE, typename RR, typename V>
__device__ __forceinline__ void pairs_apply(V (&x)[R], const RR* mr, const RR* mi, uint32_t ethr,
                                            const uint32_t (&er)[R], uint32_t cmask, uint32_t cval)
{
#pragma unroll
    for (int a = 0; a < R; ++a) {
        if (a & (1 << J)) continue;
        if (CTRL) {
            if (((ethr | er[a]) & cmask) != cval) continue;
        }
        apply_pair<TYPE, RR>(mr, mi, x[a], x[a + (1 << J)]);
    }
}

template <int J, bool CTRL, typename RR, typename V>
__device__ __forceinline__ void op_apply(V (&x)[R], int type, const RR* mr, const RR* mi, uint32_t ethr,
                                         const uint32_t (&er)[R], uint32_t cmask, uint32_t cval)
{
    switch (type) {
    case OT_SWAP: pairs_apply<J, CTRL, OT_SWAP, RR>(x, mr, mi, ethr, er, cmask, cval); break;
    case OT_ANTI: pairs_apply<J, CTRL, OT_ANTI, RR>(x, mr, mi, ethr, er, cmask, cval); break;
    case OT_DIAG1: pairs_apply<J, CTRL, OT_DIAG1, RR>(x, mr, mi, ethr, er, cmask, cval); break;
    case OT_DIAG: pairs_apply<J, CTRL, OT_DIAG, RR>(x, mr, mi, ethr, er, cmask, cval); break;
    case OT_REAL: pairs_apply<J, CTRL, OT_REAL, RR>(x, mr, mi, ethr, er, cmask, cval); break;
    case OT_RX: pairs_apply<J, CTRL, OT_RX, RR>(x, mr, mi, ethr, er, cmask, cval); break;
    default: pairs_apply<J, CTRL, OT_DENSE, RR>(x, mr, mi, ethr, er, cmask, cval); break;
    }
}

template <int J, bool CTRL, int GEN, typename VL>
__device__ __forceinline__ double pairs_grad(const double2 (&x)[R], const VL (&y)[R], const double* mr,
                                             const double* mi, uint32_t ethr, const uint32_t (&er)[R], uint32_t cmask,
                                             uint32_t cval)
{
    double g = 0;
#pragma unroll
    for (int a = 0; a < R; ++a) {
        if (a & (1 << J)) continue;
        if (CTRL) {
            if (((ethr | er[a]) & cmask) != cval) continue;
        }
        g += grad_pair<GEN, VL>(mr, mi, x[a], x[a + (1 << J)], y[a], y[a + (1 << J)]);
    }
    return g;
}

template <int J, bool CTRL, typename VL>
__device__ __forceinline__ double op_grad(const double2 (&x)[R], const VL (&y)[R], int gen, const double* mr,
                                          const double* mi, uint32_t ethr, const uint32_t (&er)[R], uint32_t cmask,
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

// Backward: gradient partial with (psi_{k+1}, lambda_{k+1}), then U^dagger on both.
template <int J, bool CTRL, typename VL>
__device__ __forceinline__ double op_bwd(double2 (&x)[R], VL (&y)[R], int type, int gen, bool grad, const double* m,
                                         uint32_t ethr, const uint32_t (&er)[R], uint32_t cmask, uint32_t cval)
{
    using RL = decltype(VL().x);
    double g = 0;
    if (grad) g = op_grad<J, CTRL, VL>(x, y, gen, m + 8, m + 12, ethr, er, cmask, cval);
    RL lr[4], li[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        lr[q] = (RL)m[q];
        li[q] = (RL)m[4 + q];
    }
    op_apply<J, CTRL, double>(x, type, m, m + 4, ethr, er, cmask, cval);
    op_apply<J, CTRL, RL>(y, type, lr, li, ethr, er, cmask, cval);
    return g;
}

// Sum over the lanes of a wave that share a batch slot (lane & (Bc-1)).
__device__ __forceinline__ double wave_sum_by_slot(double v, int Bc, int nthr)
{
    for (int off = (nthr < 64 ? nthr : 64) >> 1; off >= Bc; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename RP, typename RL, bool BWD>
__global__ __launch_bounds__(512) void k_pass(PassArgs a)
{
    using VP = vec2_t<RP>;
    using VL = vec2_t<RL>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = a.t, c = a.c;
    const int nthr = 1 << (t - kRegBits);
    const int th = threadIdx.x;
    const int Bc = 1 << c;
    const int lane = th & 63, wave = th >> 6;
    const int nwaves = (nthr + 63) >> 6;
    VP* lp = (VP*)smem;
    VL* ll = (VL*)(smem + (sizeof(VP) << t));
    double* red = (double*)(smem + ((sizeof(VP) + (BWD ? sizeof(VL) : 0)) << t));

    uint64_t base = 0;
    {
        const uint64_t tid = blockIdx.x;
        for (int j = 0; j < a.nnt; ++j) base |= ((tid >> j) & uint64_t(1)) << a.nontile_qubits[j];
    }
    const int b0 = blockIdx.y * Bc;
    const int bl = th & (Bc - 1);
    const bool bvalid = b0 + bl < a.B;
    const uint64_t B = (uint64_t)a.B;

    // ---------------------------------------------------------------- load the tile
    // element e = th + r * nthr: batch bits from th, qubit bits deposited onto tile qubits.
    uint64_t dth = 0;
    {
        const uint32_t q = (uint32_t)th >> c;
        for (int j = 0; j < t - kRegBits - c; ++j) dth |= (uint64_t)((q >> j) & 1u) << a.tile_qubits[j];
    }
    VP* gp = (VP*)a.psi;
    VL* gl = (VL*)a.lam;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        uint64_t dr = 0;
        for (int j = 0; j < kRegBits; ++j) dr |= (uint64_t)((r >> j) & 1) << a.tile_qubits[t - kRegBits - c + j];
        const uint64_t off = (base | dth | dr) * B + (uint64_t)(b0 + bl);
        const uint32_t e = (uint32_t)th + (uint32_t)r * nthr;
        VP v = mkv<VP, RP>((RP)0, (RP)0);
        if (bvalid) v = gp[off];
        lp[swz(e)] = v;
        if (BWD) {
            VL w = mkv<VL, RL>((RL)0, (RL)0);
            if (bvalid) w = gl[off];
            ll[swz(e)] = w;
        }
    }
    __syncthreads();

    for (int gi = 0; gi < a.ngroups; ++gi) {
        const PGroupDesc G = a.groups[a.group0 + gi];
        if (G.lds) {
            // ------------------------------------------------ a 2- or 3-qubit gate in LDS
            const POp op = a.ops[G.op0];
            double gacc = 0;
            if ((base & op.omask) == op.oval) {
                const int k = op.k, D = 1 << k;
                const double* m = a.mats + op.mat;
                const int DD = D * D;
                int sorted[3] = {op.tpos[0], op.tpos[1], op.tpos[2]};
                for (int i = 0; i < k; ++i)
                    for (int j = i + 1; j < k; ++j)
                        if (sorted[j] < sorted[i]) {
                            int tmp = sorted[i];
                            sorted[i] = sorted[j];
                            sorted[j] = tmp;
                        }
                const int ngr = 1 << (t - k);
                for (int gidx = th; gidx < ngr; gidx += nthr) {
                    uint32_t eb = (uint32_t)gidx;
                    for (int i = 0; i < k; ++i) {
                        const uint32_t lo = eb & ((1u << sorted[i]) - 1);
                        eb = ((eb >> sorted[i]) << (sorted[i] + 1)) | lo;
                    }
                    if ((eb & op.cmask) != op.cval) continue;
                    uint32_t idx[8];
                    for (int s = 0; s < D; ++s) {
                        uint32_t o = eb;
                        for (int j = 0; j < k; ++j)
                            if ((s >> j) & 1) o |= 1u << op.tpos[j];
                        idx[s] = swz(o);
                    }
                    if constexpr (!BWD) {
                        VP v[8], o[8];
                        for (int s = 0; s < D; ++s) v[s] = lp[idx[s]];
                        for (int r = 0; r < D; ++r) {
                            RP x = 0, y = 0;
                            for (int s = 0; s < D; ++s) {
                                const RP ur = (RP)m[r * D + s], ui = (RP)m[DD + r * D + s];
                                x = fma(ur, v[s].x, fma(-ui, v[s].y, x));
                                y = fma(ur, v[s].y, fma(ui, v[s].x, y));
                            }
                            o[r] = mkv<VP, RP>(x, y);
                        }
                        for (int s = 0; s < D; ++s) lp[idx[s]] = o[s];
                    } else {
                        double2 p[8];
                        VL l[8];
                        for (int s = 0; s < D; ++s) {
                            p[s] = ((double2*)lp)[idx[s]];
                            l[s] = ll[idx[s]];
                        }
                        if (op.slot >= 0) {
                            const double* Mr = m + 2 * DD;
                            const double* Mi = m + 3 * DD;
                            for (int r = 0; r < D; ++r) {
                                double x = 0, y = 0;
                                for (int s = 0; s < D; ++s) {
                                    x += Mr[r * D + s] * p[s].x - Mi[r * D + s] * p[s].y;
                                    y += Mr[r * D + s] * p[s].y + Mi[r * D + s] * p[s].x;
                                }
                                gacc += 2.0 * ((double)l[r].x * x + (double)l[r].y * y);
                            }
                        }
                        for (int r = 0; r < D; ++r) {
                            double x = 0, y = 0, u = 0, w = 0;
                            for (int s = 0; s < D; ++s) {
                                const double ur = m[r * D + s], ui = m[DD + r * D + s];
                                x += ur * p[s].x - ui * p[s].y;
                                y += ur * p[s].y + ui * p[s].x;
                                u += ur * (double)l[s].x - ui * (double)l[s].y;
                                w += ur * (double)l[s].y + ui * (double)l[s].x;
                            }
                            ((double2*)lp)[idx[r]] = make_double2(x, y);
                            ll[idx[r]] = mkv<VL, RL>((RL)u, (RL)w);
                        }
                    }
                }
            }
            if (BWD && op.slot >= 0) {
                double v = wave_sum_by_slot(gacc, Bc, nthr);
                if (lane < Bc) red[wave * Bc + lane] = v;
            }
            __syncthreads();
            if (BWD && op.slot >= 0) {
                if (th < Bc && b0 + th < a.B) {
                    double s = 0;
                    for (int w = 0; w < nwaves; ++w) s += red[w * Bc + th];
                    a.gpartial[((uint64_t)op.slot * a.B + b0 + th) * a.pstride + blockIdx.x] = s;
                }
                __syncthreads();
            }
            continue;
        }

        // ---------------------------------------------------------- a register group
        // Thread bits: the tile bits that are not register bits, ascending.
        uint32_t ethr = 0;
        {
            uint32_t rmask = 0;
            for (int j = 0; j < kRegBits; ++j) rmask |= 1u << G.rpos[j];
            int k = 0;
            for (int b = 0; b < t; ++b) {
                if ((rmask >> b) & 1u) continue;
                ethr |= (((uint32_t)th >> k) & 1u) << b;
                ++k;
            }
        }
        uint32_t er[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uint32_t v = 0;
#pragma unroll
            for (int j = 0; j < kRegBits; ++j) v |= ((uint32_t)(r >> j) & 1u) << G.rpos[j];
            er[r] = v;
        }
        VP x[R];
        VL y[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t p = swz(ethr | er[r]);
            x[r] = lp[p];
            if (BWD) y[r] = ll[p];
        }
        int nslot = 0;
        for (int oi = 0; oi < G.nops; ++oi) {
            const POp op = a.ops[G.op0 + oi];
            const bool on = (base & op.omask) == op.oval;
            const double* m = a.mats + op.mat;
            double g = 0;
            if (on) {
                if constexpr (!BWD) {
                    RP mr[4], mi[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        mr[q] = (RP)m[q];
                        mi[q] = (RP)m[4 + q];
                    }
#define YAO_FWD_CASE(J)                                                                       \
    case J:                                                                                   \
        if (op.cmask) op_apply<J, true, RP>(x, op.type, mr, mi, ethr, er, op.cmask, op.cval); \
        else op_apply<J, false, RP>(x, op.type, mr, mi, ethr, er, 0u, 0u);                    \
        break;
                    switch (op.rpos) { YAO_FWD_CASE(0) YAO_FWD_CASE(1) YAO_FWD_CASE(2) YAO_FWD_CASE(3) }
#undef YAO_FWD_CASE
                } else {
                    const bool gr = op.slot >= 0;
#define YAO_BWD_CASE(J)                                                                                      \
    case J:                                                                                                  \
        if (op.cmask) g = op_bwd<J, true, VL>(x, y, op.type, op.gen, gr, m, ethr, er, op.cmask, op.cval);   \
        else g = op_bwd<J, false, VL>(x, y, op.type, op.gen, gr, m, ethr, er, 0u, 0u);                      \
        break;
                    switch (op.rpos) { YAO_BWD_CASE(0) YAO_BWD_CASE(1) YAO_BWD_CASE(2) YAO_BWD_CASE(3) }
#undef YAO_BWD_CASE
                }
            }
            if (BWD && op.slot >= 0) {
                double v = wave_sum_by_slot(g, Bc, nthr);
                if (lane < Bc) red[(nslot * nwaves + wave) * Bc + lane] = v;
                ++nslot;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t p = swz(ethr | er[r]);
            lp[p] = x[r];
            if (BWD) ll[p] = y[r];
        }
        __syncthreads();
        if (BWD && nslot > 0) {
            // one thread per (slot, batch slot): sum the waves in order
            for (int idx = th; idx < nslot * Bc; idx += nthr) {
                const int sl = idx / Bc, bb = idx % Bc;
                if (b0 + bb >= a.B) continue;
                double s = 0;
                for (int w = 0; w < nwaves; ++w) s += red[(sl * nwaves + w) * Bc + bb];
                // slot of the sl-th gradient op of this group
                int cnt = -1, slot = -1;
                for (int oi = 0; oi < G.nops; ++oi) {
                    const int sv = a.ops[G.op0 + oi].slot;
                    if (sv >= 0 && ++cnt == sl) {
                        slot = sv;
                        break;
                    }
                }
                a.gpartial[((uint64_t)slot * a.B + b0 + bb) * a.pstride + blockIdx.x] = s;
            }
            __syncthreads();
        }
    }

    // ---------------------------------------------------------------- store the tile
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!bvalid) break;
        uint64_t dr = 0;
        for (int j = 0; j < kRegBits; ++j) dr |= (uint64_t)((r >> j) & 1) << a.tile_qubits[t - kRegBits - c + j];
        const uint64_t off = (base | dth | dr) * B + (uint64_t)(b0 + bl);
        const uint32_t e = (uint32_t)th + (uint32_t)r * nthr;
        gp[off] = lp[swz(e)];
        if (BWD) gl[off] = ll[swz(e)];
    }
}

}  // namespace

size_t pass_lds_bytes(int t, int dtype_psi_bytes, int lam_bytes)
{
    const size_t red = sizeof(double) * kMaxGroupSlots * 4 * 8;
    return ((size_t)(dtype_psi_bytes + lam_bytes) << t) + red;
}

int launch_pass(bool bwd, int psi_dtype, int lam_dtype, void* psi, void* lam, const POp* ops, const PGroupDesc* groups,
                const double* mats, double* gpartial, int pstride, int n, int B, int c, int t, int group0,
                int ngroups, const std::vector<int>& tile_qubits)
{
    PassArgs a;
    memset(&a, 0, sizeof(a));
    a.psi = psi;
    a.lam = lam;
    a.ops = ops;
    a.groups = groups;
    a.mats = mats;
    a.gpartial = gpartial;
    a.n = n;
    a.B = B;
    a.c = c;
    a.t = t;
    a.group0 = group0;
    a.ngroups = ngroups;
    a.ntq = (int)tile_qubits.size();
    uint64_t T = 0;
    for (int j = 0; j < a.ntq; ++j) {
        a.tile_qubits[j] = tile_qubits[j];
        T |= uint64_t(1) << tile_qubits[j];
    }
    a.nnt = 0;
    for (int q = 0; q < n; ++q)
        if (!((T >> q) & 1)) a.nontile_qubits[a.nnt++] = q;
    a.ntiles = 1 << a.nnt;
    a.pstride = pstride > a.ntiles ? pstride : a.ntiles;
    const int Bc = 1 << c;
    dim3 grid(a.ntiles, (B + Bc - 1) / Bc);
    dim3 block(1 << (t - kRegBits));
    const int pb = psi_dtype == YAO_C64 ? 8 : 16;
    const int lb = bwd ? (lam_dtype == YAO_C64 ? 8 : 16) : 0;
    const size_t lds = pass_lds_bytes(t, pb, lb);
    hipStream_t st = stream();
    if (!bwd) {
        if (psi_dtype == YAO_C64) {
            static bool attr = false;
            if (!attr) {
                YAO_HIP(hipFuncSetAttribute((const void*)k_pass<float, float, false>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
                attr = true;
            }
            k_pass<float, float, false><<<grid, block, lds, st>>>(a);
        } else {
            static bool attr = false;
            if (!attr) {
                YAO_HIP(hipFuncSetAttribute((const void*)k_pass<double, double, false>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
                attr = true;
            }
            k_pass<double, double, false><<<grid, block, lds, st>>>(a);
        }
    } else {
        if (lam_dtype == YAO_C64) {
            static bool attr = false;
            if (!attr) {
                YAO_HIP(hipFuncSetAttribute((const void*)k_pass<double, float, true>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
                attr = true;
            }
            k_pass<double, float, true><<<grid, block, lds, st>>>(a);
        } else {
            static bool attr = false;
            if (!attr) {
                YAO_HIP(hipFuncSetAttribute((const void*)k_pass<double, double, true>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
                attr = true;
            }
            k_pass<double, double, true><<<grid, block, lds, st>>>(a);
        }
    }
    YAO_HIP(hipGetLastError());
    return 0;
}

}  // namespace yao
