// Per-gate ("plain form") kernels of the gfx950 state-vector library, the Pauli-sum
// expectation and H psi kernels, and small utilities.
//
// Every kernel walks the state with the batch innermost, so consecutive lanes touch
// consecutive addresses: for a single state (B = 1) the lanes run along the low bits of the
// pair index, for a batch they run along the batch slots of one amplitude row.
#include <algorithm>
#include <cstdarg>
#include <cstdio>

#include "fused.h"
#include "runtime.h"

namespace yao {

namespace {

constexpr int kThreads = 256;

template <typename R> __device__ __forceinline__ vec2_t<R> mk(R a, R b)
{
    vec2_t<R> v;
    v.x = a;
    v.y = b;
    return v;
}

// -------------------------------------------------------------------------------- state init
template <typename R>
__global__ __launch_bounds__(kThreads) void k_fill_basis(vec2_t<R>* __restrict__ psi, uint64_t elems, int B)
{
    uint64_t e = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= elems) return;
    psi[e] = mk<R>(e < (uint64_t)B ? R(1) : R(0), R(0));
}

// |0...0> in each of a list of single-slot states (blockIdx.y selects the state).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_fill_basis_z(vec2_t<R>* const* __restrict__ ptrs, uint64_t elems)
{
    vec2_t<R>* psi = ptrs[blockIdx.y];
    for (uint64_t e = (uint64_t)blockIdx.x * kThreads + threadIdx.x; e < elems; e += (uint64_t)gridDim.x * kThreads)
        psi[e] = mk<R>(e == 0 ? R(1) : R(0), R(0));
}

// dst[y * elems + e] = src_y[e] widened to complex128 (blockIdx.y selects the state).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_convert_z(const vec2_t<R>* const* __restrict__ src,
                                                        double2* __restrict__ dst, uint64_t elems)
{
    const vec2_t<R>* a = src[blockIdx.y];
    double2* d = dst + (uint64_t)blockIdx.y * elems;
    for (uint64_t e = (uint64_t)blockIdx.x * kThreads + threadIdx.x; e < elems; e += (uint64_t)gridDim.x * kThreads)
        d[e] = make_double2((double)a[e].x, (double)a[e].y);
}

// -------------------------------------------------------------------------------- 1-qubit gate
// Work item w = j * 2^logBp + b: pair row j (2^(n-1) of them) and batch slot b (padded to a
// power of two, slots >= B idle). The pair is (i0, i0 + 2^q) with bit q of i0 clear.
template <typename R, int CLS>
__global__ __launch_bounds__(kThreads) void k_gate1(vec2_t<R>* __restrict__ psi, uint64_t nwork, int q, int logBp,
                                                    int B, uint64_t cmask, uint64_t cval, M2<R> m)
{
    using V = vec2_t<R>;
    uint64_t w = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (w >= nwork) return;
    int b = (int)(w & ((uint64_t(1) << logBp) - 1));
    if (b >= B) return;
    uint64_t j = w >> logBp;
    uint64_t i0 = insert_zero(j, q);
    if ((i0 & cmask) != cval) return;
    uint64_t o0 = i0 * (uint64_t)B + b;
    uint64_t o1 = o0 + ((uint64_t)B << q);
    if (CLS == MC_DIAG1) {
        V c = psi[o1];
        psi[o1] = mk<R>(m.re[3] * c.x - m.im[3] * c.y, m.re[3] * c.y + m.im[3] * c.x);
        return;
    }
    V a = psi[o0], c = psi[o1];
    V r0, r1;
    if (CLS == MC_DIAG) {
        r0 = mk<R>(m.re[0] * a.x - m.im[0] * a.y, m.re[0] * a.y + m.im[0] * a.x);
        r1 = mk<R>(m.re[3] * c.x - m.im[3] * c.y, m.re[3] * c.y + m.im[3] * c.x);
    } else if (CLS == MC_ANTI) {
        r0 = mk<R>(m.re[1] * c.x - m.im[1] * c.y, m.re[1] * c.y + m.im[1] * c.x);
        r1 = mk<R>(m.re[2] * a.x - m.im[2] * a.y, m.re[2] * a.y + m.im[2] * a.x);
    } else {
        R x0 = 0, y0 = 0, x1 = 0, y1 = 0;
        cmul_acc(x0, y0, m.re[0], m.im[0], a);
        cmul_acc(x0, y0, m.re[1], m.im[1], c);
        cmul_acc(x1, y1, m.re[2], m.im[2], a);
        cmul_acc(x1, y1, m.re[3], m.im[3], c);
        r0 = mk<R>(x0, y0);
        r1 = mk<R>(x1, y1);
    }
    psi[o0] = r0;
    psi[o1] = r1;
}

// -------------------------------------------------------------------------------- k-qubit gate
// Offsets of the 2^K members of a group relative to its base index, and the target bit
// positions in ascending order (for inserting the zero bits).
template <int K> struct GroupGeom {
    uint64_t off[1 << K];
    int sorted[K];
};

template <int K> __device__ __forceinline__ uint64_t group_base(uint64_t j, const GroupGeom<K>& g)
{
#pragma unroll
    for (int t = 0; t < K; ++t) j = insert_zero(j, g.sorted[t]);
    return j;
}

template <typename R, int K>
__global__ __launch_bounds__(kThreads) void k_gatek(vec2_t<R>* __restrict__ psi, uint64_t nwork, int logBp, int B,
                                                    GroupGeom<K> gg, uint64_t cmask, uint64_t cval,
                                                    const R* __restrict__ Ure, const R* __restrict__ Uim)
{
    using V = vec2_t<R>;
    constexpr int D = 1 << K;
    uint64_t w = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (w >= nwork) return;
    int b = (int)(w & ((uint64_t(1) << logBp) - 1));
    if (b >= B) return;
    uint64_t base = group_base<K>(w >> logBp, gg);
    if ((base & cmask) != cval) return;
    V a[D];
#pragma unroll
    for (int s = 0; s < D; ++s) a[s] = psi[(base + gg.off[s]) * (uint64_t)B + b];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        R x = 0, y = 0;
#pragma unroll
        for (int s = 0; s < D; ++s) cmul_acc(x, y, Ure[r * D + s], Uim[r * D + s], a[s]);
        psi[(base + gg.off[r]) * (uint64_t)B + b] = mk<R>(x, y);
    }
}

// -------------------------------------------------------------------------------- reductions
// Block reduction of one double per thread, grouped by batch slot (tid & (Bc-1)).
__device__ __forceinline__ double block_sum_by_slot(double v, int logBc, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kThreads / 2; s >= (1 << logBc); s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[threadIdx.x];
}

// Value of Re(i^ny * w) for w = wr + i wi.
__device__ __forceinline__ double re_iny(int ny, double wr, double wi)
{
    switch (ny & 3) {
    case 0: return wr;
    case 1: return -wi;
    case 2: return -wr;
    default: return wi;
    }
}

// E_b = sum_i sum_t c_t Re( conj(psi_{i ^ x_t}) i^{ny_t} (-1)^{|i & z_t|} psi_i ), using
// P|i> = i^{ny} (-1)^{|i & z|} |i ^ x> with ny = |x & z|. Rows are amplitude indices.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_expect(const vec2_t<R>* __restrict__ psi, uint64_t rows, int B,
                                                     int logBc, const PGroup* __restrict__ groups, int ngroups,
                                                     const PTerm* __restrict__ terms, double* __restrict__ partial)
{
    __shared__ double red[kThreads];
    const int bb = threadIdx.x & ((1 << logBc) - 1);
    const int b = blockIdx.y * (1 << logBc) + bb;
    const int rpb = kThreads >> logBc;
    double acc = 0;
    if (b < B) {
        for (uint64_t i = (uint64_t)blockIdx.x * rpb + (threadIdx.x >> logBc); i < rows; i += (uint64_t)gridDim.x * rpb) {
            vec2_t<R> a = psi[i * B + b];
            for (int g = 0; g < ngroups; ++g) {
                uint64_t x = groups[g].x;
                vec2_t<R> p = x ? psi[(i ^ x) * B + b] : a;
                double wr = (double)p.x * a.x + (double)p.y * a.y;
                double wi = (double)p.x * a.y - (double)p.y * a.x;
                for (int t = groups[g].t0; t < groups[g].t1; ++t) {
                    double v = re_iny(terms[t].ny, wr, wi);
                    acc += (__popcll(i & terms[t].z) & 1) ? -terms[t].c * v : terms[t].c * v;
                }
            }
        }
    }
    double s = block_sum_by_slot(acc, logBc, red);
    if ((int)threadIdx.x < (1 << logBc) && b < B) partial[(uint64_t)b * gridDim.x + blockIdx.x] = s;
}

// out_j = sum_t c_t i^{ny_t} (-1)^{|(j ^ x_t) & z_t|} psi_{j ^ x_t}, plus E from the same pass.
template <typename R, typename RO>
__global__ __launch_bounds__(kThreads) void k_hpsi(const vec2_t<R>* __restrict__ psi, vec2_t<RO>* __restrict__ out,
                                                   uint64_t rows, int B, int logBc, const PGroup* __restrict__ groups,
                                                   int ngroups, const PTerm* __restrict__ terms,
                                                   double* __restrict__ partial)
{
    __shared__ double red[kThreads];
    const int bb = threadIdx.x & ((1 << logBc) - 1);
    const int b = blockIdx.y * (1 << logBc) + bb;
    const int rpb = kThreads >> logBc;
    double acc = 0;
    if (b < B) {
        for (uint64_t j = (uint64_t)blockIdx.x * rpb + (threadIdx.x >> logBc); j < rows; j += (uint64_t)gridDim.x * rpb) {
            double orr = 0, oi = 0;
            // Partner amplitudes of 8 X-mask groups are fetched together, then combined.
            for (int g0 = 0; g0 < ngroups; g0 += 8) {
                vec2_t<R> p[8];
                uint64_t src[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    src[u] = j;
                    if (g0 + u < ngroups) {
                        src[u] = j ^ groups[g0 + u].x;
                        p[u] = psi[src[u] * B + b];
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (g0 + u >= ngroups) break;
                    double cr = 0, ci = 0;  // sum of c_t i^{ny} (-1)^{|src & z|}
                    for (int t = groups[g0 + u].t0; t < groups[g0 + u].t1; ++t) {
                        double c = (__popcll(src[u] & terms[t].z) & 1) ? -terms[t].c : terms[t].c;
                        switch (terms[t].ny & 3) {
                        case 0: cr += c; break;
                        case 1: ci += c; break;
                        case 2: cr -= c; break;
                        default: ci -= c; break;
                        }
                    }
                    orr += cr * p[u].x - ci * p[u].y;
                    oi += cr * p[u].y + ci * p[u].x;
                }
            }
            vec2_t<R> a = psi[j * B + b];
            acc += (double)a.x * orr + (double)a.y * oi;
            vec2_t<RO> o;
            o.x = (RO)orr;
            o.y = (RO)oi;
            out[j * B + b] = o;
        }
    }
    double s = block_sum_by_slot(acc, logBc, red);
    if ((int)threadIdx.x < (1 << logBc) && b < B) partial[(uint64_t)b * gridDim.x + blockIdx.x] = s;
}

// sums[r] = sum_j partial[r * nblk + j]: one wave per row, lane-strided sums and then a fixed
// butterfly, so the order (and the result) is the same on every run.
__global__ __launch_bounds__(256) void k_row_sums(const double* __restrict__ partial, int rows, int nblk,
                                                  double* __restrict__ sums)
{
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows) return;
    double s = 0;
    for (int j = lane; j < nblk; j += 64) s += partial[(uint64_t)r * nblk + j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) sums[r] = s;
}

template <typename RA, typename RB>
__global__ __launch_bounds__(kThreads) void k_convert(const vec2_t<RA>* __restrict__ a, vec2_t<RB>* __restrict__ b,
                                                      uint64_t elems)
{
    for (uint64_t e = (uint64_t)blockIdx.x * kThreads + threadIdx.x; e < elems; e += (uint64_t)gridDim.x * kThreads) {
        vec2_t<RA> v = a[e];
        vec2_t<RB> o;
        o.x = (RB)v.x;
        o.y = (RB)v.y;
        b[e] = o;
    }
}

template <typename RA, typename RB>
__global__ __launch_bounds__(kThreads) void k_maxdiff(const vec2_t<RA>* __restrict__ a, const vec2_t<RB>* __restrict__ b,
                                                      uint64_t elems, double* __restrict__ partial)
{
    __shared__ double red[kThreads];
    double m = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * kThreads + threadIdx.x; e < elems; e += (uint64_t)gridDim.x * kThreads) {
        vec2_t<RA> u = a[e];
        vec2_t<RB> v = b[e];
        double dr = (double)u.x - (double)v.x, di = (double)u.y - (double)v.y;
        m = fmax(m, sqrt(dr * dr + di * di));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// <a_b|b_b> per batch slot: real parts to partial[b][blk], imaginary parts to
// partial[B + b][blk].
template <typename RA, typename RB>
__global__ __launch_bounds__(kThreads) void k_inner(const vec2_t<RA>* __restrict__ a, const vec2_t<RB>* __restrict__ b,
                                                    uint64_t rows, int B, int logBc, double* __restrict__ partial)
{
    __shared__ double red[kThreads];
    const int bb = threadIdx.x & ((1 << logBc) - 1);
    const int s = blockIdx.y * (1 << logBc) + bb;
    const int rpb = kThreads >> logBc;
    double re = 0, im = 0;
    if (s < B) {
        for (uint64_t i = (uint64_t)blockIdx.x * rpb + (threadIdx.x >> logBc); i < rows; i += (uint64_t)gridDim.x * rpb) {
            const vec2_t<RA> u = a[i * B + s];
            const vec2_t<RB> v = b[i * B + s];
            re += (double)u.x * v.x + (double)u.y * v.y;
            im += (double)u.x * v.y - (double)u.y * v.x;
        }
    }
    double r1 = block_sum_by_slot(re, logBc, red);
    if ((int)threadIdx.x < (1 << logBc) && s < B) partial[(uint64_t)s * gridDim.x + blockIdx.x] = r1;
    __syncthreads();
    double r2 = block_sum_by_slot(im, logBc, red);
    if ((int)threadIdx.x < (1 << logBc) && s < B) partial[(uint64_t)(B + s) * gridDim.x + blockIdx.x] = r2;
}

// -------------------------------------------------------------------------------- adjoint step
// One gate of the reverse sweep (eq. apply-back): gradient partial 2 Re <lam|M|psi> over the
// controlled subspace, then psi <- Ud psi (FP64) and lam <- Ud lam. Rows are pair rows.
struct AdjMats1 {
    double udr[4], udi[4], mr[4], mi[4];
};

template <typename RL, int K, bool GRAD>
__global__ __launch_bounds__(kThreads) void k_adjoint(double2* __restrict__ psi, vec2_t<RL>* __restrict__ lam,
                                                      uint64_t rows, int B, int logBc, GroupGeom<K> gg,
                                                      uint64_t cmask, uint64_t cval, AdjMats1 m1,
                                                      const double* __restrict__ mats, double* __restrict__ partial,
                                                      int pstride)
{
    constexpr int D = 1 << K;
    constexpr int DD = D * D;
    // K == 1: matrices by value; otherwise mats holds Ud re, Ud im, M re, M im (DD doubles each).
    const double* Udr = K == 1 ? m1.udr : mats;
    const double* Udi = K == 1 ? m1.udi : mats + DD;
    const double* Mr = K == 1 ? m1.mr : mats + 2 * DD;
    const double* Mi = K == 1 ? m1.mi : mats + 3 * DD;
    __shared__ double red[kThreads];
    const int bb = threadIdx.x & ((1 << logBc) - 1);
    const int b = blockIdx.y * (1 << logBc) + bb;
    const int rpb = kThreads >> logBc;
    double acc = 0;
    if (b < B) {
        for (uint64_t j = (uint64_t)blockIdx.x * rpb + (threadIdx.x >> logBc); j < rows; j += (uint64_t)gridDim.x * rpb) {
            uint64_t base = group_base<K>(j, gg);
            if ((base & cmask) != cval) continue;
            double2 p[D];
            vec2_t<RL> l[D];
#pragma unroll
            for (int s = 0; s < D; ++s) {
                uint64_t o = (base + gg.off[s]) * (uint64_t)B + b;
                p[s] = psi[o];
                l[s] = lam[o];
            }
            if (GRAD) {
#pragma unroll
                for (int r = 0; r < D; ++r) {
                    double x = 0, y = 0;
#pragma unroll
                    for (int s = 0; s < D; ++s) cmul_acc(x, y, Mr[r * D + s], Mi[r * D + s], p[s]);
                    acc += 2.0 * ((double)l[r].x * x + (double)l[r].y * y);
                }
            }
#pragma unroll
            for (int r = 0; r < D; ++r) {
                double x = 0, y = 0, u = 0, v = 0;
#pragma unroll
                for (int s = 0; s < D; ++s) {
                    cmul_acc(x, y, Udr[r * D + s], Udi[r * D + s], p[s]);
                    cmul_acc(u, v, Udr[r * D + s], Udi[r * D + s], l[s]);
                }
                uint64_t o = (base + gg.off[r]) * (uint64_t)B + b;
                psi[o] = make_double2(x, y);
                vec2_t<RL> lo;
                lo.x = (RL)u;
                lo.y = (RL)v;
                lam[o] = lo;
            }
        }
    }
    if (GRAD) {
        double s = block_sum_by_slot(acc, logBc, red);
        if ((int)threadIdx.x < (1 << logBc) && b < B) partial[(uint64_t)b * pstride + blockIdx.x] = s;
    }
}

__global__ void k_fill(double* __restrict__ p, uint64_t count, double v)
{
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (uint64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

template <int K> GroupGeom<K> make_group_geom(const int* locs)
{
    GroupGeom<K> g;
    for (int s = 0; s < (1 << K); ++s) {
        uint64_t o = 0;
        for (int j = 0; j < K; ++j)
            if ((s >> j) & 1) o |= uint64_t(1) << locs[j];
        g.off[s] = o;
    }
    int tmp[K];
    for (int j = 0; j < K; ++j) tmp[j] = locs[j];
    for (int a = 0; a < K; ++a)
        for (int c = a + 1; c < K; ++c)
            if (tmp[c] < tmp[a]) {
                int t = tmp[a];
                tmp[a] = tmp[c];
                tmp[c] = t;
            }
    for (int j = 0; j < K; ++j) g.sorted[j] = tmp[j];
    return g;
}

unsigned grid1(uint64_t work)
{
    return (unsigned)((work + kThreads - 1) / kThreads);
}

template <typename R>
int gate_typed(void* data, int n, int B, const HostMat& U, const int* locs, CtrlSpec c, const void* dev_mat)
{
    using V = vec2_t<R>;
    V* psi = (V*)data;
    const int k = U.k;
    const int logBp = ilog2_ceil((uint64_t)B);
    const uint64_t nwork = (uint64_t(1) << (n - k)) << logBp;
    hipStream_t st = stream();
    if (k == 1) {
        M2<R> m;
        for (int t = 0; t < 4; ++t) {
            m.re[t] = (R)U.re[t];
            m.im[t] = (R)U.im[t];
        }
        const double elems = (double)(uint64_t(1) << n) * B / double(uint64_t(1) << __builtin_popcountll(c.mask));
        const int cls = classify(U);
        const int pi = prof_begin(YAO_KF_GATE);
        switch (cls) {
        case MC_DIAG1: k_gate1<R, MC_DIAG1><<<grid1(nwork), kThreads, 0, st>>>(psi, nwork, locs[0], logBp, B, c.mask, c.val, m); break;
        case MC_DIAG: k_gate1<R, MC_DIAG><<<grid1(nwork), kThreads, 0, st>>>(psi, nwork, locs[0], logBp, B, c.mask, c.val, m); break;
        case MC_ANTI: k_gate1<R, MC_ANTI><<<grid1(nwork), kThreads, 0, st>>>(psi, nwork, locs[0], logBp, B, c.mask, c.val, m); break;
        default: k_gate1<R, MC_DENSE><<<grid1(nwork), kThreads, 0, st>>>(psi, nwork, locs[0], logBp, B, c.mask, c.val, m); break;
        }
        prof_end(pi, (cls == MC_DIAG1 ? 1.0 : 2.0) * elems * sizeof(V), (cls == MC_DIAG1 ? 3.0 : cls == MC_DENSE ? 14.0 : 6.0) * elems);
        YAO_HIP(hipGetLastError());
        return 0;
    }
    if constexpr (sizeof(R) == 4) {
        // Dense 4- and 5-qubit blocks on complex64 states go to the FP32 matrix cores.
        if (options().mfma && mfma_supported(k, n, B)) return launch_dense_mfma((float2*)data, n, B, U, locs, c, dev_mat);
    }
    // k >= 2: the matrix, rounded once to R (re block then im block), lives in device memory.
    const size_t dd = size_t(1) << (2 * k);
    const R* dm = (const R*)dev_mat;
    if (!dm) {
        std::vector<R> h(2 * dd);
        for (size_t t = 0; t < dd; ++t) {
            h[t] = (R)U.re[t];
            h[dd + t] = (R)U.im[t];
        }
        dm = (const R*)ring_upload(h.data(), h.size() * sizeof(R));
        if (!dm) return YAO_ENOMEM;
    }
    const double elems = (double)(uint64_t(1) << n) * B / double(uint64_t(1) << __builtin_popcountll(c.mask));
    const int pi = prof_begin(YAO_KF_GATE);
    switch (k) {
    case 2: k_gatek<R, 2><<<grid1(nwork), kThreads, 0, st>>>(psi, nwork, logBp, B, make_group_geom<2>(locs), c.mask, c.val, dm, dm + dd); break;
    case 3: k_gatek<R, 3><<<grid1(nwork), kThreads, 0, st>>>(psi, nwork, logBp, B, make_group_geom<3>(locs), c.mask, c.val, dm, dm + dd); break;
    case 4: k_gatek<R, 4><<<grid1(nwork), kThreads, 0, st>>>(psi, nwork, logBp, B, make_group_geom<4>(locs), c.mask, c.val, dm, dm + dd); break;
    case 5: k_gatek<R, 5><<<grid1(nwork), kThreads, 0, st>>>(psi, nwork, logBp, B, make_group_geom<5>(locs), c.mask, c.val, dm, dm + dd); break;
    default: return set_error(YAO_EINVAL, "k = %d not supported", k);
    }
    prof_end(pi, 2.0 * elems * sizeof(V), (8.0 * (1 << k) - 2.0) * elems);
    YAO_HIP(hipGetLastError());
    return 0;
}

int reduce_grid_x(uint64_t rows, int logBc)
{
    uint64_t rpb = kThreads >> logBc;
    uint64_t nb = (rows + rpb - 1) / rpb;
    return (int)(nb < 1024 ? nb : 1024);
}

}  // namespace

// =========================================================================================
// Launchers
// =========================================================================================

int launch_fill_basis(void* data, int dtype, int n, int B)
{
    uint64_t elems = (uint64_t(1) << n) * (uint64_t)B;
    if (dtype == YAO_C64)
        k_fill_basis<float><<<grid1(elems), kThreads, 0, stream()>>>((float2*)data, elems, B);
    else
        k_fill_basis<double><<<grid1(elems), kThreads, 0, stream()>>>((double2*)data, elems, B);
    YAO_HIP(hipGetLastError());
    return 0;
}

int launch_fill_basis_z(void* const* ptrs, int nz, int dtype, int n)
{
    const uint64_t elems = uint64_t(1) << n;
    const dim3 grid((unsigned)std::min<uint64_t>((elems + kThreads - 1) / kThreads, 4096), nz);
    if (dtype == YAO_C64) k_fill_basis_z<float><<<grid, kThreads, 0, stream()>>>((float2* const*)ptrs, elems);
    else k_fill_basis_z<double><<<grid, kThreads, 0, stream()>>>((double2* const*)ptrs, elems);
    YAO_HIP(hipGetLastError());
    return 0;
}

int launch_convert_z(const void* const* src, int nz, int dtype, double* dst, int n)
{
    const uint64_t elems = uint64_t(1) << n;
    const dim3 grid((unsigned)std::min<uint64_t>((elems + kThreads - 1) / kThreads, 4096), nz);
    if (dtype == YAO_C64) k_convert_z<float><<<grid, kThreads, 0, stream()>>>((const float2* const*)src, (double2*)dst, elems);
    else k_convert_z<double><<<grid, kThreads, 0, stream()>>>((const double2* const*)src, (double2*)dst, elems);
    YAO_HIP(hipGetLastError());
    return 0;
}

int launch_reset(yao_state* s)
{
    return launch_fill_basis(s->data, s->dtype, s->n, s->batch);
}

size_t encode_gate_matrix(int dtype, int n, int B, const HostMat& U, std::vector<double>& pool)
{
    pool.resize((pool.size() + 3) & ~size_t(3));  // 32-byte aligned within the pool
    const size_t off = pool.size();
    const size_t dd = size_t(1) << (2 * U.k);
    if (dtype == YAO_C64 && options().mfma && mfma_supported(U.k, n, B)) {
        pool.resize(off + 2 * dd);  // 4 dd floats
        mfma_encode(U, (float*)(pool.data() + off));
    } else if (dtype == YAO_C64) {
        pool.resize(off + dd);  // 2 dd floats
        float* f = (float*)(pool.data() + off);
        for (size_t t = 0; t < dd; ++t) {
            f[t] = (float)U.re[t];
            f[dd + t] = (float)U.im[t];
        }
    } else {
        pool.insert(pool.end(), U.re.begin(), U.re.end());
        pool.insert(pool.end(), U.im.begin(), U.im.end());
    }
    return off;
}

int launch_gate(void* data, int dtype, int n, int B, const HostMat& U, const int* locs, CtrlSpec c, const void* dev_mat)
{
    return dtype == YAO_C64 ? gate_typed<float>(data, n, B, U, locs, c, dev_mat)
                            : gate_typed<double>(data, n, B, U, locs, c, dev_mat);
}

int launch_row_sums(const double* partial, int rows, int nblk, double* sums)
{
    k_row_sums<<<(rows + 3) / 4, 256, 0, stream()>>>(partial, rows, nblk, sums);
    YAO_HIP(hipGetLastError());
    return 0;
}

void pauli_group_host(yao_pauli_sum* h)
{
    static_assert(sizeof(PGroup) == 16 && sizeof(PTerm) == 24, "table record sizes");
    std::vector<PGroup> groups;
    std::vector<PTerm> terms;
    std::vector<uint64_t> xs;
    // Group the terms by X mask, keeping first-appearance order.
    for (size_t t = 0; t < h->coef.size(); ++t) {
        bool seen = false;
        for (uint64_t x : xs) seen |= (x == h->x[t]);
        if (!seen) xs.push_back(h->x[t]);
    }
    for (uint64_t x : xs) {
        PGroup g;
        g.x = x;
        g.t0 = (int)terms.size();
        for (size_t t = 0; t < h->coef.size(); ++t) {
            if (h->x[t] != x) continue;
            PTerm pt;
            pt.c = h->coef[t];
            pt.z = h->z[t];
            pt.ny = __builtin_popcountll(h->x[t] & h->z[t]);
            pt.pad = 0;
            terms.push_back(pt);
        }
        g.t1 = (int)terms.size();
        groups.push_back(g);
    }
    h->host_groups.assign(groups.size() * 2, 0);
    memcpy(h->host_groups.data(), groups.data(), sizeof(PGroup) * groups.size());
    h->host_terms.assign(terms.size() * 3, 0);
    memcpy(h->host_terms.data(), terms.data(), sizeof(PTerm) * terms.size());
}

int pauli_upload(yao_pauli_sum* h)
{
    if (h->d_groups) return 0;
    if (h->host_groups.empty()) pauli_group_host(h);
    const size_t ng = h->host_groups.size() / 2, nt = h->host_terms.size() / 3;
    void *dg = nullptr, *dt = nullptr;
    if (hipMalloc(&dg, sizeof(PGroup) * (ng + 1)) != hipSuccess) return set_error(YAO_ENOMEM, "pauli tables");
    if (hipMalloc(&dt, sizeof(PTerm) * (nt + 1)) != hipSuccess) {
        (void)hipFree(dg);
        return set_error(YAO_ENOMEM, "pauli tables");
    }
    YAO_HIP(hipMemcpy(dg, h->host_groups.data(), sizeof(PGroup) * ng, hipMemcpyHostToDevice));
    YAO_HIP(hipMemcpy(dt, h->host_terms.data(), sizeof(PTerm) * nt, hipMemcpyHostToDevice));
    h->d_groups = dg;
    h->d_terms = dt;
    h->ngroups = (int)ng;
    h->nterms_dev = (int)nt;
    return 0;
}

int expect_grid_x(int n, int B)
{
    return reduce_grid_x(uint64_t(1) << n, make_batch_geom(B).logBc);
}

int launch_expect_into(const void* data, int dtype, int n, int B, const void* groups, int ngroups, const void* terms,
                       double* partial, double* sums)
{
    BatchGeom bg = make_batch_geom(B);
    const uint64_t rows = uint64_t(1) << n;
    const int nbx = reduce_grid_x(rows, bg.logBc);
    dim3 grid(nbx, bg.nchunks);
    if (dtype == YAO_C64)
        k_expect<float><<<grid, kThreads, 0, stream()>>>((const float2*)data, rows, B, bg.logBc, (const PGroup*)groups,
                                                         ngroups, (const PTerm*)terms, partial);
    else
        k_expect<double><<<grid, kThreads, 0, stream()>>>((const double2*)data, rows, B, bg.logBc, (const PGroup*)groups,
                                                          ngroups, (const PTerm*)terms, partial);
    YAO_HIP(hipGetLastError());
    return launch_row_sums(partial, B, nbx, sums);
}

static int finish_slot_sums(double* partial, int B, int nblk, double* energy_host)
{
    double* sums = (double*)workspace(WS_PARTIAL2, sizeof(double) * B);
    if (!sums) return YAO_ENOMEM;
    YAO_TRY(launch_row_sums(partial, B, nblk, sums));
    double* hs = (double*)host_staging(sizeof(double) * B);
    if (!hs) return YAO_ENOMEM;
    YAO_HIP(hipMemcpyAsync(hs, sums, sizeof(double) * B, hipMemcpyDeviceToHost, stream()));
    YAO_HIP(hipStreamSynchronize(stream()));
    memcpy(energy_host, hs, sizeof(double) * B);
    return 0;
}

int launch_expect(const void* data, int dtype, int n, int B, yao_pauli_sum* h, double* energy_host)
{
    if (obs_passes_ok(h, n, B, dtype)) {
        const size_t np = obs_partial_doubles(h, n, B, dtype);
        if (!np) return YAO_ENOMEM;
        double* partial = (double*)workspace(WS_PARTIAL, sizeof(double) * np);
        if (!partial) return YAO_ENOMEM;
        int W = 0;
        const int pi = prof_begin(YAO_KF_EXPECT);
        YAO_TRY(launch_obs_passes(data, dtype, nullptr, dtype, n, B, h, partial, &W));
        prof_end(pi, (double)(uint64_t(1) << n) * B * (dtype == YAO_C64 ? 8 : 16),
                 (double)(uint64_t(1) << n) * B * 4.0 * (double)h->coef.size());
        return finish_slot_sums(partial, B, W, energy_host);
    }
    YAO_TRY(pauli_upload(h));
    BatchGeom bg = make_batch_geom(B);
    uint64_t rows = uint64_t(1) << n;
    int nbx = reduce_grid_x(rows, bg.logBc);
    double* partial = (double*)workspace(WS_PARTIAL, sizeof(double) * (size_t)B * nbx);
    if (!partial) return YAO_ENOMEM;
    dim3 grid(nbx, bg.nchunks);
    const int pi = prof_begin(YAO_KF_EXPECT);
    if (dtype == YAO_C64)
        k_expect<float><<<grid, kThreads, 0, stream()>>>((const float2*)data, rows, B, bg.logBc, (const PGroup*)h->d_groups,
                                                         h->ngroups, (const PTerm*)h->d_terms, partial);
    else
        k_expect<double><<<grid, kThreads, 0, stream()>>>((const double2*)data, rows, B, bg.logBc, (const PGroup*)h->d_groups,
                                                          h->ngroups, (const PTerm*)h->d_terms, partial);
    prof_end(pi, (double)rows * B * (dtype == YAO_C64 ? 8 : 16), (double)rows * B * 4.0 * h->nterms_dev);
    YAO_HIP(hipGetLastError());
    return finish_slot_sums(partial, B, nbx, energy_host);
}

int launch_hpsi(const void* data, int dtype, void* out, int out_dtype, int n, int B, yao_pauli_sum* h,
                double* energy_host)
{
    if (obs_passes_ok(h, n, B, dtype)) {
        const size_t np = obs_partial_doubles(h, n, B, dtype);
        if (!np) return YAO_ENOMEM;
        double* partial = (double*)workspace(WS_PARTIAL, sizeof(double) * np);
        if (!partial) return YAO_ENOMEM;
        int W = 0;
        YAO_TRY(launch_obs_passes(data, dtype, out, out_dtype, n, B, h, partial, &W));
        if (!energy_host) return 0;
        return finish_slot_sums(partial, B, W, energy_host);
    }
    YAO_TRY(pauli_upload(h));
    BatchGeom bg = make_batch_geom(B);
    uint64_t rows = uint64_t(1) << n;
    int nbx = reduce_grid_x(rows, bg.logBc);
    double* partial = (double*)workspace(WS_PARTIAL, sizeof(double) * (size_t)B * nbx);
    if (!partial) return YAO_ENOMEM;
    dim3 grid(nbx, bg.nchunks);
    const PGroup* G = (const PGroup*)h->d_groups;
    const PTerm* T = (const PTerm*)h->d_terms;
    hipStream_t st = stream();
    const int pi = prof_begin(YAO_KF_HPSI);
    if (dtype == YAO_C64 && out_dtype == YAO_C64)
        k_hpsi<float, float><<<grid, kThreads, 0, st>>>((const float2*)data, (float2*)out, rows, B, bg.logBc, G, h->ngroups, T, partial);
    else if (dtype == YAO_C64)
        k_hpsi<float, double><<<grid, kThreads, 0, st>>>((const float2*)data, (double2*)out, rows, B, bg.logBc, G, h->ngroups, T, partial);
    else if (out_dtype == YAO_C64)
        k_hpsi<double, float><<<grid, kThreads, 0, st>>>((const double2*)data, (float2*)out, rows, B, bg.logBc, G, h->ngroups, T, partial);
    else
        k_hpsi<double, double><<<grid, kThreads, 0, st>>>((const double2*)data, (double2*)out, rows, B, bg.logBc, G, h->ngroups, T, partial);
    prof_end(pi, (double)rows * B * ((dtype == YAO_C64 ? 8 : 16) + (out_dtype == YAO_C64 ? 8 : 16)), (double)rows * B * 6.0 * h->nterms_dev);
    YAO_HIP(hipGetLastError());
    if (!energy_host) return 0;
    return finish_slot_sums(partial, B, nbx, energy_host);
}

size_t hpsi_partial_doubles(const yao_pauli_sum* h, int n, int B, int dtype)
{
    if (obs_passes_ok(h, n, B, dtype)) return std::max<size_t>(1, obs_partial_doubles(h, n, B, dtype));
    BatchGeom bg = make_batch_geom(B);
    return (size_t)B * reduce_grid_x(uint64_t(1) << n, bg.logBc);
}

// H psi with the energy left in device memory (energy_dev[b]); nothing synchronises, so the
// launches can be captured in a graph. partial holds hpsi_partial_doubles(n, B) doubles.
int launch_hpsi_dev(const void* data, int dtype, void* out, int out_dtype, int n, int B, const yao_pauli_sum* h,
                    double* partial, double* energy_dev)
{
    if (obs_passes_ok(h, n, B, dtype)) {
        int W = 0;
        YAO_TRY(launch_obs_passes(data, dtype, out, out_dtype, n, B, h, partial, &W));
        // Over several circuits at once, their partial rows follow each other.
        return launch_row_sums(partial, B * zbatch_count(), W, energy_dev);
    }
    if (zbatch_count() > 1) return set_error(YAO_EINVAL, "observable outside the tile passes in a batched launch");
    if (!h->d_groups) return set_error(YAO_EINVAL, "observable tables not uploaded");
    BatchGeom bg = make_batch_geom(B);
    const uint64_t rows = uint64_t(1) << n;
    const int nbx = reduce_grid_x(rows, bg.logBc);
    dim3 grid(nbx, bg.nchunks);
    const PGroup* G = (const PGroup*)h->d_groups;
    const PTerm* T = (const PTerm*)h->d_terms;
    hipStream_t st = stream();
    if (dtype == YAO_C64 && out_dtype == YAO_C64)
        k_hpsi<float, float><<<grid, kThreads, 0, st>>>((const float2*)data, (float2*)out, rows, B, bg.logBc, G, h->ngroups, T, partial);
    else if (dtype == YAO_C64)
        k_hpsi<float, double><<<grid, kThreads, 0, st>>>((const float2*)data, (double2*)out, rows, B, bg.logBc, G, h->ngroups, T, partial);
    else if (out_dtype == YAO_C64)
        k_hpsi<double, float><<<grid, kThreads, 0, st>>>((const double2*)data, (float2*)out, rows, B, bg.logBc, G, h->ngroups, T, partial);
    else
        k_hpsi<double, double><<<grid, kThreads, 0, st>>>((const double2*)data, (double2*)out, rows, B, bg.logBc, G, h->ngroups, T, partial);
    YAO_HIP(hipGetLastError());
    return launch_row_sums(partial, B, nbx, energy_dev);
}

int launch_convert(const void* src, int src_dtype, void* dst, int dst_dtype, size_t elems)
{
    unsigned nb = (unsigned)std::min<uint64_t>((elems + kThreads - 1) / kThreads, 65536);
    hipStream_t st = stream();
    if (src_dtype == YAO_C64 && dst_dtype == YAO_C64)
        k_convert<float, float><<<nb, kThreads, 0, st>>>((const float2*)src, (float2*)dst, elems);
    else if (src_dtype == YAO_C64)
        k_convert<float, double><<<nb, kThreads, 0, st>>>((const float2*)src, (double2*)dst, elems);
    else if (dst_dtype == YAO_C64)
        k_convert<double, float><<<nb, kThreads, 0, st>>>((const double2*)src, (float2*)dst, elems);
    else
        k_convert<double, double><<<nb, kThreads, 0, st>>>((const double2*)src, (double2*)dst, elems);
    YAO_HIP(hipGetLastError());
    return 0;
}

int launch_inner(const void* a, int a_dtype, const void* b, int b_dtype, int n, int B, double* re, double* im)
{
    BatchGeom bg = make_batch_geom(B);
    const uint64_t rows = uint64_t(1) << n;
    const int nbx = reduce_grid_x(rows, bg.logBc);
    double* partial = (double*)workspace(WS_PARTIAL, sizeof(double) * 2 * (size_t)B * nbx);
    if (!partial) return YAO_ENOMEM;
    dim3 grid(nbx, bg.nchunks);
    hipStream_t st = stream();
    if (a_dtype == YAO_C64 && b_dtype == YAO_C64)
        k_inner<float, float><<<grid, kThreads, 0, st>>>((const float2*)a, (const float2*)b, rows, B, bg.logBc, partial);
    else if (a_dtype == YAO_C64)
        k_inner<float, double><<<grid, kThreads, 0, st>>>((const float2*)a, (const double2*)b, rows, B, bg.logBc, partial);
    else if (b_dtype == YAO_C64)
        k_inner<double, float><<<grid, kThreads, 0, st>>>((const double2*)a, (const float2*)b, rows, B, bg.logBc, partial);
    else
        k_inner<double, double><<<grid, kThreads, 0, st>>>((const double2*)a, (const double2*)b, rows, B, bg.logBc, partial);
    YAO_HIP(hipGetLastError());
    std::vector<double> both(2 * (size_t)B);
    YAO_TRY(finish_slot_sums(partial, 2 * B, nbx, both.data()));
    for (int s = 0; s < B; ++s) {
        re[s] = both[s];
        im[s] = both[B + s];
    }
    return 0;
}

int launch_maxdiff(const void* a, int a_dtype, const void* b, int b_dtype, size_t elems, double* out)
{
    const unsigned nb = 512;
    double* partial = (double*)workspace(WS_PARTIAL2, sizeof(double) * nb);
    if (!partial) return YAO_ENOMEM;
    hipStream_t st = stream();
    if (a_dtype == YAO_C128 && b_dtype == YAO_C64)
        k_maxdiff<double, float><<<nb, kThreads, 0, st>>>((const double2*)a, (const float2*)b, elems, partial);
    else if (a_dtype == YAO_C128 && b_dtype == YAO_C128)
        k_maxdiff<double, double><<<nb, kThreads, 0, st>>>((const double2*)a, (const double2*)b, elems, partial);
    else if (a_dtype == YAO_C64 && b_dtype == YAO_C64)
        k_maxdiff<float, float><<<nb, kThreads, 0, st>>>((const float2*)a, (const float2*)b, elems, partial);
    else
        k_maxdiff<float, double><<<nb, kThreads, 0, st>>>((const float2*)a, (const double2*)b, elems, partial);
    YAO_HIP(hipGetLastError());
    double* hs = (double*)host_staging(sizeof(double) * nb);
    if (!hs) return YAO_ENOMEM;
    YAO_HIP(hipMemcpyAsync(hs, partial, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    YAO_HIP(hipStreamSynchronize(st));
    double m = 0;
    for (unsigned t = 0; t < nb; ++t) m = hs[t] > m ? hs[t] : m;
    *out = m;
    return 0;
}

int adjoint_nblk(int n, int k, int B)
{
    BatchGeom bg = make_batch_geom(B);
    return reduce_grid_x(uint64_t(1) << (n - k), bg.logBc);
}

template <typename RL, int K>
static int adjoint_k(double* psi, void* lam, int n, int B, const int* locs, CtrlSpec c, const AdjMats1& m1,
                     const double* dm, bool grad, double* partial, int pstride)
{
    BatchGeom bg = make_batch_geom(B);
    uint64_t rows = uint64_t(1) << (n - K);
    int nbx = reduce_grid_x(rows, bg.logBc);
    dim3 grid(nbx, bg.nchunks);
    GroupGeom<K> gg = make_group_geom<K>(locs);
    const double elems = (double)(uint64_t(1) << n) * B / double(uint64_t(1) << __builtin_popcountll(c.mask));
    const int pi = prof_begin(YAO_KF_ADJOINT);
    if (grad)
        k_adjoint<RL, K, true><<<grid, kThreads, 0, stream()>>>((double2*)psi, (vec2_t<RL>*)lam, rows, B, bg.logBc, gg,
                                                                 c.mask, c.val, m1, dm, partial, pstride > 0 ? pstride : nbx);
    else
        k_adjoint<RL, K, false><<<grid, kThreads, 0, stream()>>>((double2*)psi, (vec2_t<RL>*)lam, rows, B, bg.logBc, gg,
                                                                  c.mask, c.val, m1, dm, partial, nbx);
    prof_end(pi, 2.0 * elems * (16 + sizeof(vec2_t<RL>)), ((grad ? 8.0 : 0.0) + 2.0 * (8.0 * (1 << K) - 2.0)) * elems);
    YAO_HIP(hipGetLastError());
    return 0;
}

static int adjoint_step_impl(double* psi, void* lam, int lam_dtype, int n, int B, const HostMat& Ud, const HostMat* M,
                             const int* locs, CtrlSpec c, const double* dev_mats, double* partial, int pstride)
{
    const int k = Ud.k;
    AdjMats1 m1;
    memset(&m1, 0, sizeof(m1));
    if (k == 1) {
        for (int t = 0; t < 4; ++t) {
            m1.udr[t] = Ud.re[t];
            m1.udi[t] = Ud.im[t];
            if (M) {
                m1.mr[t] = M->re[t];
                m1.mi[t] = M->im[t];
            }
        }
    } else if (!dev_mats) {
        const size_t dd = size_t(1) << (2 * k);
        std::vector<double> h(4 * dd, 0.0);
        for (size_t t = 0; t < dd; ++t) {
            h[t] = Ud.re[t];
            h[dd + t] = Ud.im[t];
            if (M) {
                h[2 * dd + t] = M->re[t];
                h[3 * dd + t] = M->im[t];
            }
        }
        dev_mats = (const double*)ring_upload(h.data(), h.size() * sizeof(double));
        if (!dev_mats) return YAO_ENOMEM;
    }
    const bool g = M != nullptr;
    const double* dm = dev_mats;
#define YAO_ADJ_CASES(RL)                                                                  \
    switch (k) {                                                                           \
    case 1: return adjoint_k<RL, 1>(psi, lam, n, B, locs, c, m1, dm, g, partial, pstride);          \
    case 2: return adjoint_k<RL, 2>(psi, lam, n, B, locs, c, m1, dm, g, partial, pstride);          \
    case 3: return adjoint_k<RL, 3>(psi, lam, n, B, locs, c, m1, dm, g, partial, pstride);          \
    case 4: return adjoint_k<RL, 4>(psi, lam, n, B, locs, c, m1, dm, g, partial, pstride);          \
    case 5: return adjoint_k<RL, 5>(psi, lam, n, B, locs, c, m1, dm, g, partial, pstride);          \
    default: return set_error(YAO_EINVAL, "k = %d not supported", k);                      \
    }
    if (lam_dtype == YAO_C64) {
        YAO_ADJ_CASES(float)
    } else {
        YAO_ADJ_CASES(double)
    }
#undef YAO_ADJ_CASES
}

int launch_adjoint_step(double* psi, void* lam, int lam_dtype, int n, int B, const HostMat& Ud, const HostMat* M,
                        const int* locs, CtrlSpec c, const double* dev_mats, double* partial, int* nblk)
{
    *nblk = adjoint_nblk(n, 1, B);
    return adjoint_step_impl(psi, lam, lam_dtype, n, B, Ud, M, locs, c, dev_mats, partial, *nblk);
}

// Same, with the per-slot partial rows pstride apart (pstride >= the launch's block count).
int launch_adjoint_step_strided(double* psi, void* lam, int lam_dtype, int n, int B, const HostMat& Ud,
                                const HostMat* M, const int* locs, CtrlSpec c, const double* dev_mats, double* partial,
                                int pstride)
{
    return adjoint_step_impl(psi, lam, lam_dtype, n, B, Ud, M, locs, c, dev_mats, partial, pstride);
}

int launch_fill(double* p, size_t count, double v)
{
    unsigned nb = (unsigned)std::min<uint64_t>((count + 255) / 256, 4096);
    k_fill<<<nb, 256, 0, stream()>>>(p, count, v);
    YAO_HIP(hipGetLastError());
    return 0;
}

}  // namespace yao
