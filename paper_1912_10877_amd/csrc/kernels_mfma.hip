// Dense 4- and 5-qubit gates on complex64 states with FP32 matrix cores.
//
// A K-qubit gate maps each group of D = 2^K amplitudes (the indices that differ only in the
// target bits) through a D x D complex matrix. Taking 32 groups as the columns of a
// 2D x 32 real matrix [Re a; Im a], the update is one real GEMM with the 2D x 2D matrix
// [[Re U, -Im U], [Im U, Re U]]. Each wave computes its 32 columns with
// v_mfma_f32_16x16x4f32: the gate matrix stays in the A-operand registers, the amplitudes
// of each lane's column are gathered once and fed as B operands, and the 16x16 accumulator
// tiles hold the real and imaginary halves of each output amplitude in the same lane.
#include "runtime.h"

namespace yao {

namespace {

template <int K> struct MfmaGeom {
    uint64_t off[1 << K];  // index offset of member s of a group
    int sorted[K];         // target bits ascending, for building group bases
};

template <int K> __device__ __forceinline__ uint64_t mfma_group_base(uint64_t j, const MfmaGeom<K>& g)
{
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const uint64_t lo = j & ((uint64_t(1) << g.sorted[t]) - 1);
        j = ((j >> g.sorted[t]) << (g.sorted[t] + 1)) | lo;
    }
    return j;
}

typedef float v4f __attribute__((ext_vector_type(4)));

// Lane layout of v_mfma_f32_16x16x4f32 (one block): A[i][k] from lane i + 16 k, B[k][j]
// from lane j + 16 k, D[4 (l / 16) + v][l % 16] in accumulator register v of lane l.
template <int K>
__global__ __launch_bounds__(256) void k_dense_mfma(float2* __restrict__ psi, uint64_t ngroups, uint32_t B,
                                                    MfmaGeom<K> gg, uint64_t cmask, uint64_t cval,
                                                    const float* __restrict__ M)
{
    constexpr int D = 1 << K, RD = 2 * D, RT = RD / 16, KC = RD / 4, NA = D / 4;
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const uint64_t col0 = wave * 32;
    if (col0 >= ngroups) return;
    const int q = lane >> 4, cl = lane & 15;
    float a[RT][KC];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) a[rt][kc] = M[(16 * rt + cl) * RD + 4 * kc + q];

#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        const uint64_t g = col0 + 16 * ct + cl;
        const bool valid = g < ngroups;
        const uint64_t j = valid ? g / B : 0;
        const uint64_t b = valid ? g % B : 0;
        const uint64_t base = mfma_group_base<K>(j, gg);
        const bool on = valid && ((base & cmask) == cval);
        float2 amp[NA];
#pragma unroll
        for (int m = 0; m < NA; ++m) {
            amp[m] = make_float2(0.f, 0.f);
            if (valid) amp[m] = psi[(base + gg.off[q + 4 * m]) * B + b];
        }
        v4f acc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const int m = kc % NA;
            const float bv = (kc / NA) == 0 ? amp[m].x : amp[m].y;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][kc], bv, acc[rt], 0, 0, 0);
        }
        if (on) {
#pragma unroll
            for (int rt = 0; rt < RT / 2; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int s = 16 * rt + 4 * q + v;
                    psi[(base + gg.off[s]) * B + b] = make_float2(acc[rt][v], acc[rt + RT / 2][v]);
                }
        }
    }
}

template <int K> MfmaGeom<K> mfma_geom(const int* locs)
{
    MfmaGeom<K> g;
    for (int s = 0; s < (1 << K); ++s) {
        uint64_t o = 0;
        for (int j = 0; j < K; ++j)
            if ((s >> j) & 1) o |= uint64_t(1) << locs[j];
        g.off[s] = o;
    }
    int tmp[K];
    for (int j = 0; j < K; ++j) tmp[j] = locs[j];
    for (int x = 0; x < K; ++x)
        for (int y = x + 1; y < K; ++y)
            if (tmp[y] < tmp[x]) {
                int t = tmp[x];
                tmp[x] = tmp[y];
                tmp[y] = t;
            }
    for (int j = 0; j < K; ++j) g.sorted[j] = tmp[j];
    return g;
}

}  // namespace

bool mfma_supported(int k, int n, int B)
{
    return (k == 4 || k == 5) && ((uint64_t(1) << (n - k)) * (uint64_t)B) < (uint64_t(1) << 40) && B < (1 << 30);
}

// Real form [[Ur, -Ui], [Ui, Ur]] of U in FP32, row-major 2D x 2D: the operand the kernel reads.
void mfma_encode(const HostMat& U, float* h)
{
    const int D = 1 << U.k, RD = 2 * D;
    for (int r = 0; r < D; ++r)
        for (int s = 0; s < D; ++s) {
            const float ur = (float)U.re[r * D + s], ui = (float)U.im[r * D + s];
            h[(size_t)r * RD + s] = ur;
            h[(size_t)r * RD + D + s] = -ui;
            h[(size_t)(D + r) * RD + s] = ui;
            h[(size_t)(D + r) * RD + D + s] = ur;
        }
}

// Dense k = 4 or 5 gate on a complex64 state through matrix cores. dev_mat, when given, holds
// the matrix as mfma_encode lays it out.
int launch_dense_mfma(float2* psi, int n, int B, const HostMat& U, const int* locs, CtrlSpec c, const void* dev_mat)
{
    const int k = U.k, D = 1 << k;
    const float* dm = (const float*)dev_mat;
    if (!dm) {
        std::vector<float> h((size_t)4 * D * D);
        mfma_encode(U, h.data());
        dm = (const float*)ring_upload(h.data(), h.size() * sizeof(float));
        if (!dm) return YAO_ENOMEM;
    }
    const uint64_t ngroups = (uint64_t(1) << (n - k)) * (uint64_t)B;
    const uint64_t waves = (ngroups + 31) / 32;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    const double elems = (double)(uint64_t(1) << n) * B / double(uint64_t(1) << __builtin_popcountll(c.mask));
    const int pi = prof_begin(YAO_KF_MFMA);
    if (k == 4)
        k_dense_mfma<4><<<blocks, 256, 0, stream()>>>(psi, ngroups, (uint32_t)B, mfma_geom<4>(locs), c.mask, c.val, dm);
    else
        k_dense_mfma<5><<<blocks, 256, 0, stream()>>>(psi, ngroups, (uint32_t)B, mfma_geom<5>(locs), c.mask, c.val, dm);
    prof_end(pi, 2.0 * 8.0 * elems, 8.0 * D * (double)(uint64_t(1) << n) * B);
    YAO_HIP(hipGetLastError());
    return 0;
}

}  // namespace yao
