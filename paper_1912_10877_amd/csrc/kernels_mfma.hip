// Dense 4- and 5-qubit gates on complex64 states with FP32 matrix cores.
//
// A K-qubit gate maps each group of D = 2^K amplitudes (the indices that differ only in the
// target bits) through a D x D complex matrix U = Ur + i Ui. Taking 16 groups as the columns
// of real D x 16 matrices Ar, Ai (real and imaginary parts), the update uses three real products
// instead of four: P1 = Ur Ar, P2 = Ui Ai, P3 = (Ur + Ui)(Ar + Ai), then Re = P1 - P2 and
// Im = P3 - P1 - P2 (the three-multiplication form of a complex product). Each wave computes them
// with v_mfma_f32_16x16x4f32: the three matrices stay in the A-operand registers, each lane's
// column is read once as B operands (Ar + Ai formed in registers), and the accumulator tiles of
// P1, P2, P3 hold the same output amplitudes in the same lanes.
//
// The amplitudes move through LDS: a workgroup loads a tile of 2^m index rows (the K target
// bits and the lowest other bits, so every tile row run is contiguous in memory whatever the
// targets), the waves run their columns out of LDS, and the tile is stored back the same way.
#include <algorithm>
#include <vector>

#include "runtime.h"

namespace yao {

namespace {

constexpr int kMfmaTileBits = 12;  // 2^12 complex64 rows: 32 KiB of LDS per batch slot

// Per-launch tables (the same for every workgroup).
struct MfmaTables {
    uint64_t in_lo[64], in_hi[64];   // index bits of tile row r: in_lo[r & 63] | in_hi[r >> 6]
    uint32_t col_lo[64], col_hi[64]; // tile row of column (group) g: col_lo[g & 63] | col_hi[g >> 6]
    uint32_t mem[32];                // tile-row offset of member s of a group
};

// Passed by value: a launch recorded into a graph keeps its own copy of the tables.
struct MfmaArgs {
    MfmaTables tab;
    uint64_t ntiles;
    int m, K, nrest, B;
    uint64_t cmask, cval;
    int rpos[40];  // index bit of block index bit j
};

static_assert(sizeof(MfmaArgs) + 16 <= 4096, "kernel arguments must fit the 4 KiB argument segment");

typedef float v4f __attribute__((ext_vector_type(4)));

// LDS row of tile row r: bits 5..9 XORed into bits 0..4. Tile loads and stores run along
// consecutive rows (low bits varying), a wave's 16 columns along the column bits, which sit
// above the targets when the targets are low qubits; the swizzle spreads both over the banks.
__device__ __forceinline__ int swz5(int r)
{
    return r ^ ((r >> 5) & 31);
}

// The three products of one 16-column block: B operands Ar, Ai and Ar + Ai of member
// 4 kc + (lane / 16), A operands the lane's fragments of Ur, Ui and Ur + Ui.
template <int RT, int KC>
__device__ __forceinline__ void mul3(const float (&am)[3][RT][KC], const float2 (&amp)[KC], v4f (&acc)[3][RT])
{
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[w][rt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        const float xr = amp[kc].x, xi = amp[kc].y, xs = xr + xi;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            acc[0][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[0][rt][kc], xr, acc[0][rt], 0, 0, 0);
            acc[1][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[1][rt][kc], xi, acc[1][rt], 0, 0, 0);
            acc[2][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[2][rt][kc], xs, acc[2][rt], 0, 0, 0);
        }
    }
}

// Output amplitude in accumulator register v of row tile rt: (P1 - P2, P3 - P1 - P2).
template <int RT>
__device__ __forceinline__ float2 out3(const v4f (&acc)[3][RT], int rt, int v)
{
    const float p1 = acc[0][rt][v], p2 = acc[1][rt][v];
    return make_float2(p1 - p2, acc[2][rt][v] - p1 - p2);
}

// Lane layout of v_mfma_f32_16x16x4f32 (one block): A[i][k] from lane i + 16 k, B[k][j]
// from lane j + 16 k, D[4 (l / 16) + v][l % 16] in accumulator register v of lane l.
// FULL: the tile holds exactly 4096 amplitudes, so every load and store loop has a fixed trip
// count and the wait for the next tile's registers need not include the stores issued after them.
template <int K, bool FULL>
__global__ __launch_bounds__(256) void k_dense_mfma(float2* __restrict__ psi, MfmaArgs a, const float* __restrict__ M)
{
    constexpr int D = 1 << K, RT = D / 16, KC = D / 4;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    MfmaTables* t = reinterpret_cast<MfmaTables*>(lds_raw);
    float2* tile = reinterpret_cast<float2*>(lds_raw + sizeof(MfmaTables));
    {
        const uint32_t* g = reinterpret_cast<const uint32_t*>(&a.tab);
        uint32_t* d = reinterpret_cast<uint32_t*>(t);
        for (int i = threadIdx.x; i < (int)(sizeof(MfmaTables) / 4); i += 256) d[i] = g[i];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, cl = lane & 15;
    float am[3][RT][KC];
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) am[w][rt][kc] = M[w * D * D + (16 * rt + cl) * D + 4 * kc + q];
    const int B = a.B;
    const int rows = 1 << a.m;
    const int E = FULL ? 4096 : rows * B;
    const int ncols = E >> K;  // (group, slot) columns of a tile
    // Workgroups loop over tiles, so the matrix fragments above are read once per workgroup;
    // the next tile's amplitudes are loaded into registers while the current one is computed
    // and stored (a tile holds at most 4096 amplitudes: 16 per thread).
    constexpr int kPer = 4096 / 256;
    float2 pre[kPer];
    auto tile_base = [&](uint64_t tix) {
        uint64_t base = 0;
        for (int j = 0; j < a.nrest; ++j) base |= ((tix >> j) & 1) << a.rpos[j];
        return base;
    };
    auto gload = [&](uint64_t base) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + 256 * i;
            if (FULL || e < E) {
                const int row = B == 1 ? e : e / B, b = e - row * B;
                pre[i] = psi[(base | t->in_lo[row & 63] | t->in_hi[row >> 6]) * B + b];
            }
        }
    };
    if (blockIdx.x < a.ntiles) {
        __syncthreads();  // the tables are in LDS
        gload(tile_base(blockIdx.x));
    }
    for (uint64_t tix = blockIdx.x; tix < a.ntiles; tix += gridDim.x) {
        const uint64_t base = tile_base(tix);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + 256 * i;
            if (FULL || e < E) {
                const int row = B == 1 ? e : e / B, b = e - row * B;
                tile[swz5(row) * B + b] = pre[i];
            }
        }
        __syncthreads();
        if (tix + gridDim.x < a.ntiles) gload(tile_base(tix + gridDim.x));
        for (int c0 = wave * 32; c0 < ncols; c0 += 4 * 32) {
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
                const int col = c0 + 16 * ct + cl;
                const bool valid = col < ncols;
                const int g = !valid ? 0 : (B == 1 ? col : col / B), b = valid ? col - g * B : 0;
                const int r0 = (int)(t->col_lo[g & 63] | t->col_hi[g >> 6]);
                const uint64_t idx0 = base | t->in_lo[r0 & 63] | t->in_hi[r0 >> 6];
                const bool on = valid && ((idx0 & a.cmask) == a.cval);
                float2 amp[KC];
#pragma unroll
                for (int m = 0; m < KC; ++m)
                    amp[m] = valid ? tile[swz5(r0 | t->mem[q + 4 * m]) * B + b] : make_float2(0.f, 0.f);
                v4f acc[3][RT];
                mul3<RT, KC>(am, amp, acc);
                if (on) {
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int s = 16 * rt + 4 * q + v;
                            tile[swz5(r0 | t->mem[s]) * B + b] = out3(acc, rt, v);
                        }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + 256 * i;
            if (FULL || e < E) {
                const int row = B == 1 ? e : e / B, b = e - row * B;
                psi[(base | t->in_lo[row & 63] | t->in_hi[row >> 6]) * B + b] = tile[swz5(row) * B + b];
            }
        }
    }
}

// Single-slot states with full tiles (B = 1, 2^12 rows): element e = threadIdx.x + 256 i of a
// tile is row e, so its address is base | in_lo[lane] | in_hi[wave + 4 i], a per-lane part fixed
// for the whole launch and a wave-uniform one. Two LDS tiles alternate: while the waves multiply
// one, the next tile's amplitudes (loaded into registers during the previous multiply) are
// written into the other and the finished one is stored, so each wait for loads covers only
// loads and stores issued a whole multiply earlier.
template <int K>
__global__ __launch_bounds__(256) void k_dense_mfma_b1(float2* __restrict__ psi, MfmaArgs a, const float* __restrict__ M)
{
    constexpr int D = 1 << K, RT = D / 16, KC = D / 4;
    constexpr int NBLK = (4096 >> K) / 64;  // 16-column blocks per wave
    constexpr int kPer = 16;                // amplitudes per thread and tile
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float2* buf = reinterpret_cast<float2*>(lds_raw);  // two tiles of 4096 amplitudes
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q = lane >> 4, cl = lane & 15;
    float am[3][RT][KC];
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) am[w][rt][kc] = M[w * D * D + (16 * rt + cl) * D + 4 * kc + q];
    const uint64_t lo = a.tab.in_lo[lane];
    // Group columns of this lane (block wave + 4 j): first row, and the row bits that decide
    // its controls; member offsets split into a per-lane part and a uniform part (the member
    // table is linear in the member index bits).
    int r0[NBLK];
    uint64_t tctl[NBLK];
#pragma unroll
    for (int j = 0; j < NBLK; ++j) {
        const int col = 16 * (wave + 4 * j) + cl;
        r0[j] = (int)(a.tab.col_lo[col & 63] | a.tab.col_hi[col >> 6]);
        tctl[j] = (a.tab.in_lo[r0[j] & 63] | a.tab.in_hi[r0[j] >> 6]) & a.cmask;
    }
    const int memq = (int)a.tab.mem[q], memq4 = (int)a.tab.mem[4 * q];
    auto tile_base = [&](uint64_t tix) {
        uint64_t base = 0;
        for (int j = 0; j < a.nrest; ++j) base |= ((tix >> j) & 1) << a.rpos[j];
        return base;
    };
    float2 pre[kPer];
    auto gload = [&](uint64_t base) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) pre[i] = psi[base | lo | a.tab.in_hi[wave + 4 * i]];
    };
    auto lput = [&](float2* t) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) t[swz5(threadIdx.x + 256 * i)] = pre[i];
    };
    const uint64_t G = gridDim.x;
    uint64_t tix = blockIdx.x;
    gload(tile_base(tix));
    lput(buf);
    if (tix + G < a.ntiles) gload(tile_base(tix + G));
    __syncthreads();
    int cur = 0;
    for (; tix < a.ntiles; tix += G) {
        const uint64_t base = tile_base(tix);
        float2* t = buf + cur * 4096;
#pragma unroll
        for (int j = 0; j < NBLK; ++j) {
            const bool on = ((base & a.cmask) | tctl[j]) == a.cval;
            float2 amp[KC];
#pragma unroll
            for (int m = 0; m < KC; ++m) amp[m] = t[swz5(r0[j] | memq | (int)a.tab.mem[4 * m])];
            v4f acc[3][RT];
            mul3<RT, KC>(am, amp, acc);
            if (on) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        t[swz5(r0[j] | memq4 | (int)a.tab.mem[16 * rt + v])] = out3(acc, rt, v);
            }
        }
        __syncthreads();
        const uint64_t nx = tix + G;
        if (nx < a.ntiles) lput(buf + (cur ^ 1) * 4096);
#pragma unroll
        for (int i = 0; i < kPer; ++i) psi[base | lo | a.tab.in_hi[wave + 4 * i]] = t[swz5(threadIdx.x + 256 * i)];
        if (nx + G < a.ntiles) gload(tile_base(nx + G));
        __syncthreads();
        cur ^= 1;
    }
}

}  // namespace

bool mfma_supported(int k, int n, int B)
{
    // A tile holds at least the 2^k members x B slots of a group, at most 4096 amplitudes
    // (32 KiB of LDS, 16 per thread in the prefetch registers).
    return (k == 4 || k == 5) && n >= k && n - kMfmaTileBits < 31 && ((size_t)B << k) <= 4096;
}

// Ur, Ui and Ur + Ui of U in FP32 (the sum formed in FP64), each row-major D x D, one after
// the other: the operands the kernels read.
void mfma_encode(const HostMat& U, float* h)
{
    const size_t DD = size_t(1) << (2 * U.k);
    for (size_t e = 0; e < DD; ++e) {
        h[e] = (float)U.re[e];
        h[DD + e] = (float)U.im[e];
        h[2 * DD + e] = (float)(U.re[e] + U.im[e]);
    }
}

// Dense k = 4 or 5 gate on a complex64 state through matrix cores. dev_mat, when given, holds
// the matrix as mfma_encode lays it out.
int launch_dense_mfma(float2* psi, int n, int B, const HostMat& U, const int* locs, CtrlSpec c, const void* dev_mat)
{
    const int k = U.k, D = 1 << k;
    const float* dm = (const float*)dev_mat;
    if (!dm) {
        std::vector<float> h((size_t)3 * D * D);
        mfma_encode(U, h.data());
        dm = (const float*)ring_upload(h.data(), h.size() * sizeof(float));
        if (!dm) return YAO_ENOMEM;
    }
    // Tile bits: the targets and the lowest other index bits, up to 2^12 rows (fewer rows for
    // wide batches: the tile holds 2^m rows x B slots within 32 KiB).
    int mmax = kMfmaTileBits;
    while (mmax > k && ((size_t)B << mmax) * 8 > (size_t)32 * 1024) --mmax;
    uint64_t mask = 0;
    for (int j = 0; j < k; ++j) mask |= uint64_t(1) << locs[j];
    for (int b = 0; b < n && __builtin_popcountll(mask) < std::min(n, mmax); ++b) mask |= uint64_t(1) << b;
    MfmaArgs a;
    memset(&a, 0, sizeof(a));
    a.K = k;
    a.B = B;
    a.cmask = c.mask;
    a.cval = c.val;
    std::vector<int> tpos;
    for (int b = 0; b < n; ++b) ((mask >> b) & 1 ? tpos.push_back(b) : (void)(a.rpos[a.nrest++] = b));
    a.m = (int)tpos.size();
    MfmaTables& tab = a.tab;
    for (int h = 0; h < 64; ++h)
        for (int j = 0; j < 6; ++j) {
            if (!((h >> j) & 1)) continue;
            if (j < a.m) tab.in_lo[h] |= uint64_t(1) << tpos[j];
            if (j + 6 < a.m) tab.in_hi[h] |= uint64_t(1) << tpos[j + 6];
        }
    // Row bits of the targets (member bits) and of the other tile bits (column bits).
    int trow[8], nt = 0, crow[kMfmaTileBits], nc = 0;
    for (int r = 0; r < a.m; ++r) {
        bool tgt = false;
        for (int j = 0; j < k; ++j) tgt |= tpos[r] == locs[j];
        if (tgt) continue;
        crow[nc++] = r;
    }
    for (int j = 0; j < k; ++j)
        for (int r = 0; r < a.m; ++r)
            if (tpos[r] == locs[j]) trow[nt++] = r;
    for (int s = 0; s < D; ++s) {
        uint32_t o = 0;
        for (int j = 0; j < k; ++j)
            if ((s >> j) & 1) o |= 1u << trow[j];
        tab.mem[s] = o;
    }
    for (int h = 0; h < 64; ++h)
        for (int j = 0; j < 6; ++j) {
            if (!((h >> j) & 1)) continue;
            if (j < nc) tab.col_lo[h] |= 1u << crow[j];
            if (j + 6 < nc) tab.col_hi[h] |= 1u << crow[j + 6];
        }
    a.ntiles = uint64_t(1) << a.nrest;
    if (((size_t)B << a.m) > 4096) return set_error(YAO_EINVAL, "matrix-core tile of %zu amplitudes", (size_t)B << a.m);
    // About eight workgroups per CU, each looping over tiles.
    const uint64_t blocks = std::min<uint64_t>(a.ntiles, 2048);
    const size_t lds = sizeof(MfmaTables) + ((size_t)B << a.m) * 8;
    const double elems = (double)(uint64_t(1) << n) * B;
    const int pi = prof_begin(YAO_KF_MFMA);
    const bool full = ((size_t)B << a.m) == 4096;
    if (B == 1 && full) {
        // Two tiles of 32 KiB; two workgroups per CU.
        const size_t lds2 = 2 * 4096 * sizeof(float2);
        if (k == 4) {
            YAO_HIP(hipFuncSetAttribute((const void*)k_dense_mfma_b1<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));
            k_dense_mfma_b1<4><<<(unsigned)blocks, 256, lds2, stream()>>>(psi, a, dm);
        } else {
            YAO_HIP(hipFuncSetAttribute((const void*)k_dense_mfma_b1<5>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));
            k_dense_mfma_b1<5><<<(unsigned)blocks, 256, lds2, stream()>>>(psi, a, dm);
        }
    } else if (k == 4 && full) k_dense_mfma<4, true><<<(unsigned)blocks, 256, lds, stream()>>>(psi, a, dm);
    else if (k == 4) k_dense_mfma<4, false><<<(unsigned)blocks, 256, lds, stream()>>>(psi, a, dm);
    else if (full) k_dense_mfma<5, true><<<(unsigned)blocks, 256, lds, stream()>>>(psi, a, dm);
    else k_dense_mfma<5, false><<<(unsigned)blocks, 256, lds, stream()>>>(psi, a, dm);
    // Work: one read and one write of every element; per element whose controls pass, 6 D real
    // flops on the matrix cores (three real products; the complex product by definition takes
    // 8 D, the additions forming Ar + Ai and the outputs run on the vector units).
    const double on = elems / double(uint64_t(1) << __builtin_popcountll(c.mask));
    prof_end(pi, 2.0 * 8.0 * elems, 6.0 * D * on);
    YAO_HIP(hipGetLastError());
    return 0;
}

}  // namespace yao
