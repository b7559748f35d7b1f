// Dense 4- and 5-qubit gates on complex64 states with FP32 matrix cores.
//
// A K-qubit gate maps each group of D = 2^K amplitudes (the indices that differ only in the
// target bits) through a D x D complex matrix. Taking 32 groups as the columns of a
// 2D x 32 real matrix [Re a; Im a], the update is one real GEMM with the 2D x 2D matrix
// [[Re U, -Im U], [Im U, Re U]], which each wave computes with v_mfma_f32_16x16x4f32: the gate
// matrix stays in the A-operand registers, each lane's column is read once as B operands, and
// the 16x16 accumulator tiles hold the real and imaginary halves of each output amplitude in the
// same lane.
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

// Lane layout of v_mfma_f32_16x16x4f32 (one block): A[i][k] from lane i + 16 k, B[k][j]
// from lane j + 16 k, D[4 (l / 16) + v][l % 16] in accumulator register v of lane l.
// FULL: the tile holds exactly 4096 amplitudes, so every load and store loop has a fixed trip
// count and the wait for the next tile's registers need not include the stores issued after them.
template <int K, bool FULL>
__global__ __launch_bounds__(256) void k_dense_mfma(float2* __restrict__ psi, MfmaArgs a, const float* __restrict__ M)
{
    constexpr int D = 1 << K, RD = 2 * D, RT = RD / 16, KC = RD / 4, NA = D / 4;
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
    float am[RT][KC];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) am[rt][kc] = M[(16 * rt + cl) * RD + 4 * kc + q];
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
                float2 amp[NA];
#pragma unroll
                for (int m = 0; m < NA; ++m)
                    amp[m] = valid ? tile[swz5(r0 | t->mem[q + 4 * m]) * B + b] : make_float2(0.f, 0.f);
                v4f acc[RT];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) acc[rt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) {
                    const int m = kc % NA;
                    const float bv = (kc / NA) == 0 ? amp[m].x : amp[m].y;
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[rt][kc], bv, acc[rt], 0, 0, 0);
                }
                if (on) {
#pragma unroll
                    for (int rt = 0; rt < RT / 2; ++rt)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int s = 16 * rt + 4 * q + v;
                            tile[swz5(r0 | t->mem[s]) * B + b] = make_float2(acc[rt][v], acc[rt + RT / 2][v]);
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
    constexpr int D = 1 << K, RD = 2 * D, RT = RD / 16, KC = RD / 4, NA = D / 4;
    constexpr int NBLK = (4096 >> K) / 64;  // 16-column blocks per wave
    constexpr int kPer = 16;                // amplitudes per thread and tile
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float2* buf = reinterpret_cast<float2*>(lds_raw);  // two tiles of 4096 amplitudes
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q = lane >> 4, cl = lane & 15;
    float am[RT][KC];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) am[rt][kc] = M[(16 * rt + cl) * RD + 4 * kc + q];
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
            float2 amp[NA];
#pragma unroll
            for (int m = 0; m < NA; ++m) amp[m] = t[swz5(r0[j] | memq | (int)a.tab.mem[4 * m])];
            v4f acc[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[rt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                const int m = kc % NA;
                const float bv = (kc / NA) == 0 ? amp[m].x : amp[m].y;
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[rt][kc], bv, acc[rt], 0, 0, 0);
            }
            if (on) {
#pragma unroll
                for (int rt = 0; rt < RT / 2; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        t[swz5(r0[j] | memq4 | (int)a.tab.mem[16 * rt + v])] = make_float2(acc[rt][v], acc[rt + RT / 2][v]);
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
    // Algorithmic work: one read and one write of every element; 8 D real flops per element
    // (for the elements whose controls pass).
    const double on = elems / double(uint64_t(1) << __builtin_popcountll(c.mask));
    prof_end(pi, 2.0 * 8.0 * elems, 8.0 * D * on);
    YAO_HIP(hipGetLastError());
    return 0;
}

}  // namespace yao
