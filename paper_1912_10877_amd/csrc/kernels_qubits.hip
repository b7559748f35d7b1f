// Qubit management and the QFT on a set of qubits, as HBM-bound tile kernels.
//
//  * Qubit permutation (focus! / relax!, Sec. "Active qubits and environment qubits"): qubit q
//    of the input moves to index bit perm[q] of the output. A workgroup gathers one tile, whose
//    rows are all values of a set of index bits T that contains the lowest input bits and the
//    input bits that land on the lowest output bits; the tile is read along the low input
//    bits and written along the low output bits, so both sides move rows of >= 128 contiguous
//    bytes.
//  * QFT on locs (App. "Extending QBIR: emulating QFT circuit"): with the sub-index
//    x = sum_j bit(locs[j]) 2^j, out[y] = 2^{-k/2} sum_x exp(2 pi i rev(x) y / 2^k) psi[x].
//    Writing rev(x) y / 2^k = sum_j x_j y / 2^{j+1} shows that the transform factors into k
//    stages applied in place in the order j = 0..k-1: stage j replaces bit x_j by y_j with the
//    butterfly (a, b) -> ((a + w b), (a - w b)) / sqrt 2, w = exp(2 pi i m / 2^{j+1}), where m is
//    the value of the sub-index bits below j (already y bits). No bit reversal is needed: the
//    output comes out in natural order. The inverse runs the stages backwards with the inverse
//    butterflies. A pass takes up to t consecutive stages: its tile holds their qubits plus the
//    lowest other index bits (for contiguous rows), and every stage of the pass runs in LDS.
//
// The batch stays innermost in both kernels: a tile row is B contiguous slots.
#include <algorithm>

#include "runtime.h"

namespace yao {

namespace {

constexpr int kQThreads = 256;
constexpr int kMaxTileBits = 14;
constexpr int kMaxIndexBits = 40;

// Tile geometry shared by both kernels.
struct TileGeom {
    int m;                        // tile bits (rows = 2^m)
    int nrest;                    // index bits outside the tile (block index bits)
    int B;
    int tpos[kMaxTileBits];       // index bit of tile row bit j (ascending)
    int rpos[kMaxIndexBits];      // index bit of block index bit j (ascending)
};

struct PermGeom {
    TileGeom g;
    int opos_row[kMaxTileBits];   // output index bit of output-ordered row bit j (ascending)
    int src_row[kMaxTileBits];    // input tile row bit that output-ordered row bit j comes from
    int rout[kMaxIndexBits];      // output index bit of block index bit j
};

__device__ __forceinline__ uint64_t deposit_rest(uint64_t r, const int* pos, int count)
{
    uint64_t v = 0;
    for (int j = 0; j < count; ++j) v |= ((r >> j) & 1) << pos[j];
    return v;
}

template <typename V>
__global__ __launch_bounds__(kQThreads) void k_permute(const V* __restrict__ in, V* __restrict__ out, PermGeom pg)
{
    extern __shared__ char lds_raw[];
    V* tile = reinterpret_cast<V*>(lds_raw);
    const TileGeom& g = pg.g;
    const uint64_t r = blockIdx.x;
    const uint64_t base_in = deposit_rest(r, g.rpos, g.nrest);
    const uint64_t base_out = deposit_rest(r, pg.rout, g.nrest);
    const int B = g.B;
    const int E = (1 << g.m) * B;
    for (int e = threadIdx.x; e < E; e += kQThreads) {
        const int row = e / B, b = e - row * B;
        uint64_t idx = base_in;
        for (int j = 0; j < g.m; ++j) idx |= (uint64_t)((row >> j) & 1) << g.tpos[j];
        tile[e] = in[idx * B + b];
    }
    __syncthreads();
    for (int f = threadIdx.x; f < E; f += kQThreads) {
        const int rowo = f / B, b = f - rowo * B;
        uint64_t idx = base_out;
        int row = 0;
        for (int j = 0; j < g.m; ++j) {
            const int bit = (rowo >> j) & 1;
            idx |= (uint64_t)bit << pg.opos_row[j];
            row |= bit << pg.src_row[j];
        }
        out[idx * B + b] = tile[row * B + b];
    }
}

struct QftGeom {
    TileGeom g;
    int j0, j1;                   // stages of this pass
    int stage_row[kMaxIndexBits]; // tile row bit of stage j's qubit (j0 <= j < j1)
    int sub_row[kMaxTileBits];    // sub-index bit carried by tile row bit j, or -1
    int sub_rest[kMaxIndexBits];  // sub-index bit carried by block index bit j, or -1
};

template <typename R> __device__ __forceinline__ void twiddle(uint64_t m, int j, R& c, R& s)
{
    // exp(2 pi i m / 2^{j+1}) = cospi(m / 2^j) + i sinpi(m / 2^j); m < 2^j, so m * 2^-j is exact.
    double sd, cd;
    sincospi(ldexp((double)m, -j), &sd, &cd);
    c = (R)cd;
    s = (R)sd;
}

template <typename R, bool INV>
__global__ __launch_bounds__(kQThreads) void k_qft_pass(vec2_t<R>* __restrict__ psi, QftGeom q)
{
    using V = vec2_t<R>;
    extern __shared__ char lds_raw[];
    V* tile = reinterpret_cast<V*>(lds_raw);
    const TileGeom& g = q.g;
    const uint64_t r = blockIdx.x;
    const uint64_t base = deposit_rest(r, g.rpos, g.nrest);
    uint64_t sub_base = 0;
    for (int j = 0; j < g.nrest; ++j)
        if (q.sub_rest[j] >= 0) sub_base |= ((r >> j) & 1) << q.sub_rest[j];
    const int B = g.B;
    const int E = (1 << g.m) * B;
    for (int e = threadIdx.x; e < E; e += kQThreads) {
        const int row = e / B, b = e - row * B;
        uint64_t idx = base;
        for (int j = 0; j < g.m; ++j) idx |= (uint64_t)((row >> j) & 1) << g.tpos[j];
        tile[e] = psi[idx * B + b];
    }
    const R h = (R)0.70710678118654752440;
    const int npairs = E >> 1;
    for (int st = 0; st < q.j1 - q.j0; ++st) {
        const int j = INV ? q.j1 - 1 - st : q.j0 + st;
        const int rb = q.stage_row[j];
        __syncthreads();
        for (int p = threadIdx.x; p < npairs; p += kQThreads) {
            const int prow = p / B, b = p - prow * B;
            // row with tile bit rb clear, and its partner
            const int lo = prow & ((1 << rb) - 1);
            const int row0 = ((prow >> rb) << (rb + 1)) | lo;
            const int row1 = row0 | (1 << rb);
            uint64_t sub = sub_base;
            for (int t = 0; t < g.m; ++t)
                if (q.sub_row[t] >= 0) sub |= (uint64_t)((row0 >> t) & 1) << q.sub_row[t];
            const uint64_t mval = sub & ((uint64_t(1) << j) - 1);
            R c, s;
            twiddle<R>(mval, j, c, s);
            V a = tile[row0 * B + b], bb = tile[row1 * B + b];
            V o0, o1;
            if (!INV) {
                const R wr = c * bb.x - s * bb.y, wi = c * bb.y + s * bb.x;  // w * b
                o0.x = (a.x + wr) * h;
                o0.y = (a.y + wi) * h;
                o1.x = (a.x - wr) * h;
                o1.y = (a.y - wi) * h;
            } else {
                const R dr = (a.x - bb.x) * h, di = (a.y - bb.y) * h;        // conj(w) (a - b) / sqrt 2
                o0.x = (a.x + bb.x) * h;
                o0.y = (a.y + bb.y) * h;
                o1.x = c * dr + s * di;
                o1.y = c * di - s * dr;
            }
            tile[row0 * B + b] = o0;
            tile[row1 * B + b] = o1;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < E; e += kQThreads) {
        const int row = e / B, b = e - row * B;
        uint64_t idx = base;
        for (int j = 0; j < g.m; ++j) idx |= (uint64_t)((row >> j) & 1) << g.tpos[j];
        psi[idx * B + b] = tile[e];
    }
}

// Lowest `c` index bits make rows of >= 128 contiguous bytes together with the batch.
int contiguity_bits(int B, int elem_bytes, int n)
{
    int c = 0;
    while (c < n && ((size_t)B << c) * (size_t)elem_bytes < 128) ++c;
    return c;
}

// Tile bit budget: a tile of 2^m rows x B slots stays within 32 KiB of LDS.
int tile_budget_bits(int B, int elem_bytes)
{
    int m = 0;
    while (m < kMaxTileBits && ((size_t)B << (m + 1)) * (size_t)elem_bytes <= (size_t)32 * 1024) ++m;
    return m;
}

void fill_rest(TileGeom& g, int n, uint64_t tile_mask)
{
    g.nrest = 0;
    for (int b = 0; b < n; ++b)
        if (!((tile_mask >> b) & 1)) g.rpos[g.nrest++] = b;
    g.m = 0;
    for (int b = 0; b < n; ++b)
        if ((tile_mask >> b) & 1) g.tpos[g.m++] = b;
}

}  // namespace

int launch_permute(const void* in, void* out, int dtype, int n, int B, const int* perm)
{
    const int es = dtype == YAO_C64 ? 8 : 16;
    if (n > kMaxIndexBits) return set_error(YAO_EINVAL, "too many qubits for the permutation kernel");
    int inv[kMaxIndexBits];
    for (int q = 0; q < n; ++q) inv[perm[q]] = q;
    const int c = contiguity_bits(B, es, n);
    const int budget = std::max(tile_budget_bits(B, es), std::min(n, 2 * c));
    uint64_t mask = 0;
    for (int b = 0; b < c; ++b) mask |= (uint64_t(1) << b) | (uint64_t(1) << inv[b]);
    for (int b = 0; b < n && __builtin_popcountll(mask) < std::min(n, budget); ++b) mask |= uint64_t(1) << b;
    PermGeom pg;
    memset(&pg, 0, sizeof(pg));
    pg.g.B = B;
    fill_rest(pg.g, n, mask);
    if (pg.g.m > kMaxTileBits) return set_error(YAO_EINVAL, "permutation tile of %d bits", pg.g.m);
    for (int j = 0; j < pg.g.nrest; ++j) pg.rout[j] = perm[pg.g.rpos[j]];
    // Output-ordered row bits: the tile's output positions ascending.
    int order[kMaxTileBits];
    for (int j = 0; j < pg.g.m; ++j) order[j] = j;
    std::sort(order, order + pg.g.m, [&](int a, int b) { return perm[pg.g.tpos[a]] < perm[pg.g.tpos[b]]; });
    for (int j = 0; j < pg.g.m; ++j) {
        pg.src_row[j] = order[j];
        pg.opos_row[j] = perm[pg.g.tpos[order[j]]];
    }
    const uint64_t blocks = uint64_t(1) << pg.g.nrest;
    if (blocks > 0x7fffffffull) return set_error(YAO_EINVAL, "permutation grid too large");
    const size_t lds = ((size_t)B << pg.g.m) * es;
    const int pi = prof_begin(YAO_KF_PERMUTE);
    if (dtype == YAO_C64)
        k_permute<float2><<<(unsigned)blocks, kQThreads, lds, stream()>>>((const float2*)in, (float2*)out, pg);
    else
        k_permute<double2><<<(unsigned)blocks, kQThreads, lds, stream()>>>((const double2*)in, (double2*)out, pg);
    prof_end(pi, 2.0 * (double)((uint64_t(1) << n) * B) * es, 0.0);
    YAO_HIP(hipGetLastError());
    return 0;
}

int launch_qft(void* data, int dtype, int n, int B, const int* locs, int k, bool inverse)
{
    const int es = dtype == YAO_C64 ? 8 : 16;
    if (n > kMaxIndexBits) return set_error(YAO_EINVAL, "too many qubits for the QFT kernel");
    const int c = contiguity_bits(B, es, n);
    const int budget = std::max(tile_budget_bits(B, es), 1);
    int sub_of_bit[kMaxIndexBits];
    for (int b = 0; b < n; ++b) sub_of_bit[b] = -1;
    for (int j = 0; j < k; ++j) sub_of_bit[locs[j]] = j;
    // Passes of consecutive stages: each adds stage qubits while the tile (stage qubits plus the
    // lowest other bits up to the contiguity) fits the budget.
    std::vector<std::pair<int, int>> passes;
    for (int j0 = 0; j0 < k;) {
        int j1 = j0;
        uint64_t smask = 0;
        while (j1 < k) {
            const uint64_t s2 = smask | (uint64_t(1) << locs[j1]);
            uint64_t t2 = s2;
            for (int b = 0; b < c; ++b) t2 |= uint64_t(1) << b;
            if (__builtin_popcountll(t2) > budget && j1 > j0) break;
            smask = s2;
            ++j1;
        }
        passes.push_back({j0, j1});
        j0 = j1;
    }
    // The inverse undoes the stages last to first: passes in reverse order, each pass's stages
    // descending (in the kernel).
    if (inverse) std::reverse(passes.begin(), passes.end());
    const int pi = prof_begin(YAO_KF_QFT);
    for (const auto& ps : passes) {
        QftGeom q;
        memset(&q, 0, sizeof(q));
        q.g.B = B;
        q.j0 = ps.first;
        q.j1 = ps.second;
        uint64_t mask = 0;
        for (int j = q.j0; j < q.j1; ++j) mask |= uint64_t(1) << locs[j];
        for (int b = 0; b < c; ++b) mask |= uint64_t(1) << b;
        // Grow small tiles with the lowest remaining bits (fewer, larger workgroups).
        for (int b = 0; b < n && __builtin_popcountll(mask) < std::min(n, std::min(budget, 10)); ++b)
            mask |= uint64_t(1) << b;
        fill_rest(q.g, n, mask);
        if (q.g.m > kMaxTileBits) return set_error(YAO_EINVAL, "QFT tile of %d bits", q.g.m);
        for (int j = 0; j < q.g.m; ++j) q.sub_row[j] = sub_of_bit[q.g.tpos[j]];
        for (int j = 0; j < q.g.nrest; ++j) q.sub_rest[j] = sub_of_bit[q.g.rpos[j]];
        for (int j = q.j0; j < q.j1; ++j)
            for (int t = 0; t < q.g.m; ++t)
                if (q.g.tpos[t] == locs[j]) q.stage_row[j] = t;
        const uint64_t blocks = uint64_t(1) << q.g.nrest;
        if (blocks > 0x7fffffffull) return set_error(YAO_EINVAL, "QFT grid too large");
        const size_t lds = ((size_t)B << q.g.m) * es;
        if (dtype == YAO_C64) {
            if (inverse) k_qft_pass<float, true><<<(unsigned)blocks, kQThreads, lds, stream()>>>((float2*)data, q);
            else k_qft_pass<float, false><<<(unsigned)blocks, kQThreads, lds, stream()>>>((float2*)data, q);
        } else {
            if (inverse) k_qft_pass<double, true><<<(unsigned)blocks, kQThreads, lds, stream()>>>((double2*)data, q);
            else k_qft_pass<double, false><<<(unsigned)blocks, kQThreads, lds, stream()>>>((double2*)data, q);
        }
        YAO_HIP(hipGetLastError());
    }
    // Algorithmic traffic: one read and one write of the state per pass; flops: per stage and
    // element, half a complex multiply and a complex add plus the scaling (5 real flops).
    prof_end(pi, 2.0 * (double)passes.size() * (double)((uint64_t(1) << n) * B) * es,
             5.0 * k * (double)((uint64_t(1) << n) * B));
    return 0;
}

int qft_passes(int dtype, int n, int B, const int* locs, int k)
{
    // Same pass split as launch_qft, for callers that report traffic.
    const int es = dtype == YAO_C64 ? 8 : 16;
    const int c = contiguity_bits(B, es, n);
    const int budget = std::max(tile_budget_bits(B, es), 1);
    int count = 0;
    for (int j0 = 0; j0 < k;) {
        int j1 = j0;
        uint64_t smask = 0;
        while (j1 < k) {
            const uint64_t s2 = smask | (uint64_t(1) << locs[j1]);
            uint64_t t2 = s2;
            for (int b = 0; b < c; ++b) t2 |= uint64_t(1) << b;
            if (__builtin_popcountll(t2) > budget && j1 > j0) break;
            smask = s2;
            ++j1;
        }
        ++count;
        j0 = j1;
    }
    return count;
}

}  // namespace yao
