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
#include <cmath>
#include <vector>

#include "runtime.h"

namespace yao {

namespace {

constexpr int kQThreads = 256;
constexpr int kMaxTileBits = 12;      // row index = low half (6 bits) | high half (6 bits)
constexpr int kMaxIndexBits = 40;
constexpr int kMaxStages = 10;        // stages per QFT pass
constexpr int kMaxCodes = 16;         // values of the tile bits below a pass's first stage

// Index math through two 64-entry halves: f(row) = lo[row & 63] | hi[row >> 6] for any function
// of the row's bits that is a sum (or OR) over them.
__device__ __forceinline__ uint64_t halves(const uint64_t* lo, const uint64_t* hi, int row)
{
    return lo[row & 63] | hi[row >> 6];
}

__device__ __forceinline__ uint64_t deposit_rest(uint64_t r, const int* pos, int count)
{
    uint64_t v = 0;
    for (int j = 0; j < count; ++j) v |= ((r >> j) & 1) << pos[j];
    return v;
}

// ------------------------------------------------------------------------------ permutation
// Tables of a permutation launch (the same for every block): index bits of each tile row in
// memory order of the input, of each output-ordered row, and which input row each output-ordered
// row takes.
struct PermTables {
    uint64_t in_lo[64], in_hi[64];
    uint64_t out_lo[64], out_hi[64];
    uint64_t src_lo[64], src_hi[64];
};

struct PermArgs {
    const PermTables* tab;
    int m, nrest, B;
    int rpos[kMaxIndexBits];  // input index bit of block index bit j
    int rout[kMaxIndexBits];  // output index bit of block index bit j
};

// LDS row of tile row r: the high half XORed into the low half, so that the input-ordered
// reads (low bits varying) and the output-ordered ones (often high bits varying) both spread
// over the banks.
__device__ __forceinline__ int swz_row(int r)
{
    return r ^ ((r >> 6) & 63);
}

template <typename V>
__global__ __launch_bounds__(kQThreads) void k_permute(const V* __restrict__ in, V* __restrict__ out, PermArgs pa)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    PermTables* t = reinterpret_cast<PermTables*>(lds_raw);
    V* tile = reinterpret_cast<V*>(lds_raw + sizeof(PermTables));
    {
        const uint64_t* g = reinterpret_cast<const uint64_t*>(pa.tab);
        uint64_t* d = reinterpret_cast<uint64_t*>(t);
        for (int i = threadIdx.x; i < (int)(sizeof(PermTables) / 8); i += kQThreads) d[i] = g[i];
    }
    const uint64_t r = blockIdx.x;
    const uint64_t base_in = deposit_rest(r, pa.rpos, pa.nrest);
    const uint64_t base_out = deposit_rest(r, pa.rout, pa.nrest);
    const int B = pa.B;
    const int rows = 1 << pa.m;
    __syncthreads();
    if (B == 1) {
        for (int row = threadIdx.x; row < rows; row += kQThreads)
            tile[swz_row(row)] = in[base_in | halves(t->in_lo, t->in_hi, row)];
        __syncthreads();
        for (int ro = threadIdx.x; ro < rows; ro += kQThreads)
            out[base_out | halves(t->out_lo, t->out_hi, ro)] = tile[swz_row((int)halves(t->src_lo, t->src_hi, ro))];
    } else {
        const int E = rows * B;
        for (int e = threadIdx.x; e < E; e += kQThreads) {
            const int row = B == 1 ? e : e / B, b = e - row * B;
            tile[swz_row(row) * B + b] = in[(base_in | halves(t->in_lo, t->in_hi, row)) * B + b];
        }
        __syncthreads();
        for (int f = threadIdx.x; f < E; f += kQThreads) {
            const int ro = B == 1 ? f : f / B, b = f - ro * B;
            const int row = (int)halves(t->src_lo, t->src_hi, ro);
            out[(base_out | halves(t->out_lo, t->out_hi, ro)) * B + b] = tile[swz_row(row) * B + b];
        }
    }
}

// Single-slot states with tiles of 256 * NPER rows: row e = threadIdx.x + 256 i, so the row's
// low table half is the lane's (fixed for the launch) and its high half the wave's (uniform);
// the tables come by value with the arguments (scalar loads, nothing staged in LDS) and every
// thread's NPER loads are issued before the first LDS write.
struct PermArgsB1 {
    PermTables tab;
    int nrest;
    int rpos[kMaxIndexBits];
    int rout[kMaxIndexBits];
};
static_assert(sizeof(PermArgsB1) + 16 <= 4096, "kernel arguments must fit the 4 KiB argument segment");

template <typename V, int NPER>
__global__ __launch_bounds__(kQThreads) void k_permute_b1(const V* __restrict__ in, V* __restrict__ out, PermArgsB1 pa)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    V* tile = reinterpret_cast<V*>(lds_raw);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t r = blockIdx.x;
    const uint64_t base_in = deposit_rest(r, pa.rpos, pa.nrest) | pa.tab.in_lo[lane];
    const uint64_t base_out = deposit_rest(r, pa.rout, pa.nrest) | pa.tab.out_lo[lane];
    const int slo = (int)pa.tab.src_lo[lane];
    V v[NPER];
#pragma unroll
    for (int i = 0; i < NPER; ++i) v[i] = in[base_in | pa.tab.in_hi[wave + 4 * i]];
#pragma unroll
    for (int i = 0; i < NPER; ++i) tile[swz_row(threadIdx.x + kQThreads * i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NPER; ++i)
        out[base_out | pa.tab.out_hi[wave + 4 * i]] = tile[swz_row(slo | (int)pa.tab.src_hi[wave + 4 * i])];
}

// ------------------------------------------------------------------------------ QFT passes
struct QftTables {
    uint64_t in_lo[64], in_hi[64];  // index bits of each tile row (memory order)
    uint64_t v_lo[64], v_hi[64];    // the row's stage bits, stage j at bit j - j0
    uint64_t c_lo[64], c_hi[64];    // code of the row's bits that carry sub-index bits below j0
    uint64_t code_sub[kMaxCodes];   // sub-index bits (below j0) that each code stands for
};

struct QftArgs {
    const QftTables* tab;
    int m, nrest, B, j0, nst, ncodes;
    int stage_row[kMaxStages];      // tile row bit of stage j0 + st
    int rpos[kMaxIndexBits];        // index bit of block index bit j
    int rsub[kMaxIndexBits];        // sub-index bit carried by block index bit j (-1: none)
};

template <typename R, bool INV>
__global__ __launch_bounds__(kQThreads) void k_qft_pass(vec2_t<R>* __restrict__ psi, QftArgs q)
{
    using V = vec2_t<R>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    QftTables* t = reinterpret_cast<QftTables*>(lds_raw);
    double2* bt = reinterpret_cast<double2*>(lds_raw + sizeof(QftTables));  // [nst][ncodes]
    double2* tin = bt + kMaxStages * kMaxCodes;  // exp(i pi a / 2^st) at (2^st - 1) + a, a < 2^st
    V* tile = reinterpret_cast<V*>(tin + (1 << q.nst));
    {
        const uint64_t* g = reinterpret_cast<const uint64_t*>(q.tab);
        uint64_t* d = reinterpret_cast<uint64_t*>(t);
        for (int i = threadIdx.x; i < (int)(sizeof(QftTables) / 8); i += kQThreads) d[i] = g[i];
    }
    const uint64_t r = blockIdx.x;
    const uint64_t base = deposit_rest(r, q.rpos, q.nrest);
    uint64_t sub_base = 0;
    for (int j = 0; j < q.nrest; ++j)
        if (q.rsub[j] >= 0) sub_base |= ((r >> j) & 1) << q.rsub[j];
    sub_base &= (uint64_t(1) << q.j0) - 1;
    __syncthreads();
    // Twiddle factors of a stage st = j - j0: exp(i pi a / 2^st) for the pass's own stage bits
    // below j (a < 2^st), and exp(i pi b / 2^j) for b = this block's bits below j0 plus those
    // the code's tile bits carry; the pair's factor is their product.
    for (int i = threadIdx.x; i < (1 << q.nst) - 1; i += kQThreads) {
        int st = 0;
        while ((2 << st) - 1 <= i) ++st;
        const int a = i - ((1 << st) - 1);
        double s, c;
        sincospi(ldexp((double)a, -st), &s, &c);
        tin[i] = make_double2(c, s);
    }
    for (int i = threadIdx.x; i < q.nst * q.ncodes; i += kQThreads) {
        const int st = i / q.ncodes, code = i - st * q.ncodes;
        const uint64_t b = sub_base | t->code_sub[code];
        double s, c;
        sincospi(ldexp((double)b, -(q.j0 + st)), &s, &c);
        bt[i] = make_double2(c, s);
    }
    const int B = q.B;
    const int rows = 1 << q.m;
    const int E = rows * B;
    for (int e = threadIdx.x; e < E; e += kQThreads) {
        const int row = B == 1 ? e : e / B, b = e - row * B;
        tile[e] = psi[(base | halves(t->in_lo, t->in_hi, row)) * B + b];
    }
    const R h = (R)0.70710678118654752440;
    const int npairs = E >> 1;
    for (int k = 0; k < q.nst; ++k) {
        const int st = INV ? q.nst - 1 - k : k;
        const int rb = q.stage_row[st];
        __syncthreads();
        for (int p = threadIdx.x; p < npairs; p += kQThreads) {
            const int prow = B == 1 ? p : p / B, b = p - prow * B;
            const int row0 = ((prow >> rb) << (rb + 1)) | (prow & ((1 << rb) - 1));
            const int row1 = row0 | (1 << rb);
            const int a = (int)(halves(t->v_lo, t->v_hi, row0) & ((1u << st) - 1));
            const int code = (int)halves(t->c_lo, t->c_hi, row0);
            const double2 w1 = tin[(1 << st) - 1 + a], w2 = bt[st * q.ncodes + code];
            const R c = (R)(w1.x * w2.x - w1.y * w2.y), s = (R)(w1.x * w2.y + w1.y * w2.x);
            const V x0 = tile[row0 * B + b], x1 = tile[row1 * B + b];
            V o0, o1;
            if (!INV) {
                const R wr = c * x1.x - s * x1.y, wi = c * x1.y + s * x1.x;  // w * x1
                o0.x = (x0.x + wr) * h;
                o0.y = (x0.y + wi) * h;
                o1.x = (x0.x - wr) * h;
                o1.y = (x0.y - wi) * h;
            } else {
                const R dr = (x0.x - x1.x) * h, di = (x0.y - x1.y) * h;  // conj(w) (x0 - x1) / sqrt 2
                o0.x = (x0.x + x1.x) * h;
                o0.y = (x0.y + x1.y) * h;
                o1.x = c * dr + s * di;
                o1.y = c * di - s * dr;
            }
            tile[row0 * B + b] = o0;
            tile[row1 * B + b] = o1;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < E; e += kQThreads) {
        const int row = B == 1 ? e : e / B, b = e - row * B;
        psi[(base | halves(t->in_lo, t->in_hi, row)) * B + b] = tile[e];
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

// The two 64-entry halves of f over the m bits of a row: f(row) = sum of f(bit j) over set bits.
void fill_halves(uint64_t* lo, uint64_t* hi, int m, const uint64_t* f_of_bit)
{
    for (int h = 0; h < 64; ++h) {
        uint64_t a = 0, b = 0;
        for (int j = 0; j < 6; ++j) {
            if (!((h >> j) & 1)) continue;
            if (j < m) a |= f_of_bit[j];
            if (j + 6 < m) b |= f_of_bit[j + 6];
        }
        lo[h] = a;
        hi[h] = b;
    }
}

// Tile rows: the index bits of `mask` in ascending order; block bits: the others ascending.
void split_bits(int n, uint64_t mask, std::vector<int>& tpos, std::vector<int>& rpos)
{
    tpos.clear();
    rpos.clear();
    for (int b = 0; b < n; ++b) ((mask >> b) & 1 ? tpos : rpos).push_back(b);
}

// QFT passes: runs of consecutive stages whose qubits, with the lowest c index bits, fit the
// tile budget (at most kMaxStages stages).
std::vector<std::pair<int, int>> qft_pass_list(int n, int B, int es, const int* locs, int k)
{
    const int c = contiguity_bits(B, es, n);
    const int budget = std::max(tile_budget_bits(B, es), std::min(n, c + 1));
    std::vector<std::pair<int, int>> passes;
    for (int j0 = 0; j0 < k;) {
        int j1 = j0;
        uint64_t smask = 0;
        while (j1 < k && j1 - j0 < kMaxStages) {
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
    return passes;
}

}  // namespace

int launch_permute(const void* in, void* out, int dtype, int n, int B, const int* perm)
{
    const int es = dtype == YAO_C64 ? 8 : 16;
    if (n > kMaxIndexBits) return set_error(YAO_EINVAL, "too many qubits for the permutation kernel");
    int inv[kMaxIndexBits];
    for (int q = 0; q < n; ++q) inv[perm[q]] = q;
    // Tile bits: the lowest input bits and the input bits of the lowest output bits, grown
    // alternately (longer contiguous runs on both sides) up to the budget.
    const int budget = std::min(n, std::max(tile_budget_bits(B, es), 2 * contiguity_bits(B, es, n)));
    uint64_t mask = 0;
    for (int a = 0; a < n && __builtin_popcountll(mask) < budget; ++a) {
        mask |= uint64_t(1) << a;
        if (__builtin_popcountll(mask) < budget) mask |= uint64_t(1) << inv[a];
    }
    std::vector<int> tpos, rpos;
    split_bits(n, mask, tpos, rpos);
    const int m = (int)tpos.size();
    if (m > kMaxTileBits) return set_error(YAO_EINVAL, "permutation tile of %d bits", m);
    PermArgs pa;
    memset(&pa, 0, sizeof(pa));
    pa.m = m;
    pa.nrest = (int)rpos.size();
    pa.B = B;
    for (int j = 0; j < pa.nrest; ++j) {
        pa.rpos[j] = rpos[j];
        pa.rout[j] = perm[rpos[j]];
    }
    // Output-ordered rows: the tile's bits sorted by their output position.
    std::vector<int> order(m);
    for (int j = 0; j < m; ++j) order[j] = j;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return perm[tpos[a]] < perm[tpos[b]]; });
    uint64_t fin[kMaxTileBits], fout[kMaxTileBits], fsrc[kMaxTileBits];
    for (int j = 0; j < m; ++j) {
        fin[j] = uint64_t(1) << tpos[j];
        fout[j] = uint64_t(1) << perm[tpos[order[j]]];
        fsrc[j] = uint64_t(1) << order[j];
    }
    PermTables tab;
    fill_halves(tab.in_lo, tab.in_hi, m, fin);
    fill_halves(tab.out_lo, tab.out_hi, m, fout);
    fill_halves(tab.src_lo, tab.src_hi, m, fsrc);
    if (B == 1 && m >= 8 && m <= 12) {
        // Tiles of 256 .. 4096 rows on single-slot states: the table-by-value kernel.
        PermArgsB1 pb;
        memset(&pb, 0, sizeof(pb));
        pb.tab = tab;
        pb.nrest = pa.nrest;
        for (int j = 0; j < pa.nrest; ++j) {
            pb.rpos[j] = pa.rpos[j];
            pb.rout[j] = pa.rout[j];
        }
        const uint64_t nb = uint64_t(1) << pa.nrest;
        if (nb > 0x7fffffffull) return set_error(YAO_EINVAL, "permutation grid too large");
        const size_t lds1 = ((size_t)1 << m) * es;
        const int pi = prof_begin(YAO_KF_PERMUTE);
#define YAO_PERM_B1(V, NP) k_permute_b1<V, NP><<<(unsigned)nb, kQThreads, lds1, stream()>>>((const V*)in, (V*)out, pb)
        if (dtype == YAO_C64) {
            switch (m) {
            case 8: YAO_PERM_B1(float2, 1); break;
            case 9: YAO_PERM_B1(float2, 2); break;
            case 10: YAO_PERM_B1(float2, 4); break;
            case 11: YAO_PERM_B1(float2, 8); break;
            default: YAO_PERM_B1(float2, 16); break;
            }
        } else {
            switch (m) {
            case 8: YAO_PERM_B1(double2, 1); break;
            case 9: YAO_PERM_B1(double2, 2); break;
            case 10: YAO_PERM_B1(double2, 4); break;
            case 11: YAO_PERM_B1(double2, 8); break;
            default: YAO_PERM_B1(double2, 16); break;
            }
        }
#undef YAO_PERM_B1
        prof_end(pi, 2.0 * (double)((uint64_t(1) << n) * B) * es, 0.0);
        YAO_HIP(hipGetLastError());
        return 0;
    }
    pa.tab = (const PermTables*)ring_upload(&tab, sizeof(tab));
    if (!pa.tab) return YAO_ENOMEM;
    const uint64_t blocks = uint64_t(1) << pa.nrest;
    if (blocks > 0x7fffffffull) return set_error(YAO_EINVAL, "permutation grid too large");
    const size_t lds = sizeof(PermTables) + ((size_t)B << m) * es;
    const int pi = prof_begin(YAO_KF_PERMUTE);
    if (dtype == YAO_C64)
        k_permute<float2><<<(unsigned)blocks, kQThreads, lds, stream()>>>((const float2*)in, (float2*)out, pa);
    else
        k_permute<double2><<<(unsigned)blocks, kQThreads, lds, stream()>>>((const double2*)in, (double2*)out, pa);
    prof_end(pi, 2.0 * (double)((uint64_t(1) << n) * B) * es, 0.0);
    YAO_HIP(hipGetLastError());
    return 0;
}

int launch_qft(void* data, int dtype, int n, int B, const int* locs, int k, bool inverse)
{
    const int es = dtype == YAO_C64 ? 8 : 16;
    if (n > kMaxIndexBits) return set_error(YAO_EINVAL, "too many qubits for the QFT kernel");
    const int c = contiguity_bits(B, es, n);
    const int budget = std::max(tile_budget_bits(B, es), std::min(n, c + 1));
    int sub_of_bit[kMaxIndexBits];
    for (int b = 0; b < n; ++b) sub_of_bit[b] = -1;
    for (int j = 0; j < k; ++j) sub_of_bit[locs[j]] = j;
    std::vector<std::pair<int, int>> passes = qft_pass_list(n, B, es, locs, k);
    // The inverse undoes the stages last to first: passes in reverse order, each pass's stages
    // descending (in the kernel).
    if (inverse) std::reverse(passes.begin(), passes.end());
    const double elems = (double)((uint64_t(1) << n) * B);
    for (const auto& ps : passes) {
        const int j0 = ps.first, j1 = ps.second;
        uint64_t mask = 0;
        for (int j = j0; j < j1; ++j) mask |= uint64_t(1) << locs[j];
        for (int b = 0; b < c; ++b) mask |= uint64_t(1) << b;
        // Grow small tiles (fewer, larger workgroups) with the lowest bits that carry no
        // sub-index bit below j0, so the twiddles of those bits stay per workgroup.
        for (int b = 0; b < n && __builtin_popcountll(mask) < std::min(n, std::min(budget, 10)); ++b)
            if (sub_of_bit[b] < 0 || sub_of_bit[b] >= j0) mask |= uint64_t(1) << b;
        std::vector<int> tpos, rpos;
        split_bits(n, mask, tpos, rpos);
        const int m = (int)tpos.size();
        if (m > kMaxTileBits) return set_error(YAO_EINVAL, "QFT tile of %d bits", m);
        QftArgs q;
        memset(&q, 0, sizeof(q));
        q.m = m;
        q.nrest = (int)rpos.size();
        q.B = B;
        q.j0 = j0;
        q.nst = j1 - j0;
        for (int j = 0; j < q.nrest; ++j) {
            q.rpos[j] = rpos[j];
            q.rsub[j] = sub_of_bit[rpos[j]];
        }
        uint64_t fin[kMaxTileBits], fv[kMaxTileBits], fc[kMaxTileBits];
        std::vector<uint64_t> code_bits;  // sub-index bit of each code bit
        for (int t = 0; t < m; ++t) {
            fin[t] = uint64_t(1) << tpos[t];
            const int sb = sub_of_bit[tpos[t]];
            fv[t] = (sb >= j0 && sb < j1) ? uint64_t(1) << (sb - j0) : 0;
            if (sb >= j0 && sb < j1) q.stage_row[sb - j0] = t;
            fc[t] = 0;
            if (sb >= 0 && sb < j0) {
                fc[t] = uint64_t(1) << code_bits.size();
                code_bits.push_back(uint64_t(1) << sb);
            }
        }
        q.ncodes = 1 << code_bits.size();
        if (q.ncodes > kMaxCodes) return set_error(YAO_EINVAL, "QFT tile with %d low code bits", (int)code_bits.size());
        QftTables tab;
        memset(&tab, 0, sizeof(tab));
        fill_halves(tab.in_lo, tab.in_hi, m, fin);
        fill_halves(tab.v_lo, tab.v_hi, m, fv);
        fill_halves(tab.c_lo, tab.c_hi, m, fc);
        for (int cd = 0; cd < q.ncodes; ++cd) {
            uint64_t sbits = 0;
            for (size_t j = 0; j < code_bits.size(); ++j)
                if ((cd >> j) & 1) sbits |= code_bits[j];
            tab.code_sub[cd] = sbits;
        }
        q.tab = (const QftTables*)ring_upload(&tab, sizeof(tab));
        if (!q.tab) return YAO_ENOMEM;
        const uint64_t blocks = uint64_t(1) << q.nrest;
        if (blocks > 0x7fffffffull) return set_error(YAO_EINVAL, "QFT grid too large");
        const size_t lds = sizeof(QftTables) + sizeof(double2) * (kMaxStages * kMaxCodes + (1 << q.nst)) +
                           ((size_t)B << m) * es;
        // Algorithmic work of a pass: one read and one write of the state; per stage and element
        // half a complex multiply and a complex add plus the scaling (5 real flops).
        const int pi = prof_begin(YAO_KF_QFT);
        if (dtype == YAO_C64) {
            if (inverse) k_qft_pass<float, true><<<(unsigned)blocks, kQThreads, lds, stream()>>>((float2*)data, q);
            else k_qft_pass<float, false><<<(unsigned)blocks, kQThreads, lds, stream()>>>((float2*)data, q);
        } else {
            if (inverse) k_qft_pass<double, true><<<(unsigned)blocks, kQThreads, lds, stream()>>>((double2*)data, q);
            else k_qft_pass<double, false><<<(unsigned)blocks, kQThreads, lds, stream()>>>((double2*)data, q);
        }
        prof_end(pi, 2.0 * elems * es, 5.0 * q.nst * elems);
        YAO_HIP(hipGetLastError());
    }
    return 0;
}

int qft_passes(int dtype, int n, int B, const int* locs, int k)
{
    return (int)qft_pass_list(n, B, dtype == YAO_C64 ? 8 : 16, locs, k).size();
}

}  // namespace yao
