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
//    lowest other index bits (for contiguous rows). Batched states run every stage of a pass
//    in LDS (k_qft_pass); single-slot states of >= 10 qubits run them in registers, a few
//    stages per round, with LDS only to move the tile between rounds (k_qft_b1).
//
// The batch stays innermost in every kernel: a tile row is B contiguous slots.
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

// ------------------------------------------------------------------ QFT passes, one-slot states
// A tile of 2^m rows (m = 10..12) held as 2^RR elements per thread (RR = m - 8, 256 threads).
// A layout assigns RR tile row bits to the register index and the other 8 to the thread index
// (ascending; the lowest 6 are the lanes). A round takes r <= RR consecutive stages whose rows
// are register bits 0..r-1 (the others are fillers), so its butterflies run in registers; the
// tile moves to the next round's layout through LDS, real parts first, then imaginary parts,
// so a workgroup holds half a tile of LDS (16 KiB). The tile's lowest rows are the lowest
// index bits, 256 contiguous bytes; the global load and store use the first and last round's
// layouts when those keep these rows on lanes, else a layout of memory order plus one more
// exchange.
//
// Exchange slots: for the writing layout A and the reading layout B, LDS slot = (row bits
// outside A's lanes, compressed) * 64 + P(row) with P a linear map onto 6 bits that sends A's
// lane rows to the lane numbers and B's lane rows outside A's lanes to the lane numbers of A's
// lane rows outside B's lanes. Both sides' 64 lanes then hit 64 distinct slots modulo 64, and
// slot(row) is linear in the row's bits, so a thread's slots are its thread part XOR a
// register part, from per-bit tables.
//
// Twiddles: in a round whose register bit 0 is global stage J, the y bits below J that a pair's
// twiddle needs are fixed per thread and filler group (M: the block's, the thread rows' and
// the filler rows' sub-index bits below J); the stage J + p twiddle is
// exp(i pi M / 2^{J+p}) * exp(i pi c / 2^p), c the pair's register bits below p. The first
// factor for p = r - 1 comes from four table lookups (roots of unity at 12, 24, 36 and 40 bits
// of pi M / 2^{J+r-1}), the others by squaring; the second is one of eight constants.
// The 2^{-1/2} per stage is one 2^{-nst/2} at the store.
constexpr int kQftB1MaxRounds = 6;
constexpr int kQftB1MaxEx = 7;
constexpr int kQftB1MaxStages = 12;
constexpr int kQftTwEntries = 3 * 4096 + 16;

struct QftExchange {
    uint16_t wth[8], wrg[16];  // LDS slot parts of the writing layout's thread bits / register index
    uint16_t rth[8], rrg[16];  // the same for the reading layout
};

struct QftRound {
    uint64_t tsub[8];  // per thread bit: the sub-index bit (below J) its row carries, else 0
    double2 fill[3];   // per filler bit: exp(i pi 2^s / 2^{J+r-1}) for its row's sub-index bit s
                       // below J, else 1
    int J, r;          // global stage of register bit 0; stages in the round
};

struct QftArgsB1 {
    uint64_t ld_th[8], ld_rg[16];  // state index bits of the first layout's thread bits / register index
    uint64_t st_th[8], st_rg[16];  // the same for the last layout
    int8_t rpos[kMaxIndexBits];    // state index bit of block index bit j
    int8_t rsub[kMaxIndexBits];    // sub-index bit (below the pass) of block index bit j, else -1
    QftRound rd[kQftB1MaxRounds];
    QftExchange x[kQftB1MaxEx];
    double scale;
    int nrest, nrounds, load_ex, store_ex;
};
static_assert(sizeof(QftArgsB1) + 24 <= 4096, "kernel arguments must fit the 4 KiB argument segment");

__device__ __forceinline__ double2 cmul_d(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// w * exp(i pi e / 8), e = 0..7, in the state's real type.
template <typename R, int E>
__device__ __forceinline__ vec2_t<R> rot8(vec2_t<R> w)
{
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, h = 0.70710678118654752440;
    constexpr double cs[8] = {1.0, c1, h, s1, 0.0, -s1, -h, -c1};
    constexpr double sn[8] = {0.0, s1, h, c1, 1.0, c1, h, s1};
    vec2_t<R> o;
    if constexpr (E == 0) {
        o = w;
    } else if constexpr (E == 4) {
        o.x = -w.y;
        o.y = w.x;
    } else {
        const R c = (R)cs[E], s = (R)sn[E];
        o.x = c * w.x - s * w.y;
        o.y = c * w.y + s * w.x;
    }
    return o;
}

// The twiddle of register pair (i, i | 2^P) in a round of r stages: base[g] * exp(i pi c / 2^P).
template <typename R, int P, int I>
__device__ __forceinline__ vec2_t<R> pair_twiddle(vec2_t<R> base)
{
    constexpr int c = I & ((1 << P) - 1);
    return rot8<R, (c << (3 - P)) & 7>(base);
}

template <typename R, bool INV, int NE, int P, int r, int I>
__device__ __forceinline__ void qft_pairs(vec2_t<R> (&v)[NE], const vec2_t<R> (&wb)[NE >> r][r])
{
    if constexpr (I < NE) {
        if constexpr (!((I >> P) & 1)) {
            const vec2_t<R> w = pair_twiddle<R, P, I>(wb[I >> r][P]);
            const vec2_t<R> x0 = v[I], x1 = v[I | (1 << P)];
            if (!INV) {
                const R wr = w.x * x1.x - w.y * x1.y, wi = w.x * x1.y + w.y * x1.x;
                v[I].x = x0.x + wr;
                v[I].y = x0.y + wi;
                v[I | (1 << P)].x = x0.x - wr;
                v[I | (1 << P)].y = x0.y - wi;
            } else {
                const R dr = x0.x - x1.x, di = x0.y - x1.y;
                v[I].x = x0.x + x1.x;
                v[I].y = x0.y + x1.y;
                v[I | (1 << P)].x = w.x * dr + w.y * di;
                v[I | (1 << P)].y = w.x * di - w.y * dr;
            }
        }
        qft_pairs<R, INV, NE, P, r, I + 1>(v, wb);
    }
}

template <typename R, bool INV, int NE, int r, int S>
__device__ __forceinline__ void qft_stages(vec2_t<R> (&v)[NE], const vec2_t<R> (&wb)[NE >> r][r])
{
    if constexpr (S < r) {
        qft_pairs<R, INV, NE, INV ? r - 1 - S : S, r, 0>(v, wb);
        qft_stages<R, INV, NE, r, S + 1>(v, wb);
    }
}

template <typename R, bool INV, int NE, int r>
__device__ __forceinline__ void qft_round(vec2_t<R> (&v)[NE], const double2* __restrict__ tw, uint64_t mt,
                                          const QftRound& rd)
{
    constexpr int NG = NE >> r;
    // Filler group g = 0 from the table; group g from the group without its top bit times that
    // filler bit's factor; every group's stage p < r - 1 by squaring.
    double2 w[NG];
    const uint64_t f = mt << (40 - (rd.J + r - 1));
    w[0] = cmul_d(cmul_d(tw[f >> 28], tw[4096 + ((f >> 16) & 4095)]),
                  cmul_d(tw[8192 + ((f >> 4) & 4095)], tw[12288 + (f & 15)]));
#pragma unroll
    for (int g = 1; g < NG; ++g) {
        const int top = 31 - __builtin_clz(g);
        w[g] = cmul_d(w[g ^ (1 << top)], rd.fill[top]);
    }
    vec2_t<R> wb[NG][r];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        double2 x = w[g];
#pragma unroll
        for (int p = r - 1; p >= 0; --p) {
            wb[g][p].x = (R)x.x;
            wb[g][p].y = (R)x.y;
            if (p > 0) x = cmul_d(x, x);
        }
    }
    qft_stages<R, INV, NE, r, 0>(v, wb);
}

// Moves a thread's elements from layout A to layout B through `tile` (2^m reals); waits first
// for the readers of an earlier exchange when there was one.
template <typename R, int NE>
__device__ __forceinline__ void qft_exchange(R* tile, vec2_t<R> (&v)[NE], const QftExchange& X, int t, bool wait_readers)
{
    if (wait_readers) __syncthreads();
    int ws = 0, rs = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        if ((t >> b) & 1) {
            ws ^= X.wth[b];
            rs ^= X.rth[b];
        }
#pragma unroll
    for (int i = 0; i < NE; ++i) tile[ws ^ X.wrg[i]] = v[i].x;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NE; ++i) v[i].x = tile[rs ^ X.rrg[i]];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NE; ++i) tile[ws ^ X.wrg[i]] = v[i].y;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NE; ++i) v[i].y = tile[rs ^ X.rrg[i]];
}

template <typename R, bool INV, int RR>
__global__ __launch_bounds__(kQThreads) void k_qft_b1(vec2_t<R>* __restrict__ psi, const double2* __restrict__ tw,
                                                     QftArgsB1 q)
{
    using V = vec2_t<R>;
    constexpr int NE = 1 << RR;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    R* tile = reinterpret_cast<R*>(lds_raw);
    const int t = threadIdx.x;
    const uint64_t blk = blockIdx.x;
    uint64_t base = 0, sub_base = 0;
    for (int j = 0; j < q.nrest; ++j)
        if ((blk >> j) & 1) {
            base |= uint64_t(1) << q.rpos[j];
            if (q.rsub[j] >= 0) sub_base |= uint64_t(1) << q.rsub[j];
        }
    V v[NE];
    {
        uint64_t it = base;
#pragma unroll
        for (int b = 0; b < 8; ++b)
            if ((t >> b) & 1) it |= q.ld_th[b];
#pragma unroll
        for (int i = 0; i < NE; ++i) v[i] = psi[it | q.ld_rg[i]];
    }
    int x = 0;
    if (q.load_ex) {
        qft_exchange<R, NE>(tile, v, q.x[0], t, false);
        x = 1;
    }
    for (int k = 0; k < q.nrounds; ++k) {
        if (k > 0) {
            qft_exchange<R, NE>(tile, v, q.x[x], t, x > 0);
            ++x;
        }
        const QftRound& rd = q.rd[k];
        uint64_t mt = sub_base;
#pragma unroll
        for (int b = 0; b < 8; ++b)
            if ((t >> b) & 1) mt |= rd.tsub[b];
        if constexpr (RR >= 4) {
            if (rd.r == 4) qft_round<R, INV, NE, 4>(v, tw, mt, rd);
        }
        if constexpr (RR >= 3) {
            if (rd.r == 3) qft_round<R, INV, NE, 3>(v, tw, mt, rd);
        }
        if (rd.r == 2) qft_round<R, INV, NE, 2>(v, tw, mt, rd);
        if (rd.r == 1) qft_round<R, INV, NE, 1>(v, tw, mt, rd);
    }
    if (q.store_ex) qft_exchange<R, NE>(tile, v, q.x[x], t, x > 0);
    const R sc = (R)q.scale;
    uint64_t ot = base;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        if ((t >> b) & 1) ot |= q.st_th[b];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        V o;
        o.x = v[i].x * sc;
        o.y = v[i].y * sc;
        psi[ot | q.st_rg[i]] = o;
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

// QFT passes: runs of consecutive stages (at most max_stages) whose qubits, with the lowest c
// index bits, fit a tile of `budget` bits.
std::vector<std::pair<int, int>> stage_runs(int c, int budget, int max_stages, const int* locs, int k)
{
    std::vector<std::pair<int, int>> passes;
    for (int j0 = 0; j0 < k;) {
        int j1 = j0;
        uint64_t smask = 0;
        while (j1 < k && j1 - j0 < max_stages) {
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

std::vector<std::pair<int, int>> qft_pass_list(int n, int B, int es, const int* locs, int k)
{
    const int c = contiguity_bits(B, es, n);
    return stage_runs(c, std::max(tile_budget_bits(B, es), std::min(n, c + 1)), kMaxStages, locs, k);
}

// Single-slot states of >= 10 qubits take k_qft_b1: tiles of 32 KiB of state (2^12 complex64
// or 2^11 complex128 rows; half of that in LDS), up to 12 stages per pass.
bool qft_b1_path(int n, int B)
{
    return B == 1 && n >= 10;
}

int qft_b1_tile_bits(int n, int es)
{
    return std::min(n, es == 8 ? 12 : 11);
}

// Lowest index bits of a one-slot QFT tile: 256 contiguous bytes.
int qft_b1_contig(int n, int es)
{
    return std::min(n, contiguity_bits(1, es, n) + 1);
}

std::vector<std::pair<int, int>> qft_pass_list_b1(int n, int es, const int* locs, int k)
{
    return stage_runs(qft_b1_contig(n, es), qft_b1_tile_bits(n, es), kQftB1MaxStages, locs, k);
}

// Roots of unity of the one-slot QFT kernel: exp(i pi a / 2^12), exp(i pi a / 2^24) and
// exp(i pi a / 2^36) for a < 4096, then exp(i pi a / 2^40) for a < 16, rounded from long
// double. Filled once into its own workspace slot.
const double2* qft_twiddles()
{
    static const void* filled = nullptr;
    void* d = workspace(WS_QFTTW, sizeof(double2) * kQftTwEntries);
    if (!d) return nullptr;
    if (d != filled) {
        if (recording()) {
            set_error(YAO_EINVAL, "QFT root table first filled while a graph is being recorded");
            return nullptr;
        }
        std::vector<double> h(2 * (size_t)kQftTwEntries);
        const long double pi = 3.14159265358979323846264338327950288L;
        const int bits[4] = {12, 24, 36, 40};
        for (int t = 0; t < 4; ++t)
            for (int a = 0; a < (t < 3 ? 4096 : 16); ++a) {
                const long double ang = pi * ldexpl((long double)a, -bits[t]);
                h[2 * (4096 * t + a)] = (double)cosl(ang);
                h[2 * (4096 * t + a) + 1] = (double)sinl(ang);
            }
        if (hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, stream()) != hipSuccess ||
            hipStreamSynchronize(stream()) != hipSuccess) {
            set_error(YAO_EHIP, "QFT root table upload failed");
            return nullptr;
        }
        filled = d;
    }
    return (const double2*)d;
}

// A layout of a tile of m rows: register index bit q <-> row rg[q] (RR bits), thread index bit
// b <-> row th[b] (8 bits; the lanes are b < 6).
struct QftLayout {
    int th[8];
    int rg[4];
};

// LDS slots of one exchange from layout a (writes) to layout b (reads); see k_qft_b1.
QftExchange make_exchange(const QftLayout& a, const QftLayout& b, int m, int RR)
{
    uint32_t pv[kMaxTileBits] = {};
    int lane_a[kMaxTileBits];
    bool in_lb[kMaxTileBits] = {};
    for (int t = 0; t < m; ++t) lane_a[t] = -1;
    for (int i = 0; i < 6; ++i) {
        lane_a[a.th[i]] = i;
        in_lb[b.th[i]] = true;
    }
    int free_lanes[6], nfree = 0;
    for (int i = 0; i < 6; ++i)
        if (!in_lb[a.th[i]]) free_lanes[nfree++] = i;
    int used = 0, rank = 0;
    for (int t = 0; t < m; ++t) {
        if (lane_a[t] >= 0) {
            pv[t] = 1u << lane_a[t];
            continue;
        }
        pv[t] = 1u << (6 + rank++);
        if (in_lb[t]) pv[t] |= 1u << free_lanes[used++];
    }
    QftExchange x;
    memset(&x, 0, sizeof(x));
    for (int i = 0; i < 8; ++i) {
        x.wth[i] = (uint16_t)pv[a.th[i]];
        x.rth[i] = (uint16_t)pv[b.th[i]];
    }
    for (int i = 0; i < (1 << RR); ++i)
        for (int q = 0; q < RR; ++q)
            if ((i >> q) & 1) {
                x.wrg[i] ^= (uint16_t)pv[a.rg[q]];
                x.rrg[i] ^= (uint16_t)pv[b.rg[q]];
            }
    return x;
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

namespace {

// One-slot QFT passes (k_qft_b1); see the kernel for the layouts, exchanges and twiddles.
int launch_qft_b1(void* data, int dtype, int n, const int* locs, int k, bool inverse)
{
    const int es = dtype == YAO_C64 ? 8 : 16;
    const int c = qft_b1_contig(n, es);
    const int mt = qft_b1_tile_bits(n, es);
    int sub_of_bit[kMaxIndexBits];
    for (int b = 0; b < n; ++b) sub_of_bit[b] = -1;
    for (int j = 0; j < k; ++j) sub_of_bit[locs[j]] = j;
    std::vector<std::pair<int, int>> passes = qft_pass_list_b1(n, es, locs, k);
    if (inverse) std::reverse(passes.begin(), passes.end());
    const double2* tw = qft_twiddles();
    if (!tw) return YAO_EHIP;
    const double elems = (double)(uint64_t(1) << n);
    for (const auto& ps : passes) {
        const int j0 = ps.first, j1 = ps.second, nst = j1 - j0;
        // Tile: the stage qubits and the lowest c bits, then bits that carry no sub-index bit
        // below j0 (no twiddle depends on them), then the lowest others.
        uint64_t mask = 0;
        for (int j = j0; j < j1; ++j) mask |= uint64_t(1) << locs[j];
        for (int b = 0; b < c; ++b) mask |= uint64_t(1) << b;
        for (int b = 0; b < n && __builtin_popcountll(mask) < mt; ++b)
            if (sub_of_bit[b] < 0 || sub_of_bit[b] >= j0) mask |= uint64_t(1) << b;
        for (int b = 0; b < n && __builtin_popcountll(mask) < mt; ++b) mask |= uint64_t(1) << b;
        std::vector<int> tpos, rpos;
        split_bits(n, mask, tpos, rpos);
        const int m = (int)tpos.size(), RR = m - 8;
        if (RR < 2 || RR > 4) return set_error(YAO_EINVAL, "QFT tile of %d bits", m);
        int row_sub[kMaxTileBits], stage_row[kQftB1MaxStages];
        for (int t = 0; t < m; ++t) {
            row_sub[t] = sub_of_bit[tpos[t]];
            if (row_sub[t] >= j0 && row_sub[t] < j1) stage_row[row_sub[t] - j0] = t;
        }
        QftArgsB1 q;
        memset(&q, 0, sizeof(q));
        q.nrest = (int)rpos.size();
        for (int j = 0; j < q.nrest; ++j) {
            q.rpos[j] = (int8_t)rpos[j];
            const int sb = sub_of_bit[rpos[j]];
            q.rsub[j] = (int8_t)(sb >= 0 && sb < j0 ? sb : -1);
        }
        // Rounds in execution order: runs of RR stages, ascending (forward) or descending.
        std::vector<QftLayout> lay;
        std::vector<int> seq;
        for (int st = 0; st < nst; ++st) seq.push_back(inverse ? nst - 1 - st : st);
        const int nrounds = (nst + RR - 1) / RR;
        if (nrounds > kQftB1MaxRounds) return set_error(YAO_EINVAL, "QFT pass of %d rounds", nrounds);
        for (int rk = 0; rk < nrounds; ++rk) {
            const int a = rk * RR, e = std::min(nst, a + RR);
            int st0 = seq[a];
            for (int i = a; i < e; ++i) st0 = std::min(st0, seq[i]);
            const int r = e - a;
            QftLayout L;
            bool used[kMaxTileBits] = {};
            for (int p = 0; p < r; ++p) {
                L.rg[p] = stage_row[st0 + p];
                used[L.rg[p]] = true;
            }
            for (int p = r, t = m - 1; p < RR; ++p) {  // fillers: the highest other rows
                while (used[t]) --t;
                L.rg[p] = t;
                used[t] = true;
            }
            for (int t = 0, b = 0; t < m; ++t)
                if (!used[t]) L.th[b++] = t;
            QftRound& rd = q.rd[rk];
            rd.J = j0 + st0;
            rd.r = r;
            auto below = [&](int row) -> uint64_t {
                const int sb = row_sub[row];
                return sb >= 0 && sb < rd.J ? uint64_t(1) << sb : 0;
            };
            for (int b = 0; b < 8; ++b) rd.tsub[b] = below(L.th[b]);
            for (int qb = 0; qb < 3; ++qb) {
                rd.fill[qb] = make_double2(1.0, 0.0);
                const int sb = qb < RR - r ? row_sub[L.rg[r + qb]] : -1;
                if (sb >= 0 && sb < rd.J) {
                    const long double ang = 3.14159265358979323846264338327950288L * ldexpl(1.0L, sb - (rd.J + r - 1));
                    rd.fill[qb] = make_double2((double)cosl(ang), (double)sinl(ang));
                }
            }
            lay.push_back(L);
        }
        q.nrounds = nrounds;
        // Global access in memory order (lanes on rows 0..5) unless the first / last round
        // already keeps the c contiguous rows on lanes.
        QftLayout mem;
        for (int b = 0; b < 8; ++b) mem.th[b] = b;
        for (int p = 0; p < RR; ++p) mem.rg[p] = 8 + p;
        auto lanes_contiguous = [&](const QftLayout& L) {
            for (int p = 0; p < RR; ++p)
                if (L.rg[p] < c) return false;
            return true;
        };
        q.load_ex = !lanes_contiguous(lay.front());
        q.store_ex = !lanes_contiguous(lay.back());
        if (q.load_ex) lay.insert(lay.begin(), mem);
        if (q.store_ex) lay.push_back(mem);
        if ((int)lay.size() - 1 > kQftB1MaxEx) return set_error(YAO_EINVAL, "QFT pass of %d exchanges", (int)lay.size() - 1);
        for (size_t i = 0; i + 1 < lay.size(); ++i) q.x[i] = make_exchange(lay[i], lay[i + 1], m, RR);
        const QftLayout &lf = lay.front(), &ll = lay.back();
        for (int b = 0; b < 8; ++b) {
            q.ld_th[b] = uint64_t(1) << tpos[lf.th[b]];
            q.st_th[b] = uint64_t(1) << tpos[ll.th[b]];
        }
        for (int i = 0; i < (1 << RR); ++i)
            for (int p = 0; p < RR; ++p)
                if ((i >> p) & 1) {
                    q.ld_rg[i] |= uint64_t(1) << tpos[lf.rg[p]];
                    q.st_rg[i] |= uint64_t(1) << tpos[ll.rg[p]];
                }
        q.scale = std::pow(2.0, -0.5 * nst);
        const uint64_t blocks = uint64_t(1) << q.nrest;
        if (blocks > 0x7fffffffull) return set_error(YAO_EINVAL, "QFT grid too large");
        const size_t lds = ((size_t)1 << m) * es / 2;
        const int pi = prof_begin(YAO_KF_QFT);
#define YAO_QFT_B1(R, INV, RRv)                                                                \
    do {                                                                                      \
        const void* kf = reinterpret_cast<const void*>(&k_qft_b1<R, INV, RRv>);              \
        k_qft_b1<R, INV, RRv><<<(unsigned)blocks, kQThreads, lds, stream()>>>( \
            (vec2_t<R>*)data, tw, q);                                                        \
    } while (0)
#define YAO_QFT_B1_RR(R, INV)          \
    do {                               \
        if (RR == 2) YAO_QFT_B1(R, INV, 2); \
        else if (RR == 3) YAO_QFT_B1(R, INV, 3); \
        else YAO_QFT_B1(R, INV, 4);    \
    } while (0)
        if (dtype == YAO_C64) {
            if (inverse) YAO_QFT_B1_RR(float, true);
            else YAO_QFT_B1_RR(float, false);
        } else {
            if (inverse) YAO_QFT_B1_RR(double, true);
            else YAO_QFT_B1_RR(double, false);
        }
#undef YAO_QFT_B1_RR
#undef YAO_QFT_B1
        prof_end(pi, 2.0 * elems * es, 5.0 * nst * elems);
        YAO_HIP(hipGetLastError());
    }
    return 0;
}

}  // namespace

int launch_qft(void* data, int dtype, int n, int B, const int* locs, int k, bool inverse)
{
    const int es = dtype == YAO_C64 ? 8 : 16;
    if (n > kMaxIndexBits) return set_error(YAO_EINVAL, "too many qubits for the QFT kernel");
    if (qft_b1_path(n, B)) return launch_qft_b1(data, dtype, n, locs, k, inverse);
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
    const int es = dtype == YAO_C64 ? 8 : 16;
    if (qft_b1_path(n, B)) return (int)qft_pass_list_b1(n, es, locs, k).size();
    return (int)qft_pass_list(n, B, es, locs, k).size();
}

}  // namespace yao
