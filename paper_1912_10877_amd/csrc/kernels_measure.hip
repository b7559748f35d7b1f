// Measurement of batched registers (Listing "instruct! and measure": measure samples bit strings,
// measure! also collapses the state; Sec. "Batched Quantum Registers": every batch slot is
// measured on its own).
//
// Outcomes of the qubits locs are the sub-index x = sum_j bit(locs[j]) 2^j. The pipeline, all in
// FP64 and in a fixed order (so results repeat bit for bit):
//   1. probabilities P[b][x] of every outcome: |psi|^2 summed over the other qubits (the locs
//      are first moved onto the lowest index bits by a qubit permutation unless they already
//      are 0..k-1 in order);
//   2. the cumulative sums C[b][x] = sum_{y <= x} P[b][y], held as chunks of 2048 outcomes
//      scanned in LDS (Q) and the exclusive scan of the chunk totals per slot (O), so that
//      C[x] = Q[x] + O[chunk of x] (chunk 0: Q[x]);
//   3. each shot s of slot b takes the smallest x with C[b][x] > u[b][s] * C[b][last] for a
//      caller-supplied uniform number u in [0, 1): a binary search over the chunk boundaries,
//      then one inside the chunk;
//   4. measure! keeps the amplitudes whose locs read the outcome and divides them by
//      sqrt(P[b][x_b]); the others become 0.
#include <algorithm>

#include "runtime.h"

namespace yao {

namespace {

constexpr int kMThreads = 256;
constexpr int kChunk = 2048;          // outcomes per scanned chunk (8 per thread)

// P[b][x] = sum_e |psi[(e * 2^k + x) * B + b]|^2. Memory row t = x * B + b (rows = B * 2^k of
// them, contiguous) repeats for every env index e. A block takes RB = min(rows, 256) consecutive
// rows and the env range of chunk blockIdx.y; its threads form G env groups (G the largest power
// of two with G * RB <= 256), each summing every G-th env row, and the groups are added in LDS
// in a fixed tree. The chunk's sum
// goes to partial[chunk][b * 2^k + x].
template <typename R>
__global__ __launch_bounds__(kMThreads) void k_marginal(const vec2_t<R>* __restrict__ psi, int k, int B, int RB,
                                                        uint64_t nenv, uint64_t env_per_chunk,
                                                        double* __restrict__ partial)
{
    __shared__ double red[kMThreads];
    const uint64_t rows = (uint64_t)B << k;
    int G = 1;  // env groups: a power of two, G * RB <= 256
    while (G * 2 * RB <= kMThreads) G *= 2;
    const int g = threadIdx.x / RB, rr = threadIdx.x - g * RB;
    const uint64_t t = (uint64_t)blockIdx.x * RB + rr;
    const uint64_t c = blockIdx.y;
    const uint64_t e0 = c * env_per_chunk;
    const uint64_t e1 = e0 + env_per_chunk < nenv ? e0 + env_per_chunk : nenv;
    double acc = 0;
    if (g < G && t < rows)
        for (uint64_t e = e0 + g; e < e1; e += G) {
            const vec2_t<R> a = psi[e * rows + t];
            acc += (double)a.x * a.x + (double)a.y * a.y;
        }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = G >> 1; h > 0; h >>= 1) {
        if (g < h) red[threadIdx.x] += red[threadIdx.x + h * RB];
        __syncthreads();
    }
    if (g == 0 && t < rows) {
        const uint64_t x = t / B, b = t - x * B;
        partial[c * rows + (b << k) + x] = red[threadIdx.x];
    }
}

// out[r] = sum_c partial[c][r] in chunk order.
__global__ __launch_bounds__(kMThreads) void k_sum_chunks(const double* __restrict__ partial, uint64_t rows, int nchunks,
                                                          double* __restrict__ out)
{
    const uint64_t r = (uint64_t)blockIdx.x * kMThreads + threadIdx.x;
    if (r >= rows) return;
    double s = 0;
    for (int c = 0; c < nchunks; ++c) s += partial[(uint64_t)c * rows + r];
    out[r] = s;
}

// Inclusive scan of one chunk of kChunk values of slot b (rows of length len) from p to q
// (which may be p); chunk totals to tot[b * nchunks + chunk]. The chunk goes through LDS so that
// global loads and stores run along contiguous addresses (element e = threadIdx.x + 256 i);
// thread i then scans the 8 consecutive values 8i..8i+7 (one padding slot per 32 values keeps
// those reads on distinct banks), the 256 thread sums are scanned in LDS (Hillis-Steele, fixed
// order), and each thread adds its prefix.
__global__ __launch_bounds__(kMThreads) void k_scan_chunks(const double* p, double* q, uint64_t len, int nchunks,
                                                           double* __restrict__ tot)
{
    __shared__ double vals[kChunk + kChunk / 32];
    __shared__ double sh[2][kMThreads];
    const int b = blockIdx.y;
    const uint64_t base = (uint64_t)b * len + (uint64_t)blockIdx.x * kChunk;
    const uint64_t lim = len - (uint64_t)blockIdx.x * kChunk;
    auto slot = [](int e) { return e + (e >> 5); };
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int e = threadIdx.x + kMThreads * i;
        vals[slot(e)] = (uint64_t)e < lim ? p[base + e] : 0.0;
    }
    __syncthreads();
    double v[8];
    double run = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        run += vals[slot(threadIdx.x * 8 + j)];
        v[j] = run;
    }
    int cur = 0;
    sh[cur][threadIdx.x] = run;
    __syncthreads();
    for (int d = 1; d < kMThreads; d <<= 1) {
        const double add = (int)threadIdx.x >= d ? sh[cur][threadIdx.x - d] : 0.0;
        sh[cur ^ 1][threadIdx.x] = sh[cur][threadIdx.x] + add;
        cur ^= 1;
        __syncthreads();
    }
    const double prefix = threadIdx.x > 0 ? sh[cur][threadIdx.x - 1] : 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) vals[slot(threadIdx.x * 8 + j)] = v[j] + prefix;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int e = threadIdx.x + kMThreads * i;
        if ((uint64_t)e < lim) q[base + e] = vals[slot(e)];
    }
    if (threadIdx.x == kMThreads - 1) tot[(uint64_t)b * nchunks + blockIdx.x] = sh[cur][kMThreads - 1];
}

// Exclusive scan of the chunk totals of slot b = blockIdx.x: thread i scans a contiguous
// segment, the segment totals are scanned in LDS, then each thread writes its exclusive prefixes
// O[c]; then the last cumulative sum of every chunk, Q[last of c] + O[c], to tot[B * nchunks +
// b * nchunks + c] (the table the sampling searches first).
__global__ __launch_bounds__(kMThreads) void k_scan_totals(double* __restrict__ tot, int nchunks,
                                                           const double* __restrict__ q, uint64_t len)
{
    __shared__ double sh[2][kMThreads];
    double* t = tot + (uint64_t)blockIdx.x * nchunks;
    const int seg = (nchunks + kMThreads - 1) / kMThreads;
    const int c0 = threadIdx.x * seg, c1 = c0 + seg < nchunks ? c0 + seg : nchunks;
    double run = 0;
    for (int c = c0; c < c1; ++c) run += t[c];
    int cur = 0;
    sh[cur][threadIdx.x] = run;
    __syncthreads();
    for (int d = 1; d < kMThreads; d <<= 1) {
        const double add = (int)threadIdx.x >= d ? sh[cur][threadIdx.x - d] : 0.0;
        sh[cur ^ 1][threadIdx.x] = sh[cur][threadIdx.x] + add;
        cur ^= 1;
        __syncthreads();
    }
    double pre = threadIdx.x > 0 ? sh[cur][threadIdx.x - 1] : 0.0;
    for (int c = c0; c < c1; ++c) {
        const double v = t[c];
        t[c] = pre;
        pre += v;
    }
    __syncthreads();
    double* last = tot + (uint64_t)gridDim.x * nchunks + (uint64_t)blockIdx.x * nchunks;
    const double* Q = q + (uint64_t)blockIdx.x * len;
    for (int c = threadIdx.x; c < nchunks; c += kMThreads) {
        const uint64_t e = (uint64_t)c * kChunk + kChunk - 1;
        const double v = Q[e < len ? e : len - 1];
        last[c] = c > 0 ? v + t[c] : v;
    }
}

// Shots s of slot b: smallest x with C[b][x] > u * C[b][last], C[x] = Q[x] + O[x / kChunk]
// (chunk 0: Q[x]). First the chunk: the smallest c whose last entry C exceeds the target; then
// the entry inside it. Each thread takes kShots shots of one slot whose searches run level by
// level together, so their loads are in flight at once.
constexpr int kShots = 2;
__global__ __launch_bounds__(kMThreads) void k_sample(const double* __restrict__ q, const double* __restrict__ off,
                                                      uint64_t len, int nchunks, int B, int nshots,
                                                      const double* __restrict__ u, uint64_t* __restrict__ out)
{
    const int per = (nshots + kShots - 1) / kShots;
    const uint64_t t = (uint64_t)blockIdx.x * kMThreads + threadIdx.x;
    if (t >= (uint64_t)B * per) return;
    const uint64_t b = t / per;
    const int s0 = (int)(t - b * per) * kShots;
    const double* Q = q + b * len;
    const double* O = off + b * (uint64_t)nchunks;
    const int lastc = nchunks - 1;
    const double total = Q[len - 1] + (lastc > 0 ? O[lastc] : 0.0);
    double target[kShots];
    int clo[kShots], chi[kShots];
#pragma unroll
    for (int i = 0; i < kShots; ++i) {
        const int s = s0 + i < nshots ? s0 + i : nshots - 1;
        target[i] = u[b * nshots + s] * total;
        clo[i] = 0;
        chi[i] = lastc;
    }
    // Chunk: smallest c in [0, lastc] whose last entry exceeds the target (c = lastc when none).
    const double* Last = off + ((uint64_t)B + b) * (uint64_t)nchunks;
    auto chunk_last = [&](int c) { return Last[c]; };
    for (int step = 0; step < 32; ++step) {
        bool any = false;
#pragma unroll
        for (int i = 0; i < kShots; ++i)
            if (clo[i] < chi[i]) {
                any = true;
                const int mid = (clo[i] + chi[i]) >> 1;
                if (chunk_last(mid) > target[i]) chi[i] = mid;
                else clo[i] = mid + 1;
            }
        if (!any) break;
    }
    uint64_t lo[kShots], hi[kShots];
    double o[kShots];
#pragma unroll
    for (int i = 0; i < kShots; ++i) {
        lo[i] = (uint64_t)clo[i] * kChunk;
        const uint64_t end = lo[i] + kChunk;
        hi[i] = (end < len ? end : len) - 1;
        o[i] = clo[i] > 0 ? O[clo[i]] : 0.0;
    }
    for (int step = 0; step < 32; ++step) {
        bool any = false;
#pragma unroll
        for (int i = 0; i < kShots; ++i)
            if (lo[i] < hi[i]) {
                any = true;
                const uint64_t mid = (lo[i] + hi[i]) >> 1;
                const double c = clo[i] > 0 ? Q[mid] + o[i] : Q[mid];
                if (c > target[i]) hi[i] = mid;
                else lo[i] = mid + 1;
            }
        if (!any) break;
    }
#pragma unroll
    for (int i = 0; i < kShots; ++i)
        if (s0 + i < nshots) out[b * nshots + s0 + i] = lo[i];
}

// Per slot: the index bits the outcome fixes (deposit of x_b on locs) and 1/sqrt(P[b][x_b]).
__global__ void k_collapse_prep(const double* __restrict__ probs, uint64_t len, int B, const uint64_t* __restrict__ x,
                                const int* __restrict__ locs, int k, uint64_t* __restrict__ dep,
                                double* __restrict__ scale, double* __restrict__ prob)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const uint64_t xb = x[b];
    const double p = probs[(uint64_t)b * len + xb];
    uint64_t d = 0;
    for (int j = 0; j < k; ++j) d |= ((xb >> j) & 1) << locs[j];
    dep[b] = d;
    prob[b] = p;
    scale[b] = p > 0 ? 1.0 / sqrt(p) : 0.0;
}

template <typename R>
__global__ __launch_bounds__(kMThreads) void k_collapse(vec2_t<R>* __restrict__ psi, uint64_t elems, int B,
                                                        uint64_t mask, const uint64_t* __restrict__ dep,
                                                        const double* __restrict__ scale)
{
    for (uint64_t e = (uint64_t)blockIdx.x * kMThreads + threadIdx.x; e < elems; e += (uint64_t)gridDim.x * kMThreads) {
        const uint64_t i = e / B, b = e - i * B;
        vec2_t<R> a = psi[e];
        if ((i & mask) == dep[b]) {
            const R s = (R)scale[b];
            a.x *= s;
            a.y *= s;
        } else {
            a.x = 0;
            a.y = 0;
        }
        psi[e] = a;
    }
}

// Blocks of a grid-stride elementwise launch over `count` items.
unsigned grid_blocks(uint64_t count)
{
    const uint64_t nb = (count + kMThreads - 1) / kMThreads;
    return (unsigned)(nb < 65536 ? nb : 65536);
}

bool locs_are_low(const int* locs, int k)
{
    for (int j = 0; j < k; ++j)
        if (locs[j] != j) return false;
    return true;
}

}  // namespace

// Probabilities P[b][x] of the outcomes of locs into prob (device, B * 2^k doubles).
int launch_outcome_probs(const yao_state* s, const int* locs, int k, double* prob)
{
    const int n = s->n, B = s->batch;
    const void* data = s->data;
    if (!locs_are_low(locs, k)) {
        std::vector<int> perm(n, -1);
        for (int j = 0; j < k; ++j) perm[locs[j]] = j;
        int next = k;
        for (int q = 0; q < n; ++q)
            if (perm[q] < 0) perm[q] = next++;
        void* tmp = workspace(WS_PERM, s->bytes());
        if (!tmp) return YAO_ENOMEM;
        YAO_TRY(launch_permute(s->data, tmp, s->dtype, n, B, perm.data()));
        data = tmp;
    }
    const uint64_t rows = (uint64_t)B << k;
    const uint64_t nenv = uint64_t(1) << (n - k);
    const int RB = (int)std::min<uint64_t>(rows, kMThreads);
    uint64_t G = 1;
    while (G * 2 * RB <= kMThreads) G *= 2;
    const uint64_t row_blocks = (rows + RB - 1) / RB;
    // About 4096 blocks, each env group of a block summing at least 8 env rows.
    uint64_t nchunks = std::max<uint64_t>(1, std::min<uint64_t>(nenv / (8 * G), 4096 / row_blocks));
    nchunks = std::min<uint64_t>(nchunks, 65535);
    const uint64_t per = (nenv + nchunks - 1) / nchunks;
    nchunks = (nenv + per - 1) / per;
    double* partial = prob;
    if (nchunks > 1) {
        partial = (double*)workspace(WS_PARTIAL, sizeof(double) * rows * nchunks);
        if (!partial) return YAO_ENOMEM;
    }
    const int pi = prof_begin(YAO_KF_MEASURE);
    dim3 grid((unsigned)row_blocks, (unsigned)nchunks);
    if (s->dtype == YAO_C64)
        k_marginal<float><<<grid, kMThreads, 0, stream()>>>((const float2*)data, k, B, RB, nenv, per, partial);
    else
        k_marginal<double><<<grid, kMThreads, 0, stream()>>>((const double2*)data, k, B, RB, nenv, per, partial);
    YAO_HIP(hipGetLastError());
    if (nchunks > 1) {
        k_sum_chunks<<<(unsigned)((rows + kMThreads - 1) / kMThreads), kMThreads, 0, stream()>>>(partial, rows,
                                                                                                  (int)nchunks, prob);
        YAO_HIP(hipGetLastError());
    }
    prof_end(pi, (double)s->bytes() + 8.0 * rows * (1 + (nchunks > 1 ? 2.0 * nchunks : 0.0)), 3.0 * s->elems());
    return 0;
}

// Cumulative sums of each slot's row of len = 2^k doubles, p -> q (q may be p); tot: B * nchunks
// doubles.
int launch_cdf(const double* p, double* q, int k, int B, double* tot)
{
    const uint64_t len = uint64_t(1) << k;
    const int nchunks = (int)((len + kChunk - 1) / kChunk);
    const int pi = prof_begin(YAO_KF_MEASURE);
    k_scan_chunks<<<dim3(nchunks, B), kMThreads, 0, stream()>>>(p, q, len, nchunks, tot);
    YAO_HIP(hipGetLastError());
    if (nchunks > 1) {
        k_scan_totals<<<B, kMThreads, 0, stream()>>>(tot, nchunks, q, len);
        YAO_HIP(hipGetLastError());
    }
    prof_end(pi, 8.0 * B * (double)len * 2.0, (double)B * len);
    return 0;
}

size_t cdf_tot_doubles(int k, int B)
{
    return 2 * (size_t)B * (((uint64_t(1) << k) + kChunk - 1) / kChunk);
}

int launch_sample(const double* cdf, const double* tot, int k, int B, int nshots, const double* u, uint64_t* out)
{
    const uint64_t total = (uint64_t)B * nshots;
    const uint64_t len = uint64_t(1) << k;
    const int nchunks = (int)((len + kChunk - 1) / kChunk);
    const uint64_t threads = (uint64_t)B * ((nshots + kShots - 1) / kShots);
    const int pi = prof_begin(YAO_KF_MEASURE);
    k_sample<<<(unsigned)((threads + kMThreads - 1) / kMThreads), kMThreads, 0, stream()>>>(cdf, tot, len, nchunks, B,
                                                                                            nshots, u, out);
    prof_end(pi, 16.0 * total + 8.0 * k * total, 0.0);
    YAO_HIP(hipGetLastError());
    return 0;
}

int launch_collapse(yao_state* s, const double* probs, const int* locs_dev, const int* locs, int k, const uint64_t* x,
                    uint64_t* dep, double* scale, double* prob)
{
    const int B = s->batch;
    k_collapse_prep<<<(B + 63) / 64, 64, 0, stream()>>>(probs, uint64_t(1) << k, B, x, locs_dev, k, dep, scale, prob);
    YAO_HIP(hipGetLastError());
    uint64_t mask = 0;
    for (int j = 0; j < k; ++j) mask |= uint64_t(1) << locs[j];
    const uint64_t elems = s->elems();
    const int pi = prof_begin(YAO_KF_MEASURE);
    if (s->dtype == YAO_C64)
        k_collapse<float><<<grid_blocks(elems), kMThreads, 0, stream()>>>((float2*)s->data, elems, B, mask, dep,
                                                                           scale);
    else
        k_collapse<double><<<grid_blocks(elems), kMThreads, 0, stream()>>>((double2*)s->data, elems, B, mask, dep,
                                                                            scale);
    prof_end(pi, 2.0 * (double)s->bytes(), 2.0 * (double)elems);
    YAO_HIP(hipGetLastError());
    return 0;
}

}  // namespace yao
