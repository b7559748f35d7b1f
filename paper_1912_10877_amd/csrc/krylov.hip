// Time evolution psi <- exp(-i H t) psi under a Pauli sum by the Krylov (Lanczos) method: the
// Hamiltonian is applied to the register over and over, as Sec. "Matrix Representation" says of
// time_evolve, and the small projected problem is exponentiated on the host.
//
// Per slot b and substep tau: v_0 = psi / |psi|; for j = 0..m-1: w = H v_j and
// alpha_j = Re <v_j|H v_j> from the same pass (the H psi tile passes), w -= alpha_j v_j +
// beta_j v_{j-1}, beta_{j+1} = |w|, v_{j+1} = w / beta_{j+1}. With T the tridiagonal matrix of the
// alphas and betas, psi(tau) ~ |psi| V exp(-i tau T) e_1, whose error is estimated by
// |psi| beta_m |(exp(-i tau T) e_1)_{m-1}|; tau is halved until that estimate is below the
// tolerance (the Krylov space does not depend on tau), and substeps repeat until t is covered.
// Every vector operation stays on the device with per-slot coefficients in device memory; the
// host waits once per substep, for the alphas and betas.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "runtime.h"

namespace yao {

namespace {

constexpr int kKThreads = 256;

struct SlotGeom {
    int logBc, nchunks;
};

SlotGeom slot_geom(int B)
{
    int lb = 0;
    while ((1 << lb) < B) ++lb;
    SlotGeom g;
    g.logBc = lb < 6 ? lb : 6;
    g.nchunks = (B + (1 << g.logBc) - 1) >> g.logBc;
    return g;
}

int grid_x(uint64_t rows, int logBc)
{
    const uint64_t rpb = kKThreads >> logBc;
    const uint64_t nb = (rows + rpb - 1) / rpb;
    return (int)(nb < 1024 ? nb : 1024);
}

__device__ __forceinline__ double block_sum_slot(double v, int logBc, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kKThreads / 2; s >= (1 << logBc); s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[threadIdx.x];
}

// partial[b][blk] = sum over this block's rows of |x|^2.
template <typename R>
__global__ __launch_bounds__(kKThreads) void k_norm2(const vec2_t<R>* __restrict__ x, uint64_t rows, int B, int logBc,
                                                     double* __restrict__ partial)
{
    __shared__ double red[kKThreads];
    const int b = blockIdx.y * (1 << logBc) + (threadIdx.x & ((1 << logBc) - 1));
    const int rpb = kKThreads >> logBc;
    double acc = 0;
    if (b < B)
        for (uint64_t i = (uint64_t)blockIdx.x * rpb + (threadIdx.x >> logBc); i < rows; i += (uint64_t)gridDim.x * rpb) {
            const vec2_t<R> a = x[i * B + b];
            acc += (double)a.x * a.x + (double)a.y * a.y;
        }
    const double s = block_sum_slot(acc, logBc, red);
    if ((int)threadIdx.x < (1 << logBc) && b < B) partial[(uint64_t)b * gridDim.x + blockIdx.x] = s;
}

// w <- w - alpha[b] v - beta[b] vp (vp null for the first step), with partial norms of the new w.
template <typename R>
__global__ __launch_bounds__(kKThreads) void k_lanczos_orth(vec2_t<R>* __restrict__ w, const vec2_t<R>* __restrict__ v,
                                                            const vec2_t<R>* __restrict__ vp,
                                                            const double* __restrict__ alpha,
                                                            const double* __restrict__ beta, uint64_t rows, int B,
                                                            int logBc, double* __restrict__ partial)
{
    __shared__ double red[kKThreads];
    const int b = blockIdx.y * (1 << logBc) + (threadIdx.x & ((1 << logBc) - 1));
    const int rpb = kKThreads >> logBc;
    double acc = 0;
    if (b < B) {
        const R a = (R)alpha[b];
        const R bt = vp ? (R)beta[b] : R(0);
        for (uint64_t i = (uint64_t)blockIdx.x * rpb + (threadIdx.x >> logBc); i < rows; i += (uint64_t)gridDim.x * rpb) {
            const uint64_t e = i * B + b;
            vec2_t<R> x = w[e];
            const vec2_t<R> y = v[e];
            x.x -= a * y.x;
            x.y -= a * y.y;
            if (vp) {
                const vec2_t<R> z = vp[e];
                x.x -= bt * z.x;
                x.y -= bt * z.y;
            }
            w[e] = x;
            acc += (double)x.x * x.x + (double)x.y * x.y;
        }
    }
    const double s = block_sum_slot(acc, logBc, red);
    if ((int)threadIdx.x < (1 << logBc) && b < B) partial[(uint64_t)b * gridDim.x + blockIdx.x] = s;
}

// out = in / sqrt(sumsq[b]) (0 where the norm vanishes: the Krylov space closed), beta[b] = the norm.
template <typename R>
__global__ __launch_bounds__(kKThreads) void k_normalize(vec2_t<R>* __restrict__ out, const vec2_t<R>* __restrict__ in,
                                                         const double* __restrict__ sumsq, double* __restrict__ beta,
                                                         uint64_t elems, int B)
{
    for (uint64_t e = (uint64_t)blockIdx.x * kKThreads + threadIdx.x; e < elems; e += (uint64_t)gridDim.x * kKThreads) {
        const int b = (int)(e % (uint64_t)B);
        const double nrm = sqrt(sumsq[b]);
        const R inv = nrm > 1e-300 ? (R)(1.0 / nrm) : R(0);
        vec2_t<R> x = in[e];
        x.x *= inv;
        x.y *= inv;
        out[e] = x;
        if (e < (uint64_t)B) beta[b] = nrm;
    }
}

// psi = sum_j y[j][b] V_j for the m Krylov vectors (stride elements apart).
template <typename R>
__global__ __launch_bounds__(kKThreads) void k_combine(vec2_t<R>* __restrict__ psi, const vec2_t<R>* __restrict__ V,
                                                       uint64_t stride, int m, const double2* __restrict__ y,
                                                       uint64_t elems, int B)
{
    for (uint64_t e = (uint64_t)blockIdx.x * kKThreads + threadIdx.x; e < elems; e += (uint64_t)gridDim.x * kKThreads) {
        const int b = (int)(e % (uint64_t)B);
        double re = 0, im = 0;
        for (int j = 0; j < m; ++j) {
            const vec2_t<R> v = V[(uint64_t)j * stride + e];
            const double2 c = y[(uint64_t)j * B + b];
            re += c.x * v.x - c.y * v.y;
            im += c.x * v.y + c.y * v.x;
        }
        vec2_t<R> o;
        o.x = (R)re;
        o.y = (R)im;
        psi[e] = o;
    }
}

using cplx = std::complex<double>;

// exp(A) for a small complex matrix (row-major, d x d) by scaling and squaring of a Taylor series.
std::vector<cplx> small_expm(const std::vector<cplx>& A, int d)
{
    double nrm = 0;
    for (int c = 0; c < d; ++c) {
        double col = 0;
        for (int r = 0; r < d; ++r) col += std::abs(A[(size_t)r * d + c]);
        nrm = std::max(nrm, col);
    }
    int s = 0;
    while (nrm > 0.5) {
        nrm /= 2;
        ++s;
    }
    const double sc = std::ldexp(1.0, -s);
    std::vector<cplx> X(A.size()), E((size_t)d * d, 0.0), term((size_t)d * d, 0.0), tmp((size_t)d * d);
    for (size_t i = 0; i < A.size(); ++i) X[i] = A[i] * sc;
    for (int i = 0; i < d; ++i) E[(size_t)i * d + i] = term[(size_t)i * d + i] = 1.0;
    auto mul = [&](const std::vector<cplx>& P, const std::vector<cplx>& Q, std::vector<cplx>& R) {
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) {
                cplx acc = 0;
                for (int t = 0; t < d; ++t) acc += P[(size_t)r * d + t] * Q[(size_t)t * d + c];
                R[(size_t)r * d + c] = acc;
            }
    };
    for (int j = 1; j <= 24; ++j) {  // |X| <= 1/2: the remainder after 24 terms is < 1e-31
        mul(term, X, tmp);
        for (size_t i = 0; i < tmp.size(); ++i) term[i] = tmp[i] / (double)j;
        for (size_t i = 0; i < E.size(); ++i) E[i] += term[i];
    }
    for (int q = 0; q < s; ++q) {
        mul(E, E, tmp);
        E.swap(tmp);
    }
    return E;
}

template <typename R>
int lanczos_substep(void* psi, int n, int B, int dtype, const yao_pauli_sum* h, double t_left, double tol, int mmax,
                    double* tau_done)
{
    using V = vec2_t<R>;
    const uint64_t rows = uint64_t(1) << n;
    const uint64_t elems = rows * B;
    const size_t es = sizeof(V);
    SlotGeom sg = slot_geom(B);
    const int nbx = grid_x(rows, sg.logBc);
    const size_t hp = hpsi_partial_doubles(h, n, B, dtype);
    // Vectors V_0..V_mmax, the work vector w; coefficient arrays on the device.
    char* ws = (char*)workspace(WS_KRYLOV, es * elems * (size_t)(mmax + 2));
    double* dv = (double*)workspace(WS_MISC, sizeof(double) * (hp + (size_t)B * nbx + (size_t)B * (2 * mmax + 4) +
                                                               2 * (size_t)B * (mmax + 1) + 64));
    if (!ws || !dv) return YAO_ENOMEM;
    V* Vk = (V*)ws;
    V* w = (V*)(ws + es * elems * (size_t)(mmax + 1));
    double* hpart = dv;
    double* part = hpart + hp;
    double* alpha = part + (size_t)B * nbx;         // [mmax][B]
    double* beta = alpha + (size_t)B * mmax;        // [mmax + 1][B]; beta[0] = |psi|
    double* sums = beta + (size_t)B * (mmax + 1);   // [B]
    double2* ydev = (double2*)(sums + (size_t)B + 8);
    hipStream_t st = stream();
    dim3 grid(nbx, sg.nchunks);
    const unsigned eb = (unsigned)std::min<uint64_t>((elems + kKThreads - 1) / kKThreads, 65536);
    const int pi = prof_begin(YAO_KF_KRYLOV);
    k_norm2<R><<<grid, kKThreads, 0, st>>>((const V*)psi, rows, B, sg.logBc, part);
    YAO_TRY(launch_row_sums(part, B, nbx, sums));
    k_normalize<R><<<eb, kKThreads, 0, st>>>(Vk, (const V*)psi, sums, beta, elems, B);
    YAO_HIP(hipGetLastError());
    for (int j = 0; j < mmax; ++j) {
        V* vj = Vk + (size_t)j * elems;
        YAO_TRY(launch_hpsi_dev(vj, dtype, w, dtype, n, B, h, hpart, alpha + (size_t)j * B));
        k_lanczos_orth<R><<<grid, kKThreads, 0, st>>>(w, vj, j > 0 ? vj - elems : nullptr, alpha + (size_t)j * B,
                                                      beta + (size_t)j * B, rows, B, sg.logBc, part);
        YAO_TRY(launch_row_sums(part, B, nbx, sums));
        k_normalize<R><<<eb, kKThreads, 0, st>>>(vj + elems, w, sums, beta + (size_t)(j + 1) * B, elems, B);
        YAO_HIP(hipGetLastError());
    }
    prof_end(pi, (double)elems * es * (2.0 + 6.0 * mmax), (double)elems * mmax * 12.0);
    std::vector<double> ab((size_t)B * (2 * mmax + 1));
    YAO_HIP(hipMemcpyAsync(ab.data(), alpha, sizeof(double) * ab.size(), hipMemcpyDeviceToHost, st));
    YAO_HIP(hipStreamSynchronize(st));
    const double* ha = ab.data();
    const double* hb = ab.data() + (size_t)B * mmax;
    // Largest tau <= t_left (halving) whose error estimate is below tol in every slot.
    double tau = t_left;
    std::vector<cplx> y((size_t)mmax * B);
    for (int attempt = 0;; ++attempt) {
        double worst = 0;
        for (int b = 0; b < B; ++b) {
            std::vector<cplx> A((size_t)mmax * mmax, 0.0);
            for (int j = 0; j < mmax; ++j) {
                A[(size_t)j * mmax + j] = cplx(0, -tau * ha[(size_t)j * B + b]);
                if (j + 1 < mmax) {
                    const double off = hb[(size_t)(j + 1) * B + b];
                    A[(size_t)j * mmax + j + 1] = A[(size_t)(j + 1) * mmax + j] = cplx(0, -tau * off);
                }
            }
            const std::vector<cplx> E = small_expm(A, mmax);
            const double nrm = hb[b];
            for (int j = 0; j < mmax; ++j) y[(size_t)j * B + b] = nrm * E[(size_t)j * mmax];
            const double err = nrm * hb[(size_t)mmax * B + b] * std::abs(E[(size_t)(mmax - 1) * mmax]);
            worst = std::max(worst, err);
        }
        if (worst <= tol * std::max(1.0, tau)) break;
        if (attempt >= 60) return set_error(YAO_EINVAL, "time evolution: no step size reaches tolerance %.3g", tol);
        tau *= 0.5;
    }
    std::vector<double> yh((size_t)2 * mmax * B);
    for (size_t i = 0; i < y.size(); ++i) {
        yh[2 * i] = y[i].real();
        yh[2 * i + 1] = y[i].imag();
    }
    YAO_HIP(hipMemcpyAsync(ydev, yh.data(), sizeof(double) * yh.size(), hipMemcpyHostToDevice, st));
    const int pc = prof_begin(YAO_KF_KRYLOV);
    k_combine<R><<<eb, kKThreads, 0, st>>>((V*)psi, Vk, elems, mmax, ydev, elems, B);
    prof_end(pc, (double)elems * es * (mmax + 1), (double)elems * mmax * 8.0);
    YAO_HIP(hipGetLastError());
    YAO_HIP(hipStreamSynchronize(st));  // yh is pageable host memory
    *tau_done = tau;
    return 0;
}

}  // namespace

int time_evolve(yao_state* s, yao_pauli_sum* h, double t, double tol, int krylov_dim, int* nsteps)
{
    if (tol <= 0) tol = s->dtype == YAO_C64 ? 1e-6 : 1e-12;
    const int mmax = krylov_dim > 0 ? krylov_dim : 30;
    YAO_TRY(pauli_upload(h));
    double left = t;
    int steps = 0;
    while (std::fabs(left) > 0) {
        double done = 0;
        if (s->dtype == YAO_C64) YAO_TRY(lanczos_substep<float>(s->data, s->n, s->batch, s->dtype, h, left, tol, mmax, &done));
        else YAO_TRY(lanczos_substep<double>(s->data, s->n, s->batch, s->dtype, h, left, tol, mmax, &done));
        ++steps;
        // The last substep lands exactly on t.
        left = (done == left) ? 0.0 : left - done;
    }
    if (nsteps) *nsteps = steps;
    return 0;
}

}  // namespace yao
