// extern "C" entry points of the rows beyond the gradient path: qubit permutations (focus! /
// relax!) and the QFT. Validation on the host, then the kernels of kernels_qubits.hip.
#include <cmath>
#include <vector>

#include "runtime.h"

using namespace yao;

namespace {

int check_state(const yao_state* s)
{
    if (!s) return set_error(YAO_EINVAL, "state is NULL");
    if (!s->data) return set_error(YAO_EINVAL, "state has no memory");
    return 0;
}

// Tile kernels keep one row of B slots contiguous in LDS.
int check_tile_batch(const yao_state* s)
{
    if ((size_t)s->batch * s->elem_bytes() > 16384)
        return set_error(YAO_EINVAL, "batch %d too large for the tile kernels (batch * element bytes <= 16 KiB)",
                         s->batch);
    return 0;
}

int check_locs(int n, const int* locs, int k)
{
    if (!locs) return set_error(YAO_EINVAL, "locs is NULL");
    if (k < 1 || k > n) return set_error(YAO_EINVAL, "k = %d out of range 1..%d", k, n);
    uint64_t used = 0;
    for (int j = 0; j < k; ++j) {
        if (locs[j] < 0 || locs[j] >= n) return set_error(YAO_EINVAL, "loc %d out of range for %d qubits", locs[j], n);
        if ((used >> locs[j]) & 1) return set_error(YAO_EINVAL, "qubit %d repeated", locs[j]);
        used |= uint64_t(1) << locs[j];
    }
    return 0;
}

// Permute s in place: into the workspace, then back.
int permute_in_place(yao_state* s, const int* perm)
{
    bool identity = true;
    for (int q = 0; q < s->n; ++q) identity &= perm[q] == q;
    if (identity) return 0;
    void* tmp = workspace(WS_PERM, s->bytes());
    if (!tmp) return YAO_ENOMEM;
    YAO_TRY(launch_permute(s->data, tmp, s->dtype, s->n, s->batch, perm));
    YAO_HIP(hipMemcpyAsync(s->data, tmp, s->bytes(), hipMemcpyDeviceToDevice, stream()));
    return 0;
}

// focus!(locs): locs[j] -> j, the others after them in ascending order.
std::vector<int> focus_perm(int n, const int* locs, int k)
{
    std::vector<int> perm(n, -1);
    for (int j = 0; j < k; ++j) perm[locs[j]] = j;
    int next = k;
    for (int q = 0; q < n; ++q)
        if (perm[q] < 0) perm[q] = next++;
    return perm;
}

constexpr int kMaxOutcomeBits = 30;

int check_measure(const yao_state* s, const int* locs, int k)
{
    YAO_TRY(check_state(s));
    YAO_TRY(check_locs(s->n, locs, k));
    YAO_TRY(check_tile_batch(s));
    if (k > kMaxOutcomeBits) return set_error(YAO_EINVAL, "k = %d outcome bits exceed %d", k, kMaxOutcomeBits);
    return ensure_device();
}

// Probabilities, cumulative sums and nshots samples per slot, all on the device; with collapse
// (nshots = 1) the state is projected onto the sampled outcome. Results copied to the host.
int measure_impl(yao_state* s, const int* locs, int k, int nshots, const double* u, uint64_t* out, bool collapse,
                 double* prob_out)
{
    const int B = s->batch;
    const size_t len = size_t(1) << k;
    const size_t nt = cdf_tot_doubles(k, B);
    const size_t shots = (size_t)B * nshots;
    const size_t words = 2 * (size_t)B * len + nt + 2 * shots + 3 * (size_t)B + 64;
    double* P = (double*)workspace(WS_MEAS, sizeof(double) * words);
    if (!P) return YAO_ENOMEM;
    double* C = P + (size_t)B * len;
    double* tot = C + (size_t)B * len;
    double* du = tot + nt;
    uint64_t* dout = (uint64_t*)(du + shots);
    uint64_t* dep = dout + shots;
    double* scale = (double*)(dep + B);
    double* dprob = scale + B;
    int* dlocs = (int*)(dprob + B);
    hipStream_t st = stream();
    YAO_TRY(launch_outcome_probs(s, locs, k, P));
    YAO_TRY(launch_cdf(P, C, k, B, tot));
    YAO_HIP(hipMemcpyAsync(du, u, sizeof(double) * shots, hipMemcpyHostToDevice, st));
    YAO_TRY(launch_sample(C, tot, k, B, nshots, du, dout));
    if (collapse) {
        YAO_HIP(hipMemcpyAsync(dlocs, locs, sizeof(int) * k, hipMemcpyHostToDevice, st));
        YAO_TRY(launch_collapse(s, P, dlocs, locs, k, dout, dep, scale, dprob));
    }
    char* hs = (char*)host_staging(sizeof(uint64_t) * shots + sizeof(double) * B);
    if (!hs) return YAO_ENOMEM;
    YAO_HIP(hipMemcpyAsync(hs, dout, sizeof(uint64_t) * shots, hipMemcpyDeviceToHost, st));
    if (collapse) YAO_HIP(hipMemcpyAsync(hs + sizeof(uint64_t) * shots, dprob, sizeof(double) * B,
                                         hipMemcpyDeviceToHost, st));
    YAO_HIP(hipStreamSynchronize(st));
    memcpy(out, hs, sizeof(uint64_t) * shots);
    if (collapse && prob_out) memcpy(prob_out, hs + sizeof(uint64_t) * shots, sizeof(double) * B);
    return 0;
}

int check_uniforms(const double* u, size_t count)
{
    if (!u) return set_error(YAO_EINVAL, "u is NULL");
    for (size_t i = 0; i < count; ++i)
        if (!(u[i] >= 0.0 && u[i] < 1.0)) return set_error(YAO_EINVAL, "u[%zu] = %g is not in [0, 1)", i, u[i]);
    return 0;
}

}  // namespace

extern "C" {

int yao_shift_grad(const yao_state* s, const yao_circuit* c, const double* params, const yao_pauli_sum* h,
                   double* energy, double* grad)
{
    YAO_TRY(check_state(s));
    if (!c || !h) return set_error(YAO_EINVAL, "circuit or observable is NULL");
    if (c->n != s->n || h->n != s->n) return set_error(YAO_EINVAL, "qubit counts of state, circuit, observable differ");
    if (s->batch != 1) return set_error(YAO_EINVAL, "the shift-rule gradient takes a batch-1 state, got %d", s->batch);
    if (c->nparams > 0 && (!params || !grad)) return set_error(YAO_EINVAL, "params or grad is NULL");
    if (!energy) return set_error(YAO_EINVAL, "energy is NULL");
    for (int p = 0; p < c->nparams; ++p)
        if (!std::isfinite(params[p])) return set_error(YAO_EINVAL, "params[%d] is not finite", p);
    YAO_TRY(ensure_device());
    return shift_grad(s, c, params, const_cast<yao_pauli_sum*>(h), energy, grad);
}

int yao_time_evolve(yao_state* s, const yao_pauli_sum* h, double t, double tol, int krylov_dim, int* nsteps)
{
    YAO_TRY(check_state(s));
    if (!h) return set_error(YAO_EINVAL, "pauli sum is NULL");
    if (h->n != s->n) return set_error(YAO_EINVAL, "observable on %d qubits, state has %d", h->n, s->n);
    if (!std::isfinite(t)) return set_error(YAO_EINVAL, "t is not finite");
    if (!(tol >= 0) || !std::isfinite(tol)) return set_error(YAO_EINVAL, "tol must be >= 0");
    if (krylov_dim < 0 || krylov_dim > 64) return set_error(YAO_EINVAL, "krylov_dim must be 0..64");
    if (krylov_dim > 0 && krylov_dim < 2) return set_error(YAO_EINVAL, "krylov_dim must be >= 2");
    YAO_TRY(ensure_device());
    if (nsteps) *nsteps = 0;
    if (t == 0) return 0;
    return time_evolve(s, const_cast<yao_pauli_sum*>(h), t, tol, krylov_dim, nsteps);
}

int yao_probs(const yao_state* s, const int* locs, int k, double* probs)
{
    YAO_TRY(check_measure(s, locs, k));
    if (!probs) return set_error(YAO_EINVAL, "probs is NULL");
    const size_t count = ((size_t)s->batch) << k;
    double* P = (double*)workspace(WS_MEAS, sizeof(double) * count);
    if (!P) return YAO_ENOMEM;
    YAO_TRY(launch_outcome_probs(s, locs, k, P));
    YAO_HIP(hipMemcpyAsync(probs, P, sizeof(double) * count, hipMemcpyDeviceToHost, stream()));
    YAO_HIP(hipStreamSynchronize(stream()));
    return 0;
}

int yao_measure(const yao_state* s, const int* locs, int k, int nshots, const double* u, uint64_t* out)
{
    YAO_TRY(check_measure(s, locs, k));
    if (nshots < 1) return set_error(YAO_EINVAL, "nshots = %d must be >= 1", nshots);
    if (!out) return set_error(YAO_EINVAL, "out is NULL");
    YAO_TRY(check_uniforms(u, (size_t)s->batch * nshots));
    return measure_impl(const_cast<yao_state*>(s), locs, k, nshots, u, out, false, nullptr);
}

int yao_measure_collapse(yao_state* s, const int* locs, int k, const double* u, uint64_t* out, double* prob)
{
    YAO_TRY(check_measure(s, locs, k));
    if (!out) return set_error(YAO_EINVAL, "out is NULL");
    YAO_TRY(check_uniforms(u, (size_t)s->batch));
    return measure_impl(s, locs, k, 1, u, out, true, prob);
}


int yao_permute_qubits(const yao_state* src, yao_state* dst, const int* perm)
{
    YAO_TRY(check_state(src));
    YAO_TRY(check_state(dst));
    if (!perm) return set_error(YAO_EINVAL, "perm is NULL");
    if (src->n != dst->n || src->batch != dst->batch || src->dtype != dst->dtype)
        return set_error(YAO_EINVAL, "src and dst differ in n, batch or dtype");
    YAO_TRY(check_tile_batch(src));
    uint64_t seen = 0;
    for (int q = 0; q < src->n; ++q) {
        if (perm[q] < 0 || perm[q] >= src->n || ((seen >> perm[q]) & 1))
            return set_error(YAO_EINVAL, "perm is not a permutation of 0..%d", src->n - 1);
        seen |= uint64_t(1) << perm[q];
    }
    YAO_TRY(ensure_device());
    if (src->data == dst->data) return permute_in_place(dst, perm);
    return launch_permute(src->data, dst->data, src->dtype, src->n, src->batch, perm);
}

int yao_focus(yao_state* s, const int* locs, int k)
{
    YAO_TRY(check_state(s));
    YAO_TRY(check_locs(s->n, locs, k));
    YAO_TRY(check_tile_batch(s));
    YAO_TRY(ensure_device());
    const std::vector<int> perm = focus_perm(s->n, locs, k);
    return permute_in_place(s, perm.data());
}

int yao_relax(yao_state* s, const int* locs, int k)
{
    YAO_TRY(check_state(s));
    YAO_TRY(check_locs(s->n, locs, k));
    YAO_TRY(check_tile_batch(s));
    YAO_TRY(ensure_device());
    const std::vector<int> fp = focus_perm(s->n, locs, k);
    std::vector<int> inv(s->n);
    for (int q = 0; q < s->n; ++q) inv[fp[q]] = q;
    return permute_in_place(s, inv.data());
}

int yao_qft(yao_state* s, const int* locs, int k, int inverse)
{
    YAO_TRY(check_state(s));
    YAO_TRY(check_locs(s->n, locs, k));
    YAO_TRY(check_tile_batch(s));
    YAO_TRY(ensure_device());
    return launch_qft(s->data, s->dtype, s->n, s->batch, locs, k, inverse != 0);
}

}  // extern "C"
