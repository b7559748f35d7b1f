// extern "C" entry points: validation, object lifetime, and the forward / backward drivers
// that choose between the per-gate form and the fused tile passes.
#include <cmath>
#include <cstdio>

#include "driver.h"
#include "fused.h"
#include "tuner.h"
#include "runtime.h"

using namespace yao;

namespace yao {
int noalloc_setup();
const char* last_error();
void set_stream(hipStream_t s);
void set_options(const yao_options& o);
void default_options(yao_options& o);
}  // namespace yao

namespace {

constexpr int kMaxQubits = 34;
constexpr int kMaxK = 5;
constexpr int kMaxCtrl = 8;

int check_qubits(int n, const int* locs, int k, int nctrl, const int* ctrls, const int* cvals)
{
    if (k < 1 || k > kMaxK) return set_error(YAO_EINVAL, "k = %d out of range 1..%d", k, kMaxK);
    if (nctrl < 0 || nctrl > kMaxCtrl) return set_error(YAO_EINVAL, "nctrl = %d out of range 0..%d", nctrl, kMaxCtrl);
    if (!locs) return set_error(YAO_EINVAL, "locs is NULL");
    if (nctrl > 0 && !ctrls) return set_error(YAO_EINVAL, "ctrls is NULL");
    uint64_t used = 0;
    for (int j = 0; j < k; ++j) {
        if (locs[j] < 0 || locs[j] >= n) return set_error(YAO_EINVAL, "loc %d out of range for %d qubits", locs[j], n);
        if ((used >> locs[j]) & 1) return set_error(YAO_EINVAL, "qubit %d repeated", locs[j]);
        used |= uint64_t(1) << locs[j];
    }
    for (int m = 0; m < nctrl; ++m) {
        if (ctrls[m] < 0 || ctrls[m] >= n) return set_error(YAO_EINVAL, "control %d out of range for %d qubits", ctrls[m], n);
        if ((used >> ctrls[m]) & 1) return set_error(YAO_EINVAL, "control %d repeats a qubit", ctrls[m]);
        used |= uint64_t(1) << ctrls[m];
        if (cvals && cvals[m] != 0 && cvals[m] != 1) return set_error(YAO_EINVAL, "control value %d not 0 or 1", cvals[m]);
    }
    return 0;
}

// A rotation exp(-i theta G / 2) = cos(theta/2) I - i sin(theta/2) G needs G Hermitian and
// reflexive (G G = I; Sec. "Forward Mode"), or the formula is not the exponential and not
// unitary. Checked entry-wise to 1e-12.
int check_reflexive(const double* G, int k)
{
    const int d = 1 << k;
    auto re = [&](int r, int c) { return G[2 * ((size_t)r * d + c)]; };
    auto im = [&](int r, int c) { return G[2 * ((size_t)r * d + c) + 1]; };
    constexpr double tol = 1e-12;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            if (std::fabs(re(r, c) - re(c, r)) > tol || std::fabs(im(r, c) + im(c, r)) > tol)
                return set_error(YAO_EINVAL, "rotation generator is not Hermitian at (%d, %d)", r, c);
            double sr = 0, si = 0;
            for (int m = 0; m < d; ++m) {
                sr += re(r, m) * re(m, c) - im(r, m) * im(m, c);
                si += re(r, m) * im(m, c) + im(r, m) * re(m, c);
            }
            if (std::fabs(sr - (r == c ? 1.0 : 0.0)) > tol || std::fabs(si) > tol)
                return set_error(YAO_EINVAL, "rotation generator G does not satisfy G G = I at (%d, %d)", r, c);
        }
    return 0;
}

int check_gate_kind(int g, int k, const double* G)
{
    if (g < YAO_X || g > YAO_DENSE) return set_error(YAO_EINVAL, "unknown gate kind %d", g);
    if (g == YAO_ROT || g == YAO_DENSE) {
        if (!G) return set_error(YAO_EINVAL, "gate kind %d needs a matrix", g);
    } else if (k != 1) {
        return set_error(YAO_EINVAL, "gate kind %d acts on one qubit, got k = %d", g, k);
    }
    if (G && (g == YAO_ROT || g == YAO_DENSE)) {
        const size_t n = size_t(2) << (2 * k);
        for (size_t t = 0; t < n; ++t)
            if (!std::isfinite(G[t])) return set_error(YAO_EINVAL, "matrix entry %zu is not finite", t);
    }
    if (g == YAO_ROT) YAO_TRY(check_reflexive(G, k));
    return 0;
}

GateRec make_rec(int g, int param, double theta, const double* G, const int* locs, int k, int nctrl, const int* ctrls,
                 const int* cvals)
{
    GateRec r;
    r.kind = g;
    r.param = param;
    r.theta = theta;
    r.k = k;
    for (int j = 0; j < k; ++j) r.locs[j] = locs[j];
    r.nctrl = nctrl;
    for (int m = 0; m < nctrl; ++m) {
        r.ctrls[m] = ctrls[m];
        r.cvals[m] = cvals ? cvals[m] : 1;
    }
    if (G && (g == YAO_ROT || g == YAO_DENSE)) r.G.assign(G, G + (size_t(2) << (2 * k)));
    return r;
}

int check_state(const yao_state* s)
{
    if (!s) return set_error(YAO_EINVAL, "state is NULL");
    if (!s->data) return set_error(YAO_EINVAL, "state has no memory");
    return 0;
}

}  // namespace

extern "C" {

int yao_init(void)
{
    YAO_TRY(ensure_device());
    YAO_TRY(noalloc_setup());
    yao_options o;
    default_options(o);
    set_options(o);
    return 0;
}

const char* yao_last_error(void)
{
    return last_error();
}

int yao_set_stream(void* hip_stream)
{
    set_stream((hipStream_t)hip_stream);
    return 0;
}

int yao_synchronize(void)
{
    YAO_HIP(hipStreamSynchronize(stream()));
    return 0;
}

int yao_set_options(const yao_options* opt)
{
    if (!opt) return set_error(YAO_EINVAL, "options is NULL");
    if (opt->fuse_width < 0 || opt->fuse_width > 5) return set_error(YAO_EINVAL, "fuse_width must be 0..5");
    if (opt->tile_qubits < 0 || opt->tile_qubits > 14) return set_error(YAO_EINVAL, "tile_qubits must be 0..14");
    if (opt->checkpoint_every < 0) return set_error(YAO_EINVAL, "checkpoint_every must be >= 0");
    if (!(opt->drift_tol >= 0)) return set_error(YAO_EINVAL, "drift_tol must be >= 0");
    if (opt->jit < 0) return set_error(YAO_EINVAL, "jit must be >= 0");
    set_options(*opt);
    return 0;
}

int yao_get_options(yao_options* opt)
{
    if (!opt) return set_error(YAO_EINVAL, "options is NULL");
    *opt = options();
    return 0;
}

// ------------------------------------------------------------------------------- states
int yao_state_create(int n, int batch, enum yao_dtype dt, yao_state** out)
{
    if (!out) return set_error(YAO_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > kMaxQubits) return set_error(YAO_EINVAL, "n = %d out of range 1..%d", n, kMaxQubits);
    if (batch < 1) return set_error(YAO_EINVAL, "batch = %d must be >= 1", batch);
    if (dt != YAO_C64 && dt != YAO_C128) return set_error(YAO_EINVAL, "unknown dtype %d", (int)dt);
    YAO_TRY(ensure_device());
    yao_state* s = new yao_state{nullptr, n, batch, (int)dt, true};
    hipError_t e = hipMalloc(&s->data, s->bytes());
    if (e != hipSuccess) {
        delete s;
        return set_error(YAO_ENOMEM, "state of %d qubits x %d: %s", n, batch, hipGetErrorString(e));
    }
    int r = launch_reset(s);
    if (r) {
        (void)hipFree(s->data);
        delete s;
        return r;
    }
    *out = s;
    return 0;
}

int yao_state_wrap(void* dev_ptr, int n, int batch, enum yao_dtype dt, yao_state** out)
{
    if (!out) return set_error(YAO_EINVAL, "out is NULL");
    *out = nullptr;
    if (!dev_ptr) return set_error(YAO_EINVAL, "dev_ptr is NULL");
    if (n < 1 || n > kMaxQubits) return set_error(YAO_EINVAL, "n = %d out of range 1..%d", n, kMaxQubits);
    if (batch < 1) return set_error(YAO_EINVAL, "batch = %d must be >= 1", batch);
    if (dt != YAO_C64 && dt != YAO_C128) return set_error(YAO_EINVAL, "unknown dtype %d", (int)dt);
    if (((uintptr_t)dev_ptr) % 16) return set_error(YAO_EINVAL, "dev_ptr must be 16-byte aligned");
    *out = new yao_state{dev_ptr, n, batch, (int)dt, false};
    return 0;
}

int yao_state_destroy(yao_state* s)
{
    if (!s) return 0;
    drop_batch(s);
    if (s->owns && s->data) {
        hipError_t e = hipFree(s->data);
        delete s;
        if (e != hipSuccess) return hip_fail(e, "hipFree");
        return 0;
    }
    delete s;
    return 0;
}

int yao_state_reset(yao_state* s)
{
    YAO_TRY(check_state(s));
    return launch_reset(s);
}

int yao_state_upload(yao_state* s, const void* host, size_t bytes)
{
    YAO_TRY(check_state(s));
    if (!host) return set_error(YAO_EINVAL, "host is NULL");
    if (bytes != s->bytes()) return set_error(YAO_EINVAL, "bytes = %zu, state holds %zu", bytes, s->bytes());
    YAO_HIP(hipMemcpyAsync(s->data, host, bytes, hipMemcpyHostToDevice, stream()));
    YAO_HIP(hipStreamSynchronize(stream()));
    return 0;
}

int yao_state_download(const yao_state* s, void* host, size_t bytes)
{
    YAO_TRY(check_state(s));
    if (!host) return set_error(YAO_EINVAL, "host is NULL");
    if (bytes != s->bytes()) return set_error(YAO_EINVAL, "bytes = %zu, state holds %zu", bytes, s->bytes());
    YAO_HIP(hipMemcpyAsync(host, s->data, bytes, hipMemcpyDeviceToHost, stream()));
    YAO_HIP(hipStreamSynchronize(stream()));
    return 0;
}

int yao_state_info(const yao_state* s, void** dev_ptr, int* n, int* batch, int* dtype)
{
    if (!s) return set_error(YAO_EINVAL, "state is NULL");
    if (dev_ptr) *dev_ptr = s->data;
    if (n) *n = s->n;
    if (batch) *batch = s->batch;
    if (dtype) *dtype = s->dtype;
    return 0;
}

// ------------------------------------------------------------------------------- gates
int yao_apply(yao_state* s, const double* U, int k, const int* locs, int nctrl, const int* ctrls, const int* ctrl_vals)
{
    YAO_TRY(check_state(s));
    if (!U) return set_error(YAO_EINVAL, "U is NULL");
    YAO_TRY(check_qubits(s->n, locs, k, nctrl, ctrls, ctrl_vals));
    YAO_TRY(check_gate_kind(YAO_DENSE, k, U));
    GateRec g = make_rec(YAO_DENSE, -1, 0.0, U, locs, k, nctrl, ctrls, ctrl_vals);
    return apply_one(s, g, 0.0);
}

int yao_apply_gate(yao_state* s, enum yao_gate g, double theta, const double* G, const int* locs, int k, int nctrl,
                   const int* ctrls, const int* ctrl_vals)
{
    YAO_TRY(check_state(s));
    YAO_TRY(check_qubits(s->n, locs, k, nctrl, ctrls, ctrl_vals));
    YAO_TRY(check_gate_kind(g, k, G));
    if (!std::isfinite(theta)) return set_error(YAO_EINVAL, "theta is not finite");
    GateRec r = make_rec(g, -1, theta, G, locs, k, nctrl, ctrls, ctrl_vals);
    return apply_one(s, r, theta);
}

// ------------------------------------------------------------------------------- observables
int yao_pauli_sum_create(int n, int nterms, const double* coef, const uint64_t* xmask, const uint64_t* zmask,
                         yao_pauli_sum** out)
{
    if (!out) return set_error(YAO_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > kMaxQubits) return set_error(YAO_EINVAL, "n = %d out of range 1..%d", n, kMaxQubits);
    if (nterms < 1) return set_error(YAO_EINVAL, "nterms = %d must be >= 1", nterms);
    if (!coef || !xmask || !zmask) return set_error(YAO_EINVAL, "coef/xmask/zmask is NULL");
    const uint64_t allowed = n == 64 ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
    for (int t = 0; t < nterms; ++t) {
        if ((xmask[t] | zmask[t]) & ~allowed) return set_error(YAO_EINVAL, "term %d acts outside %d qubits", t, n);
        if (!std::isfinite(coef[t])) return set_error(YAO_EINVAL, "coef[%d] is not finite", t);
    }
    yao_pauli_sum* h = new yao_pauli_sum;
    h->n = n;
    h->coef.assign(coef, coef + nterms);
    h->x.assign(xmask, xmask + nterms);
    h->z.assign(zmask, zmask + nterms);
    pauli_group_host(h);
    *out = h;
    return 0;
}

int yao_pauli_sum_destroy(yao_pauli_sum* h)
{
    if (!h) return 0;
    drop_batch(h);
    drop_obs_plans(h);
    if (h->d_groups) (void)hipFree(h->d_groups);
    if (h->d_terms) (void)hipFree(h->d_terms);
    delete h;
    return 0;
}

int yao_expect(const yao_state* s, const yao_pauli_sum* h, double* energy)
{
    YAO_TRY(check_state(s));
    if (!h || !energy) return set_error(YAO_EINVAL, "pauli sum or energy is NULL");
    if (h->n != s->n) return set_error(YAO_EINVAL, "observable on %d qubits, state has %d", h->n, s->n);
    return launch_expect(s->data, s->dtype, s->n, s->batch, const_cast<yao_pauli_sum*>(h), energy);
}

int yao_hpsi(const yao_state* s, const yao_pauli_sum* h, yao_state* out, double* energy)
{
    YAO_TRY(check_state(s));
    YAO_TRY(check_state(out));
    if (!h) return set_error(YAO_EINVAL, "pauli sum is NULL");
    if (h->n != s->n) return set_error(YAO_EINVAL, "observable on %d qubits, state has %d", h->n, s->n);
    if (out->n != s->n || out->batch != s->batch || out->dtype != s->dtype)
        return set_error(YAO_EINVAL, "out must match the state in n, batch and dtype");
    if (out->data == s->data) return set_error(YAO_EINVAL, "out must not alias the state");
    return launch_hpsi(s->data, s->dtype, out->data, out->dtype, s->n, s->batch, const_cast<yao_pauli_sum*>(h), energy);
}

int yao_inner(const yao_state* a, const yao_state* b, double* re, double* im)
{
    YAO_TRY(check_state(a));
    YAO_TRY(check_state(b));
    if (!re || !im) return set_error(YAO_EINVAL, "re or im is NULL");
    if (a->n != b->n || a->batch != b->batch) return set_error(YAO_EINVAL, "states differ in n or batch");
    return launch_inner(a->data, a->dtype, b->data, b->dtype, a->n, a->batch, re, im);
}

// ------------------------------------------------------------------------------- circuits
int yao_circuit_create(int n, yao_circuit** out)
{
    if (!out) return set_error(YAO_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > kMaxQubits) return set_error(YAO_EINVAL, "n = %d out of range 1..%d", n, kMaxQubits);
    yao_circuit* c = new yao_circuit;
    c->n = n;
    c->nparams = 0;
    c->version = 0;
    *out = c;
    return 0;
}

int yao_circuit_destroy(yao_circuit* c)
{
    if (!c) return 0;
    drop_batch(c);
    drop_tuning(c);
    drop_plans(c);
    drop_fused(c);
    delete c;
    return 0;
}

int yao_circuit_push(yao_circuit* c, enum yao_gate g, int param_index, double theta_fixed, const double* G,
                     const int* locs, int k, int nctrl, const int* ctrls, const int* ctrl_vals)
{
    if (!c) return set_error(YAO_EINVAL, "circuit is NULL");
    YAO_TRY(check_qubits(c->n, locs, k, nctrl, ctrls, ctrl_vals));
    YAO_TRY(check_gate_kind(g, k, G));
    if (param_index < -1) return set_error(YAO_EINVAL, "param_index = %d must be >= -1", param_index);
    if (param_index >= 0 && !is_param_kind(g)) return set_error(YAO_EINVAL, "gate kind %d takes no parameter", (int)g);
    if (param_index < 0 && !std::isfinite(theta_fixed)) return set_error(YAO_EINVAL, "theta_fixed is not finite");
    c->gates.push_back(make_rec(g, param_index, theta_fixed, G, locs, k, nctrl, ctrls, ctrl_vals));
    if (param_index + 1 > c->nparams) c->nparams = param_index + 1;
    c->version++;
    return 0;
}

int yao_circuit_nparams(const yao_circuit* c, int* out)
{
    if (!c || !out) return set_error(YAO_EINVAL, "circuit or out is NULL");
    *out = c->nparams;
    return 0;
}

// ------------------------------------------------------------------------------- forward / backward
int yao_forward(yao_state* s, const yao_circuit* c, const double* params)
{
    YAO_TRY(check_state(s));
    if (!c) return set_error(YAO_EINVAL, "circuit is NULL");
    if (c->n != s->n) return set_error(YAO_EINVAL, "circuit on %d qubits, state has %d", c->n, s->n);
    if (c->nparams > 0 && !params) return set_error(YAO_EINVAL, "params is NULL");
    for (int p = 0; p < c->nparams; ++p)
        if (!std::isfinite(params[p])) return set_error(YAO_EINVAL, "params[%d] is not finite", p);
    return forward(s, c, params);
}

int yao_backward(yao_state* s, const yao_circuit* c, const double* params, const yao_pauli_sum* h,
                 enum yao_grad_mode mode, int reduce_batch, double* energy, double* grad, double* drift)
{
    YAO_TRY(check_state(s));
    if (!c || !h) return set_error(YAO_EINVAL, "circuit or observable is NULL");
    if (c->n != s->n || h->n != s->n) return set_error(YAO_EINVAL, "qubit counts of state, circuit, observable differ");
    if (c->nparams > 0 && (!params || !grad)) return set_error(YAO_EINVAL, "params or grad is NULL");
    if (!energy) return set_error(YAO_EINVAL, "energy is NULL");
    if (mode != YAO_GRAD_REVERSIBLE && mode != YAO_GRAD_CHECKPOINT && mode != YAO_GRAD_AUTO)
        return set_error(YAO_EINVAL, "unknown gradient mode %d", (int)mode);
    for (int p = 0; p < c->nparams; ++p)
        if (!std::isfinite(params[p])) return set_error(YAO_EINVAL, "params[%d] is not finite", p);
    return backward(s, c, params, const_cast<yao_pauli_sum*>(h), (int)mode, reduce_batch != 0, energy, grad, drift);
}

int yao_auto_fallbacks(long* count)
{
    if (!count) return set_error(YAO_EINVAL, "count is NULL");
    *count = auto_fallbacks();
    return 0;
}

int yao_batch_run(int ncirc, yao_state* const* states, const yao_circuit* const* circs, const double* const* params,
                  const yao_pauli_sum* const* h, double* energy, double* const* grad)
{
    if (ncirc < 1) return set_error(YAO_EINVAL, "ncirc = %d must be >= 1", ncirc);
    if (!states || !circs || !params || !h || !energy || !grad) return set_error(YAO_EINVAL, "NULL array");
    for (int c = 0; c < ncirc; ++c) {
        YAO_TRY(check_state(states[c]));
        if (!circs[c] || !h[c]) return set_error(YAO_EINVAL, "circuit or observable %d is NULL", c);
        if (states[c]->batch != 1) return set_error(YAO_EINVAL, "state %d has batch %d, needs 1", c, states[c]->batch);
        if (circs[c]->n != states[c]->n || h[c]->n != states[c]->n)
            return set_error(YAO_EINVAL, "qubit counts of circuit %d differ", c);
        if (states[c]->dtype != states[0]->dtype) return set_error(YAO_EINVAL, "all states need one dtype");
        if (circs[c]->nparams > 0 && (!params[c] || !grad[c])) return set_error(YAO_EINVAL, "params/grad %d is NULL", c);
        for (int p = 0; p < circs[c]->nparams; ++p)
            if (!std::isfinite(params[c][p])) return set_error(YAO_EINVAL, "params[%d][%d] is not finite", c, p);
    }
    return batch_run(ncirc, states, circs, params, const_cast<yao_pauli_sum* const*>(h), energy, grad);
}

int yao_profile_enable(int on)
{
    return prof_enable(on != 0);
}

int yao_profile_read(int family, int* launches, double* total_ms, double* algo_bytes, double* algo_flops)
{
    if (family < 0 || family >= YAO_KF_COUNT) return set_error(YAO_EINVAL, "unknown kernel family %d", family);
    return prof_read(family, launches, total_ms, algo_bytes, algo_flops);
}

int yao_jit_stats(long long* out)
{
    if (!out) return set_error(YAO_EINVAL, "out is NULL");
    yao::jit_stats(out);
    return 0;
}

int yao_jit_selfcheck(const yao_circuit* c, enum yao_dtype dt, int reverse, int tile_qubits, int* npasses,
                      int* njit)
{
    if (!c || !npasses || !njit) return set_error(YAO_EINVAL, "NULL argument");
    if (dt != YAO_C64 && dt != YAO_C128) return set_error(YAO_EINVAL, "unknown dtype %d", (int)dt);
    if (tile_qubits < 0 || tile_qubits > 14) return set_error(YAO_EINVAL, "tile_qubits must be 0..14");
    if (c->n > kMaxQubits) return set_error(YAO_EINVAL, "too many qubits");
    return yao::jit_selfcheck(c, dt, reverse, tile_qubits, npasses, njit);
}

int yao_plan_selfcheck(const yao_circuit* c, const double* params, enum yao_dtype dt, int reverse, int tile_qubits,
                       double* max_err, int* npasses)
{
    if (!c || !max_err || !npasses) return set_error(YAO_EINVAL, "null argument");
    if (dt != YAO_C64 && dt != YAO_C128) return set_error(YAO_EINVAL, "unknown dtype %d", (int)dt);
    if (tile_qubits < 0 || tile_qubits > 14) return set_error(YAO_EINVAL, "tile_qubits must be 0..14");
    if (c->nparams > 0 && !params) return set_error(YAO_EINVAL, "circuit takes %d parameters", c->nparams);
    return yao::plan_selfcheck(c, params, dt, reverse, tile_qubits, max_err, npasses);
}

}  // extern "C"
