// Per-gate ("plain") form: one kernel launch per gate for the forward sweep, one fused
// gradient + uncompute launch per gate for the reverse sweep (Sec. "Reverse Mode").
#include <cmath>

#include "driver.h"

namespace yao {

int launch_fill(double* p, size_t count, double v);

int apply_one(yao_state* s, const GateRec& g, double theta)
{
    HostMat U;
    if (!gate_matrix(g, theta, U)) return set_error(YAO_EINVAL, "unknown gate kind %d", g.kind);
    return launch_gate(s->data, s->dtype, s->n, s->batch, U, g.locs, make_ctrl(g.nctrl, g.ctrls, g.cvals));
}

int forward_plain(void* data, int dtype, int n, int B, const yao_circuit* c, const double* params)
{
    // Matrices of k >= 2 gates go to the device in one copy, rounded to the state's precision.
    std::vector<HostMat> mats(c->gates.size());
    std::vector<size_t> off(c->gates.size(), 0);
    std::vector<char> blob;
    const size_t rs = dtype == YAO_C64 ? 4 : 8;
    for (size_t t = 0; t < c->gates.size(); ++t) {
        const GateRec& g = c->gates[t];
        if (!gate_matrix(g, gate_theta(g, params), mats[t])) return set_error(YAO_EINVAL, "bad gate %zu", t);
        if (g.k < 2) continue;
        const size_t dd = size_t(1) << (2 * g.k);
        off[t] = blob.size();
        blob.resize(blob.size() + 2 * dd * rs);
        char* p = blob.data() + off[t];
        for (size_t e = 0; e < dd; ++e) {
            if (rs == 4) {
                ((float*)p)[e] = (float)mats[t].re[e];
                ((float*)p)[dd + e] = (float)mats[t].im[e];
            } else {
                ((double*)p)[e] = mats[t].re[e];
                ((double*)p)[dd + e] = mats[t].im[e];
            }
        }
    }
    char* dblob = nullptr;
    if (!blob.empty()) {
        dblob = (char*)upload_to(WS_MAT, blob.data(), blob.size());
        if (!dblob) return YAO_ENOMEM;
    }
    for (size_t t = 0; t < c->gates.size(); ++t) {
        const GateRec& g = c->gates[t];
        YAO_TRY(launch_gate(data, dtype, n, B, mats[t], g.locs, make_ctrl(g.nctrl, g.ctrls, g.cvals),
                            g.k >= 2 ? dblob + off[t] : nullptr));
    }
    return 0;
}

int backward_plain(yao_state* s, const yao_circuit* c, const double* params, yao_pauli_sum* h, bool reduce_batch,
                   double* energy, double* grad, double* drift)
{
    const int n = s->n, B = s->batch;
    const size_t elems = s->elems();
    hipStream_t st = stream();
    void* psi0 = workspace(WS_PSI0, s->bytes());
    if (!psi0) return YAO_ENOMEM;
    YAO_HIP(hipMemcpyAsync(psi0, s->data, s->bytes(), hipMemcpyDeviceToDevice, st));
    YAO_TRY(forward_plain(s->data, s->dtype, n, B, c, params));

    // psi in FP64 for the uncompute; lambda = H psi in the state's precision.
    double* psi = (double*)workspace(WS_PSI64, elems * 16);
    void* lam = workspace(WS_LAM, s->bytes());
    if (!psi || !lam) return YAO_ENOMEM;
    YAO_TRY(launch_convert(s->data, s->dtype, psi, YAO_C128, elems));
    YAO_TRY(launch_hpsi(s->data, s->dtype, lam, s->dtype, n, B, h, energy));

    // Matrices of the reverse sweep: Ud and (for parametric gates) M = (dU/dtheta) Ud, one copy.
    const size_t G = c->gates.size();
    std::vector<HostMat> Ud(G), M(G);
    std::vector<int> slot(G, -1);
    std::vector<size_t> off(G, 0);
    std::vector<double> blob;
    int nslots = 0;
    for (size_t t = 0; t < G; ++t) {
        const GateRec& g = c->gates[t];
        HostMat U;
        const double th = gate_theta(g, params);
        gate_matrix(g, th, U);
        Ud[t] = dagger(U);
        if (is_param_kind(g.kind) && g.param >= 0) {
            gate_grad_matrix(g, th, M[t]);
            slot[t] = nslots++;
        }
        if (g.k >= 2) {
            const size_t dd = size_t(1) << (2 * g.k);
            off[t] = blob.size();
            blob.resize(blob.size() + 4 * dd, 0.0);
            double* p = blob.data() + off[t];
            for (size_t e = 0; e < dd; ++e) {
                p[e] = Ud[t].re[e];
                p[dd + e] = Ud[t].im[e];
                if (slot[t] >= 0) {
                    p[2 * dd + e] = M[t].re[e];
                    p[3 * dd + e] = M[t].im[e];
                }
            }
        }
    }
    double* dblob = nullptr;
    if (!blob.empty()) {
        dblob = (double*)upload_to(WS_MAT, blob.data(), blob.size() * sizeof(double));
        if (!dblob) return YAO_ENOMEM;
    }
    const int nblk = adjoint_nblk(n, 1, B);
    double* partial = (double*)workspace(WS_PARTIAL, sizeof(double) * (size_t)(nslots > 0 ? nslots : 1) * B * nblk);
    if (!partial) return YAO_ENOMEM;
    // Gates of k >= 2 launch fewer blocks than the row stride; the rest of each row stays zero.
    if (nslots) YAO_TRY(launch_fill(partial, (size_t)nslots * B * nblk, 0.0));
    for (size_t tt = G; tt-- > 0;) {
        const GateRec& g = c->gates[tt];
        int nb = 0;
        YAO_TRY(launch_adjoint_step(psi, lam, s->dtype, n, B, Ud[tt], slot[tt] >= 0 ? &M[tt] : nullptr, g.locs,
                                    make_ctrl(g.nctrl, g.ctrls, g.cvals), g.k >= 2 ? dblob + off[tt] : nullptr,
                                    slot[tt] >= 0 ? partial + (size_t)slot[tt] * B * nblk : nullptr, &nb));
    }
    // Per-gate sums over blocks on the device, then the parameter map on the host.
    if (nslots > 0) {
        double* sums = (double*)workspace(WS_PARTIAL2, sizeof(double) * (size_t)nslots * B);
        if (!sums) return YAO_ENOMEM;
        YAO_TRY(launch_row_sums(partial, nslots * B, nblk, sums));
        double* hs = (double*)host_staging(sizeof(double) * (size_t)nslots * B);
        if (!hs) return YAO_ENOMEM;
        YAO_HIP(hipMemcpyAsync(hs, sums, sizeof(double) * (size_t)nslots * B, hipMemcpyDeviceToHost, st));
        YAO_HIP(hipStreamSynchronize(st));
        const int P = c->nparams;
        const size_t glen = reduce_batch ? (size_t)P : (size_t)P * B;
        for (size_t e = 0; e < glen; ++e) grad[e] = 0.0;
        for (size_t tt = G; tt-- > 0;) {
            if (slot[tt] < 0) continue;
            const int p = c->gates[tt].param;
            for (int b = 0; b < B; ++b) {
                double v = hs[(size_t)slot[tt] * B + b];
                if (reduce_batch) grad[p] += v;
                else grad[(size_t)b * P + p] += v;
            }
        }
    } else if (c->nparams > 0) {
        const size_t glen = reduce_batch ? (size_t)c->nparams : (size_t)c->nparams * B;
        for (size_t e = 0; e < glen; ++e) grad[e] = 0.0;
    }
    if (drift) YAO_TRY(launch_maxdiff(psi, YAO_C128, psi0, s->dtype, elems, drift));
    else YAO_HIP(hipStreamSynchronize(st));
    return 0;
}

}  // namespace yao
