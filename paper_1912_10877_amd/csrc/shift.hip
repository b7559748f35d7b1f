// Faithful gradient by the shift rule (Sec. "Forward Mode: Faithful Quantum Gradients", eq.
// shiftrule), every shifted circuit in one batched register.
//
// For every parametrised gate occurrence k (a rotation exp(-i theta G / 2) with G reflexive, or a
// phase shift), the energies with that gate's angle moved by +pi/2 and -pi/2 give
// (E+ - E-) / 2, added to the gradient of the gate's parameter. A rotation by theta + pi/2 is the
// rotation by theta followed by the rotation by pi/2 about the same generator (likewise for the
// phase shift), so the shifted circuit is the circuit with one extra fixed gate right after gate
// k, carrying gate k's controls.
//
// All 2K shifted circuits (and the unshifted one) run at once on a register of n + s qubits:
// slot j = the top s index bits holds circuit j's copy of the n-qubit state, every gate of the
// circuit acts on all slots, and the extra gate of slot j is controlled by the slot bits reading
// j. So the whole batch is one forward sweep of one circuit through the fused tile passes (the
// slot controls lie outside every tile and become per-tile predicates), followed by one
// expectation pass with per-slot sums. Slots are cut into chunks when the register would exceed
// the memory budget.
#include <cmath>
#include <vector>

#include "driver.h"
#include "fused.h"
#include "runtime.h"

namespace yao {

namespace {

constexpr int kSThreads = 256;

template <typename V>
__global__ __launch_bounds__(kSThreads) void k_broadcast(const V* __restrict__ src, V* __restrict__ dst,
                                                         uint64_t per_slot, uint64_t total)
{
    for (uint64_t e = (uint64_t)blockIdx.x * kSThreads + threadIdx.x; e < total; e += (uint64_t)gridDim.x * kSThreads)
        dst[e] = src[e & (per_slot - 1)];
}

// Energy of every slot of a register [slot][2^n] with 2^n <= 4096 amplitudes per slot: one
// workgroup per slot loads it into LDS and sums c_t Re(conj(psi[i ^ x]) i^ny (-1)^{|i & z|} psi[i])
// over its amplitudes and the Pauli terms (tables grouped by X mask), then a fixed-tree reduction.
template <typename R>
__global__ __launch_bounds__(kSThreads) void k_slot_expect(const vec2_t<R>* __restrict__ psi, int n,
                                                           const PGroup* __restrict__ groups, int ngroups,
                                                           const PTerm* __restrict__ terms, double* __restrict__ out)
{
    extern __shared__ char lds_raw[];
    vec2_t<R>* t = reinterpret_cast<vec2_t<R>*>(lds_raw);
    __shared__ double red[kSThreads];
    const uint64_t N = uint64_t(1) << n;
    const vec2_t<R>* p = psi + (uint64_t)blockIdx.x * N;
    for (uint64_t i = threadIdx.x; i < N; i += kSThreads) t[i] = p[i];
    __syncthreads();
    double acc = 0;
    for (uint64_t i = threadIdx.x; i < N; i += kSThreads) {
        const vec2_t<R> a = t[i];
        for (int g = 0; g < ngroups; ++g) {
            const vec2_t<R> q = t[i ^ groups[g].x];
            const double wr = (double)q.x * a.x + (double)q.y * a.y;
            const double wi = (double)q.x * a.y - (double)q.y * a.x;
            for (int k = groups[g].t0; k < groups[g].t1; ++k) {
                double v;
                switch (terms[k].ny & 3) {
                case 0: v = wr; break;
                case 1: v = -wi; break;
                case 2: v = -wr; break;
                default: v = wi; break;
                }
                acc += (__popcll(i & terms[k].z) & 1) ? -terms[k].c * v : terms[k].c * v;
            }
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kSThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// out[s] = sum over the observable passes p and the tiles j of slot s of
// partial[p * ntiles + s * per + j] (the slot bits are the top bits of the tile index).
__global__ void k_slot_sums(const double* __restrict__ partial, int npass, uint64_t ntiles, uint64_t per, int nslots,
                            double* __restrict__ out)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    double acc = 0;
    for (int p = 0; p < npass; ++p)
        for (uint64_t j = 0; j < per; ++j) acc += partial[(uint64_t)p * ntiles + (uint64_t)s * per + j];
    out[s] = acc;
}

// Dynamic LDS above 64 KiB (a 12-qubit complex128 slot) needs the kernel's limit raised once.
int slot_expect_lds_limit()
{
    static bool done = false;
    if (done) return 0;
    YAO_HIP(hipFuncSetAttribute((const void*)k_slot_expect<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                96 * 1024));
    YAO_HIP(hipFuncSetAttribute((const void*)k_slot_expect<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                96 * 1024));
    done = true;
    return 0;
}

bool shiftable(const GateRec& g)
{
    return g.param >= 0 && is_param_kind(g.kind);
}

}  // namespace

int shift_grad(const yao_state* st, const yao_circuit* c, const double* params, yao_pauli_sum* h, double* energy,
               double* grad)
{
    const int n = st->n;
    const int dtype = st->dtype;
    const size_t es = st->elem_bytes();
    std::vector<int> occ;  // gate index of each shiftable occurrence
    for (int gi = 0; gi < (int)c->gates.size(); ++gi)
        if (shiftable(c->gates[gi])) occ.push_back(gi);
    const long K = (long)occ.size();
    const long nslots = 2 * K + 1;  // slot 2K: the unshifted circuit
    int s_all = 0;
    while ((1L << s_all) < nslots) ++s_all;
    // Memory budget of the register: a quarter of the free device memory, at most 64 GiB.
    size_t freeb = 0, totalb = 0;
    YAO_HIP(hipMemGetInfo(&freeb, &totalb));
    const size_t budget = std::min<size_t>(freeb / 4, size_t(64) << 30);
    if ((es << n) > budget) return set_error(YAO_ENOMEM, "a %d-qubit slot exceeds the memory budget", n);
    int s_max = 0;  // slot bits of a chunk
    while (s_max < s_all && (es << (n + s_max + 1)) <= budget && n + s_max + 1 <= 34) ++s_max;
    const long per_chunk = 1L << s_max;
    std::vector<double> E(nslots, 0.0);
    for (int p = 0; p < c->nparams; ++p) grad[p] = 0.0;

    void* reg = nullptr;
    const size_t reg_bytes = es << (n + s_max);
    if (hipMalloc(&reg, reg_bytes) != hipSuccess) return set_error(YAO_ENOMEM, "shifted-circuit register %zu bytes", reg_bytes);
    int rc = 0;
    yao_pauli_sum hx;
    for (long j0 = 0; j0 < nslots && rc == 0; j0 += per_chunk) {
        const long cnt = std::min(per_chunk, nslots - j0);
        int s = 0;
        while ((1L << s) < cnt) ++s;
        const int nx = n + s;
        // The circuit on n + s qubits: every gate, then after occurrence k the +pi/2 gate on slot
        // 2k and the -pi/2 gate on slot 2k + 1 (when those slots lie in this chunk).
        yao_circuit cx;
        cx.n = nx;
        cx.nparams = c->nparams;
        cx.version = 0;
        long k = 0;
        for (int gi = 0; gi < (int)c->gates.size(); ++gi) {
            const GateRec& g = c->gates[gi];
            cx.gates.push_back(g);
            if (!shiftable(g)) continue;
            for (int sign = 0; sign < 2; ++sign) {
                const long slot = 2 * k + sign - j0;
                if (slot < 0 || slot >= cnt) continue;
                if (g.nctrl + s > kGateMaxCtrl) {
                    rc = set_error(YAO_EINVAL, "gate %d has too many controls for the shifted register", gi);
                    break;
                }
                GateRec x = g;
                x.param = -1;
                x.theta = sign == 0 ? M_PI / 2 : -M_PI / 2;
                for (int b = 0; b < s; ++b) {
                    x.ctrls[x.nctrl] = n + b;
                    x.cvals[x.nctrl] = (int)((slot >> b) & 1);
                    ++x.nctrl;
                }
                cx.gates.push_back(x);
            }
            ++k;
        }
        if (rc) break;
        const uint64_t per_slot = uint64_t(1) << n;
        const uint64_t total = per_slot << s;
        const unsigned nb = (unsigned)std::min<uint64_t>((total + kSThreads - 1) / kSThreads, 65536);
        if (dtype == YAO_C64)
            k_broadcast<float2><<<nb, kSThreads, 0, stream()>>>((const float2*)st->data, (float2*)reg, per_slot, total);
        else
            k_broadcast<double2><<<nb, kSThreads, 0, stream()>>>((const double2*)st->data, (double2*)reg, per_slot, total);
        {
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) {
                rc = hip_fail(e, "k_broadcast");
                break;
            }
        }
        // Runs of one-qubit gates merge into one matrix (the extra gates are controlled, so they
        // stay apart).
        rc = forward_sweep(reg, dtype, nx, 1, &cx, params, 1, options().tile_qubits, nullptr);
        if (rc) {
            drop_plans(&cx);
            drop_fused(&cx);
            break;
        }
        // Per-slot energies.
        double* dE = (double*)workspace(WS_MISC, sizeof(double) * (size_t)(1L << s));
        if (!dE) {
            rc = YAO_ENOMEM;
            drop_plans(&cx);
            drop_fused(&cx);
            break;
        }
        if (n <= 12) {
            if ((rc = pauli_upload(h)) == 0) rc = slot_expect_lds_limit();
            if (rc == 0) {
                const size_t lds = es << n;
                if (dtype == YAO_C64)
                    k_slot_expect<float><<<(unsigned)(1L << s), kSThreads, lds, stream()>>>(
                        (const float2*)reg, n, (const PGroup*)h->d_groups, h->ngroups, (const PTerm*)h->d_terms, dE);
                else
                    k_slot_expect<double><<<(unsigned)(1L << s), kSThreads, lds, stream()>>>(
                        (const double2*)reg, n, (const PGroup*)h->d_groups, h->ngroups, (const PTerm*)h->d_terms, dE);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) rc = hip_fail(e, "k_slot_expect");
            }
        } else {
            // The observable on the wide register: tiles of the low qubits only (n >= 13 fills a
            // tile), so every tile belongs to one slot.
            hx.n = nx;
            hx.coef = h->coef;
            hx.x = h->x;
            hx.z = h->z;
            const size_t np = obs_partial_doubles(&hx, nx, 1, dtype);
            double* part = np ? (double*)workspace(WS_PARTIAL, sizeof(double) * np) : nullptr;
            int W = 0;
            if (!part) rc = YAO_ENOMEM;
            else rc = launch_obs_passes(reg, dtype, nullptr, dtype, nx, 1, &hx, part, &W);
            if (rc == 0) {
                const uint64_t ntiles = uint64_t(1) << (nx - obs_tile_qubits(&hx, nx, 1, dtype));
                const int npass = (int)(W / ntiles);
                k_slot_sums<<<(unsigned)(((1L << s) + 63) / 64), 64, 0, stream()>>>(part, npass, ntiles,
                                                                                     ntiles >> s, (int)(1L << s), dE);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) rc = hip_fail(e, "k_slot_sums");
            }
            drop_obs_plans(&hx);
        }
        if (rc == 0) {
            hipError_t e = hipMemcpyAsync(E.data() + j0, dE, sizeof(double) * cnt, hipMemcpyDeviceToHost, stream());
            if (e == hipSuccess) e = hipStreamSynchronize(stream());
            if (e != hipSuccess) rc = hip_fail(e, "energies");
        }
        drop_plans(&cx);
        drop_fused(&cx);
    }
    (void)hipFree(reg);
    if (rc) return rc;
    for (long k = 0; k < K; ++k) grad[c->gates[occ[k]].param] += 0.5 * (E[2 * k] - E[2 * k + 1]);
    *energy = E[2 * K];
    return 0;
}

}  // namespace yao
