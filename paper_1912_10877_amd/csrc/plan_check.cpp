// Host check of the pass planner: the passes of a plan are run on a host copy of a state the
// way the pass kernels run them -- each tile gathered from the index bits of the pass's tile,
// every op applied on tile bits from its device record (controls inside the tile as tile-bit
// masks, controls outside as a predicate on the tile's base index, dense blocks on their
// register bits), the tile stored back through the pass's bit permutation, standalone gates
// applied on the index bits of the pass's layout -- and compared with the circuit's gates
// applied one by one on the canonical layout. No GPU is used.
#include <cmath>
#include <complex>
#include <random>
#include <vector>

#include "driver.h"
#include "fused.h"

namespace yao {
namespace {

using cd = std::complex<double>;

// One gate (U, or U^dagger when dag) on qubits locs with controls, on a state of n qubits.
void apply_host(std::vector<cd>& s, int n, int k, const int* locs, int nctrl, const int* ctrls, const int* cvals,
                const HostMat& U, bool dag)
{
    const int D = 1 << k;
    std::vector<uint64_t> idx(D);
    std::vector<cd> in(D);
    for (uint64_t i = 0; i < (uint64_t(1) << n); ++i) {
        bool ok = true;
        for (int j = 0; j < k; ++j) ok &= !((i >> locs[j]) & 1);
        for (int m = 0; m < nctrl; ++m) ok &= (int)((i >> ctrls[m]) & 1) == cvals[m];
        if (!ok) continue;
        for (int a = 0; a < D; ++a) {
            uint64_t e = i;
            for (int j = 0; j < k; ++j) e |= uint64_t((a >> j) & 1) << locs[j];
            idx[a] = e;
            in[a] = s[e];
        }
        for (int r = 0; r < D; ++r) {
            cd acc = 0;
            for (int a = 0; a < D; ++a)
                acc += (dag ? std::conj(cd(U.re[a * D + r], U.im[a * D + r])) : cd(U.re[r * D + a], U.im[r * D + a])) *
                       in[a];
            s[idx[r]] = acc;
        }
    }
}

// D x D matrix m (row-major, dim D) on the tile elements that differ in bits pos[0 .. k).
void apply_tile(std::vector<cd>& loc, int k, const int* pos, uint32_t cmask, uint32_t cval, const cd* m)
{
    const int D = 1 << k;
    std::vector<uint64_t> idx(D);
    std::vector<cd> in(D);
    for (uint64_t e = 0; e < loc.size(); ++e) {
        bool ok = (e & cmask) == cval;
        for (int j = 0; j < k; ++j) ok &= !((e >> pos[j]) & 1);
        if (!ok) continue;
        for (int a = 0; a < D; ++a) {
            uint64_t f = e;
            for (int j = 0; j < k; ++j) f |= uint64_t((a >> j) & 1) << pos[j];
            idx[a] = f;
            in[a] = loc[f];
        }
        for (int r = 0; r < D; ++r) {
            cd acc = 0;
            for (int a = 0; a < D; ++a) acc += m[r * D + a] * in[a];
            loc[idx[r]] = acc;
        }
    }
}

int run_passes(const Plan& P, const Program& prog, const yao_circuit* c, const double* params, std::vector<cd>& s)
{
    const int n = P.n;
    for (size_t p = 0; p < P.passes.size(); ++p) {
        const HostPass& pass = P.passes[p];
        if (pass.standalone >= 0) {
            const GateRec& g = c->gates[P.ops[pass.standalone].gate];
            HostMat U;
            if (!gate_matrix(g, gate_theta(g, params), U)) return set_error(YAO_EINVAL, "bad gate");
            int locs[8], ctrls[kGateMaxCtrl];
            for (int j = 0; j < g.k; ++j) locs[j] = pass.phys.empty() ? g.locs[j] : pass.phys[g.locs[j]];
            for (int m = 0; m < g.nctrl; ++m) ctrls[m] = pass.phys.empty() ? g.ctrls[m] : pass.phys[g.ctrls[m]];
            apply_host(s, n, g.k, locs, g.nctrl, ctrls, g.cvals, U, P.reverse);
            continue;
        }
        const int tq = (int)pass.tile_qubits.size();
        uint64_t TP = 0;
        for (int q : pass.tile_qubits) TP |= uint64_t(1) << q;
        std::vector<int> outside;
        for (int q = 0; q < n; ++q)
            if (!((TP >> q) & 1)) outside.push_back(q);
        std::vector<cd> loc(size_t(1) << tq), out(loc.size());
        auto addr = [&](uint64_t base, uint64_t e) {
            for (int j = 0; j < tq; ++j) base |= ((e >> j) & 1) << pass.tile_qubits[j];
            return base;
        };
        for (uint64_t b = 0; b < (uint64_t(1) << outside.size()); ++b) {
            uint64_t base = 0;
            for (size_t j = 0; j < outside.size(); ++j) base |= ((b >> j) & 1) << outside[j];
            for (uint64_t e = 0; e < loc.size(); ++e) loc[e] = s[addr(base, e)];
            for (size_t gi = 0; gi < pass.groups.size(); ++gi) {
                const PGroupDesc& gd = prog.groups[prog.pass_group0[p] + gi];
                for (int oi = 0; oi < gd.nops; ++oi) {
                    const POp& op = prog.ops[prog.pass_op0[p] + gd.op0 + oi];
                    if ((base & op.omask) != op.oval) continue;
                    if (gd.lds == 2) {
                        // Dense block: 16 x 16, column-major re[16] then im[16] (complex128 programs).
                        const double* F = prog.mats.data() + prog.pass_dmat0[p] + (size_t)op.mat * 512;
                        std::vector<cd> M(256);
                        for (int r = 0; r < 16; ++r)
                            for (int a = 0; a < 16; ++a) M[r * 16 + a] = cd(F[a * 32 + r], F[a * 32 + 16 + r]);
                        apply_tile(loc, 4, gd.rpos, op.cmask, op.cval, M.data());
                        continue;
                    }
                    const int D = 1 << op.k;
                    std::vector<cd> M(D * D);
                    if (op.k == 1) {
                        for (int e = 0; e < 4; ++e) M[e] = cd(op.u[e], op.u[4 + e]);
                        // Reverse Z-generator diagonal ops hold d1 / d0; the kernel applies d0
                        // as a phase of the whole tile at the store.
                        if (P.reverse && op.var / P.reg_bits == 1) M[3] *= M[0];
                    } else {
                        const double* m = prog.mats.data() + op.mat;
                        for (int e = 0; e < D * D; ++e) M[e] = cd(m[e], m[D * D + e]);
                    }
                    apply_tile(loc, op.k, op.tpos, op.cmask, op.cval, M.data());
                }
            }
            for (uint64_t e = 0; e < loc.size(); ++e) {
                uint64_t src = e;
                if (!pass.store_src.empty()) {
                    src = 0;
                    for (int i = 0; i < tq; ++i) src |= ((e >> i) & 1) << pass.store_src[i];
                }
                out[e] = loc[src];
            }
            for (uint64_t e = 0; e < loc.size(); ++e) s[addr(base, e)] = out[e];
        }
    }
    return 0;
}

}  // namespace

int plan_selfcheck(const yao_circuit* c, const double* params, int dtype, int reverse, int tile_qubits, double* max_err,
                   int* npasses)
{
    const int n = c->n;
    if (n > 20) return set_error(YAO_EINVAL, "plan self-check runs on the host: at most 20 qubits");
    int t, cb, L;
    tile_geometry_tq(n, 1, dtype, reverse != 0, tile_qubits, &t, &cb, &L);
    if (t - cb < kMaxRegBits + 1) return set_error(YAO_EINVAL, "circuit too small for tile passes");
    const Plan& P = get_plan(c, 0, (int)c->gates.size(), 1, t, cb, L, reverse != 0, dtype == YAO_C64 ? 8 : 16);
    if (!P.valid) return set_error(YAO_EINVAL, "pass plan could not restore the qubit layout");
    Program prog;
    YAO_TRY(build_program(P, c, params, reverse != 0, YAO_C128, prog));
    std::mt19937_64 rng(12345);
    std::normal_distribution<double> N01;
    std::vector<cd> ref(size_t(1) << n);
    for (cd& v : ref) v = cd(N01(rng), N01(rng));
    std::vector<cd> got = ref;
    const int G = (int)c->gates.size();
    for (int e = 0; e < G; ++e) {
        const GateRec& g = c->gates[reverse ? G - 1 - e : e];
        HostMat U;
        if (!gate_matrix(g, gate_theta(g, params), U)) return set_error(YAO_EINVAL, "bad gate");
        apply_host(ref, n, g.k, g.locs, g.nctrl, g.ctrls, g.cvals, U, reverse != 0);
    }
    YAO_TRY(run_passes(P, prog, c, params, got));
    double err = 0;
    for (size_t i = 0; i < ref.size(); ++i) err = std::max(err, std::abs(ref[i] - got[i]));
    *max_err = err;
    *npasses = (int)P.passes.size();
    return 0;
}

}  // namespace yao
