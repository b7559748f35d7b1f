// Host planner of the fused tile passes.
//
// Gates are taken in order. A gate may join the pass being formed when its targets fit in the
// tile and it shares no qubit (target or control) with a gate that was deferred earlier in
// this scan -- so moving it ahead of those gates cannot change the result, since operators
// on disjoint qubits commute. The same rule, with 3 or 4 register bits in place of the
// tile, splits a pass into register groups.
#include <algorithm>

#include "fused.h"

namespace yao {

static int popc(uint64_t v)
{
    return __builtin_popcountll(v);
}

void tile_geometry(int n, int B, int dtype, bool backward, int* t, int* cbits, int* low_fixed)
{
    tile_geometry_tq(n, B, dtype, backward, options().tile_qubits, t, cbits, low_fixed);
}

void tile_geometry_tq(int n, int B, int dtype, bool backward, int tq, int* t, int* cbits, int* low_fixed)
{
    const int lb = ilog2_ceil((uint64_t)B);
    const int c = lb < 3 ? lb : 3;
    if (tq <= 0) tq = 12 - c;
    if (tq < kMaxRegBits + 1) tq = kMaxRegBits + 1;
    int tt = c + std::min(tq, n);
    // LDS per tile element: forward 8 or 16 bytes; backward 16 (psi) + 8 or 16 (lambda), plus
    // the gradient partials, within 160 KiB.
    const int tmax = backward ? (dtype == YAO_C64 ? 12 : 11) : (dtype == YAO_C64 ? 13 : 12);
    if (tt > tmax) tt = tmax;
    *t = tt;
    *cbits = c;
    // Keep enough of the lowest qubits in every tile that each row of the tile spans at least
    // 128 contiguous bytes (16 complex64 or 8 complex128 elements).
    const int want = (dtype == YAO_C64 ? 4 : 3) - c;
    *low_fixed = std::max(0, std::min(want, tt - c));
}

bool fused_supported(int n, int B)
{
    (void)B;
    return n >= kMaxRegBits + 1;
}

Plan make_plan(const yao_circuit* circ, int g0, int g1, int B, int t, int cbits, int low_fixed, bool reverse,
               int reg_bits, int max_ops)
{
    Plan P;
    P.reg_bits = reg_bits;
    P.g0 = g0;
    P.g1 = g1;
    P.n = circ->n;
    P.B = B;
    P.c = cbits;
    P.t = t;
    P.reverse = reverse;
    for (int e = g0; e < g1; ++e) {
        const int gi = reverse ? g1 - 1 - (e - g0) : e;
        const GateRec& g = circ->gates[gi];
        HostOp op;
        op.gate = gi;
        op.tmask = 0;
        for (int j = 0; j < g.k; ++j) op.tmask |= uint64_t(1) << g.locs[j];
        op.qmask = op.tmask;
        for (int m = 0; m < g.nctrl; ++m) op.qmask |= uint64_t(1) << g.ctrls[m];
        P.ops.push_back(op);
    }
    const int tq = t - cbits;
    const uint64_t low = low_fixed > 0 ? ((uint64_t(1) << low_fixed) - 1) : 0;
    // Widest gate a pass takes: forward passes over tiles of >= 64 register-group columns apply
    // k <= 4 gates as dense blocks on a register group; other passes apply k <= 3 gates in LDS.
    const bool dense_ok = !reverse && t - reg_bits >= 6 && reg_bits >= kMaxDenseK;
    const int maxk = dense_ok ? kMaxDenseK : kMaxFusedK;
    std::vector<int> remaining(P.ops.size());
    for (size_t e = 0; e < remaining.size(); ++e) remaining[e] = (int)e;

    while (!remaining.empty()) {
        HostPass pass;
        // A gate too wide for a tile runs alone when it is next.
        const GateRec& first = circ->gates[P.ops[remaining[0]].gate];
        if (first.k > maxk) {
            pass.standalone = remaining[0];
            remaining.erase(remaining.begin());
            P.passes.push_back(pass);
            continue;
        }
        // The fixed low qubits give way when the first gate would not fit next to them.
        uint64_t T = popc(low | P.ops[remaining[0]].tmask) <= tq ? low : 0;
        uint64_t blocked = 0;
        std::vector<int> sel, rest;
        int ndense = 0;
        for (int oi : remaining) {
            const HostOp& op = P.ops[oi];
            const int k = circ->gates[op.gate].k;
            const bool dense = dense_ok && k > 1;
            if ((op.qmask & blocked) || k > maxk || (int)sel.size() >= max_ops ||
                (dense && ndense >= kMaxPassDense)) {
                blocked |= op.qmask;
                rest.push_back(oi);
                continue;
            }
            if (popc(T | op.tmask) <= tq) {
                T |= op.tmask;
                sel.push_back(oi);
                ndense += dense ? 1 : 0;
            } else {
                blocked |= op.qmask;
                rest.push_back(oi);
            }
        }
        // Fill the tile with the lowest unused qubits.
        for (int q = 0; q < P.n && popc(T) < tq; ++q) T |= uint64_t(1) << q;
        for (int q = 0; q < P.n; ++q)
            if ((T >> q) & 1) pass.tile_qubits.push_back(q);
        auto tile_bit = [&](int q) {
            int r = 0;
            for (int j = 0; j < q; ++j) r += (T >> j) & 1;
            return cbits + r;
        };
        // Register groups.
        std::vector<int> prem = sel;
        while (!prem.empty()) {
            HostGroup grp;
            uint64_t R = 0, gblocked = 0;
            std::vector<int> gsel, grest;
            bool lds_first = circ->gates[P.ops[prem[0]].gate].k > 1;
            if (lds_first && dense_ok) {
                // Dense block on a register group: its targets, its controls inside the tile
                // while they fit (they are folded into the matrix), then padding bits.
                const HostOp& op = P.ops[prem[0]];
                const GateRec& gr = circ->gates[op.gate];
                grp.dense = true;
                grp.ops.push_back(prem[0]);
                for (int j = 0; j < gr.k; ++j) R |= uint64_t(1) << tile_bit(gr.locs[j]);
                for (int m = 0; m < gr.nctrl; ++m) {
                    const int q = gr.ctrls[m];
                    if (((T >> q) & 1) && popc(R | (uint64_t(1) << tile_bit(q))) <= reg_bits)
                        R |= uint64_t(1) << tile_bit(q);
                }
                for (int b = t - 1; b >= cbits && popc(R) < reg_bits; --b) R |= uint64_t(1) << b;
                grp.rbits = R;
                prem.erase(prem.begin());
                pass.groups.push_back(grp);
                continue;
            }
            if (lds_first) {
                grp.lds = true;
                grp.ops.push_back(prem[0]);
                const HostOp& op = P.ops[prem[0]];
                for (int q = 0; q < P.n; ++q)
                    if ((op.tmask >> q) & 1) R |= uint64_t(1) << tile_bit(q);
                grp.rbits = R;
                prem.erase(prem.begin());
                pass.groups.push_back(grp);
                continue;
            }
            int nslot = 0;
            for (int oi : prem) {
                const HostOp& op = P.ops[oi];
                const GateRec& gr = circ->gates[op.gate];
                const int k = gr.k;
                const bool grad = is_param_kind(gr.kind) && gr.param >= 0;
                uint64_t rb = 0;
                for (int q = 0; q < P.n; ++q)
                    if ((op.tmask >> q) & 1) rb |= uint64_t(1) << tile_bit(q);
                if ((op.qmask & gblocked) || k > 1 || (grad && nslot >= kMaxGroupSlots)) {
                    gblocked |= op.qmask;
                    grest.push_back(oi);
                    continue;
                }
                if (popc(R | rb) <= reg_bits) {
                    R |= rb;
                    gsel.push_back(oi);
                    nslot += grad ? 1 : 0;
                } else {
                    gblocked |= op.qmask;
                    grest.push_back(oi);
                }
            }
            // Fill the register bits with the highest unused tile bits, which keeps the thread
            // bits on the low (contiguous) end of the tile.
            for (int b = t - 1; b >= cbits && popc(R) < reg_bits; --b) R |= uint64_t(1) << b;
            grp.rbits = R;
            grp.ops = gsel;
            pass.groups.push_back(grp);
            prem = grest;
        }
        P.passes.push_back(pass);
        remaining = rest;
    }
    return P;
}

}  // namespace yao
