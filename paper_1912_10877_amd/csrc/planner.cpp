// Host planner of the fused tile passes.
//
// Gates are taken in order. A gate may join a pass when its targets lie in the pass's tile
// and neither its targets touch a qubit of a gate deferred earlier in this scan nor its
// controls touch such a gate's targets -- so moving it ahead of those gates cannot change the
// result: two controlled gates that share only control qubits are block diagonal in those
// qubits and act on disjoint targets, so they commute like gates on disjoint qubits. The same
// rule, with 3 or 4 register bits in place of the tile, splits a pass into register groups.
//
// Tiles are grown one qubit at a time, each time adding the qubit that lets the pass take the
// most gates. On a layered circuit this alternates between overlapping windows whose gates
// form a staircase, several layers deep, rather than one layer slice per pass. Successive
// tiles share at least `low_fixed` qubits: each pass stores its tile with those shared
// qubits moved onto the lowest index bits, so every tile spans whole contiguous rows of
// memory without fixing which qubits live there. The last pass (or a few plain permuting
// passes after it) puts every qubit back on its own bit.
#include <algorithm>
#include <climits>

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

namespace {

uint64_t bit(int q)
{
    return uint64_t(1) << q;
}

// The ops of `remaining` a pass over tile T (a qubit mask) takes, in order. With sel and rest
// null it only counts, and stops once every qubit of `all` is blocked.
int take_ops(const Plan& P, const yao_circuit* circ, const std::vector<int>& remaining, uint64_t T, int maxk,
             bool dense_ok, int max_ops, uint64_t all, std::vector<int>* sel, std::vector<int>* rest)
{
    uint64_t blocked = 0, blocked_t = 0;  // qubits / targets of the deferred ops
    int nsel = 0, ndense = 0;
    for (int oi : remaining) {
        const HostOp& op = P.ops[oi];
        const int k = circ->gates[op.gate].k;
        const bool dense = dense_ok && k > 1;
        if ((op.tmask & blocked) || (op.qmask & blocked_t) || (op.tmask & ~T) || k > maxk || nsel >= max_ops ||
            (dense && ndense >= kMaxPassDense)) {
            blocked |= op.qmask;
            blocked_t |= op.tmask;
            if (rest) rest->push_back(oi);
            else if ((blocked & all) == all) break;
            continue;
        }
        ++nsel;
        ndense += dense ? 1 : 0;
        if (sel) sel->push_back(oi);
    }
    return nsel;
}

// Tile of tq qubits for the next pass: the targets of the first remaining op, then one qubit
// at a time the one that lets the pass take the most ops (ties: the qubit the remaining ops
// use soonest). At least `need` of its qubits come from `cand` when that is possible.
uint64_t choose_tile(const Plan& P, const yao_circuit* circ, const std::vector<int>& remaining, int tq,
                     uint64_t cand, int need, int maxk, bool dense_ok, int max_ops)
{
    const int n = P.n;
    const uint64_t all = n >= 64 ? ~uint64_t(0) : bit(n) - 1;
    if (tq >= n) return all;
    std::vector<int> first(n, INT_MAX);
    uint64_t seen = 0;
    for (size_t i = 0; i < remaining.size() && seen != all; ++i) {
        uint64_t m = P.ops[remaining[i]].qmask & ~seen;
        seen |= m;
        for (; m; m &= m - 1) first[__builtin_ctzll(m)] = (int)i;
    }
    uint64_t T = P.ops[remaining[0]].tmask;
    need = std::min(need, popc(cand));
    while (popc(T) < tq) {
        const bool must = need - popc(T & cand) >= tq - popc(T);
        int best = -1, bq = -1;
        for (int q = 0; q < n; ++q) {
            if (((T >> q) & 1) || (must && !((cand >> q) & 1))) continue;
            const int v = take_ops(P, circ, remaining, T | bit(q), maxk, dense_ok, max_ops, all, nullptr, nullptr);
            if (v > best || (v == best && first[q] < first[bq])) {
                best = v;
                bq = q;
            }
        }
        if (bq < 0) break;
        T |= bit(bq);
    }
    return T;
}

// Sets pass.tile_qubits (the index bits of tile T under layout phys) and moves the qubits of T
// to new bits within them: lg (index bit -> qubit) is updated and pass.store_src records the
// move. place(positions, qubits, lg) assigns the tile's qubits to its bits.
template <typename Place>
void permute_tile(HostPass& pass, uint64_t T, int c, std::vector<int>& phys, std::vector<int>& lg, Place place)
{
    std::vector<int> pos;
    for (int q = 0; q < (int)phys.size(); ++q)
        if ((T >> q) & 1) pos.push_back(phys[q]);
    std::sort(pos.begin(), pos.end());
    pass.tile_qubits = pos;
    const std::vector<int> old_lg = lg;
    place(pos, lg);
    // LDS tile bit of each index bit before the move.
    std::vector<int> src(c + pos.size());
    for (int b = 0; b < c; ++b) src[b] = b;
    bool ident = true;
    for (size_t j = 0; j < pos.size(); ++j) {
        const int q = lg[pos[j]];
        size_t from = 0;
        while (old_lg[pos[from]] != q) ++from;
        src[c + j] = c + (int)from;
        ident &= from == j;
    }
    if (!ident) pass.store_src = src;
    for (int p : pos) phys[lg[p]] = p;
}

}  // namespace

Plan make_plan(const yao_circuit* circ, int g0, int g1, int B, int t, int cbits, int low_fixed, bool reverse,
               int reg_bits, int max_ops, int max_slots)
{
    Plan P;
    P.reg_bits = reg_bits;
    P.max_slots = max_slots;
    P.g0 = g0;
    P.g1 = g1;
    P.n = circ->n;
    P.B = B;
    P.c = cbits;
    P.t = t;
    P.reverse = reverse;
    const int n = P.n;
    for (int e = g0; e < g1; ++e) {
        const int gi = reverse ? g1 - 1 - (e - g0) : e;
        const GateRec& g = circ->gates[gi];
        HostOp op;
        op.gate = gi;
        op.tmask = 0;
        for (int j = 0; j < g.k; ++j) op.tmask |= bit(g.locs[j]);
        op.qmask = op.tmask;
        for (int m = 0; m < g.nctrl; ++m) op.qmask |= bit(g.ctrls[m]);
        P.ops.push_back(op);
    }
    const int tq = t - cbits;
    const int L = std::min(low_fixed, tq);
    // Widest gate a pass takes: forward passes over tiles of >= 64 register-group columns apply
    // k <= 4 gates as dense blocks on a register group; other passes apply k <= 3 gates in LDS.
    const bool dense_ok = !reverse && t - reg_bits >= 6 && reg_bits >= kMaxDenseK;
    const int maxk = dense_ok ? kMaxDenseK : kMaxFusedK;
    std::vector<int> remaining(P.ops.size());
    for (size_t e = 0; e < remaining.size(); ++e) remaining[e] = (int)e;

    // Tiles and their ops. The first tile must hold the qubits on the low index bits (the
    // state comes in with qubit q on bit q); each later one shares L qubits with the one
    // before it.
    std::vector<uint64_t> tiles;
    std::vector<std::vector<int>> taken;
    uint64_t cand = L > 0 ? bit(L) - 1 : 0;
    while (!remaining.empty()) {
        HostPass pass;
        // A gate too wide for a tile runs alone when it is next.
        const GateRec& first = circ->gates[P.ops[remaining[0]].gate];
        if (first.k > maxk) {
            pass.standalone = remaining[0];
            remaining.erase(remaining.begin());
            P.passes.push_back(pass);
            tiles.push_back(0);
            taken.emplace_back();
            continue;
        }
        const uint64_t T = choose_tile(P, circ, remaining, tq, cand, L, maxk, dense_ok, max_ops);
        std::vector<int> sel, rest;
        take_ops(P, circ, remaining, T, maxk, dense_ok, max_ops, 0, &sel, &rest);
        P.passes.push_back(pass);
        tiles.push_back(T);
        taken.push_back(sel);
        remaining = rest;
        cand = T;
    }

    // Layouts: each pass moves qubits it shares with the next tile onto the low bits; the last
    // puts back every qubit it can.
    std::vector<int> phys(n), lg(n);
    for (int q = 0; q < n; ++q) phys[q] = lg[q] = q;
    auto identity = [&]() {
        for (int q = 0; q < n; ++q)
            if (phys[q] != q) return false;
        return true;
    };
    auto restore_in = [&](const std::vector<int>& pos, std::vector<int>& l) {
        // Bits whose own qubit is in the tile take it; the others take the rest in order.
        std::vector<int> qs, rest_q, free_p;
        for (int p : pos) qs.push_back(l[p]);
        std::vector<char> placed(n, 0);
        for (int p : pos)
            if (std::find(qs.begin(), qs.end(), p) != qs.end()) placed[p] = 1;
        for (int q : qs)
            if (!placed[q]) rest_q.push_back(q);
        for (int p : pos)
            if (!placed[p]) free_p.push_back(p);
        for (int p : pos)
            if (placed[p]) l[p] = p;
        for (size_t j = 0; j < free_p.size(); ++j) l[free_p[j]] = rest_q[j];
    };
    for (size_t k = 0; k < P.passes.size(); ++k) {
        HostPass& pass = P.passes[k];
        if (!identity()) pass.phys = phys;
        if (pass.standalone >= 0) continue;
        size_t nx = k + 1;
        while (nx < P.passes.size() && P.passes[nx].standalone >= 0) ++nx;
        const uint64_t T = tiles[k];
        if (nx < P.passes.size()) {
            const uint64_t want = T & tiles[nx];
            permute_tile(pass, T, cbits, phys, lg, [&](const std::vector<int>& pos, std::vector<int>& l) {
                // Each low bit of the tile takes, if the next tile wants it: its own qubit,
                // else the qubit it holds, else another wanted qubit from higher in the tile.
                // Preferring a bit's own qubit keeps the layout close to the identity.
                auto at = [&](int q) {
                    for (int p : pos)
                        if (l[p] == q) return p;
                    return -1;
                };
                std::vector<int> lows, target;
                for (int p = 0; p < L; ++p)
                    if (std::find(pos.begin(), pos.end(), p) != pos.end()) lows.push_back(p);
                target.assign(lows.size(), -1);
                uint64_t used = 0;
                for (size_t i = 0; i < lows.size(); ++i) {
                    const int p = lows[i];
                    if (((want >> p) & 1) && at(p) >= 0) {
                        target[i] = p;
                        used |= bit(p);
                    }
                }
                for (size_t i = 0; i < lows.size(); ++i) {
                    const int q = l[lows[i]];
                    if (target[i] < 0 && ((want >> q) & 1) && !((used >> q) & 1)) {
                        target[i] = q;
                        used |= bit(q);
                    }
                }
                for (size_t i = 0; i < lows.size(); ++i) {
                    if (target[i] >= 0) continue;
                    for (int p : pos) {
                        const int q = l[p];
                        if (p >= L && ((want >> q) & 1) && !((used >> q) & 1)) {
                            target[i] = q;
                            used |= bit(q);
                            break;
                        }
                    }
                }
                for (size_t i = 0; i < lows.size(); ++i)
                    if (target[i] >= 0) std::swap(l[lows[i]], l[at(target[i])]);
            });
        } else {
            permute_tile(pass, T, cbits, phys, lg, restore_in);
        }
    }
    // Plain permuting passes until every qubit is on its own bit: each takes whole runs along
    // the cycles of the layout (the bit of a qubit, then the bit of the qubit that sits on
    // that qubit's own bit, ...), then the low bits, then the lowest others.
    for (int guard = 0; !identity(); ++guard) {
        if (guard > 2 * n) {
            P.valid = false;
            return P;
        }
        HostPass pass;
        pass.phys = phys;
        uint64_t S = 0;
        std::vector<char> seen(n, 0);
        for (int p0 = 0; p0 < n && popc(S) < tq; ++p0) {
            if (lg[p0] == p0 || seen[p0]) continue;
            std::vector<int> cyc;
            for (int p = p0; !seen[p]; p = lg[p]) {
                seen[p] = 1;
                cyc.push_back(p);
            }
            const int room = tq - popc(S);
            if ((int)cyc.size() <= room || S == 0)
                for (int j = 0; j < (int)cyc.size() && j < room; ++j) S |= bit(cyc[j]);
        }
        for (int p = 0; p < L && popc(S) < tq; ++p) S |= bit(p);
        for (int p = 0; p < n && popc(S) < tq; ++p) S |= bit(p);
        uint64_t T = 0;  // the qubits on those bits
        for (int p = 0; p < n; ++p)
            if ((S >> p) & 1) T |= bit(lg[p]);
        permute_tile(pass, T, cbits, phys, lg, restore_in);
        P.passes.push_back(pass);
        tiles.push_back(T);
        taken.emplace_back();
    }

    // Register groups, on the tile bits of each pass's layout.
    for (size_t k = 0; k < P.passes.size(); ++k) {
        HostPass& pass = P.passes[k];
        if (pass.standalone >= 0) continue;
        std::vector<int> ph(n);
        for (int q = 0; q < n; ++q) ph[q] = pass.phys.empty() ? q : pass.phys[q];
        uint64_t TP = 0;  // tile index bits
        for (int p : pass.tile_qubits) TP |= bit(p);
        auto tile_bit = [&](int q) {
            int r = 0;
            for (int j = 0; j < ph[q]; ++j) r += (TP >> j) & 1;
            return cbits + r;
        };
        auto in_tile = [&](int q) { return ((TP >> ph[q]) & 1) != 0; };
        std::vector<int> prem = taken[k];
        while (!prem.empty()) {
            HostGroup grp;
            uint64_t R = 0, gblocked = 0, gblocked_t = 0;
            std::vector<int> gsel, grest;
            bool lds_first = circ->gates[P.ops[prem[0]].gate].k > 1;
            if (lds_first && dense_ok) {
                // Dense block on a register group: its targets, its controls inside the tile
                // while they fit (they are folded into the matrix), then padding bits.
                const HostOp& op = P.ops[prem[0]];
                const GateRec& gr = circ->gates[op.gate];
                grp.dense = true;
                grp.ops.push_back(prem[0]);
                for (int j = 0; j < gr.k; ++j) R |= bit(tile_bit(gr.locs[j]));
                for (int m = 0; m < gr.nctrl; ++m) {
                    const int q = gr.ctrls[m];
                    if (in_tile(q) && popc(R | bit(tile_bit(q))) <= reg_bits) R |= bit(tile_bit(q));
                }
                for (int b = t - 1; b >= cbits && popc(R) < reg_bits; --b) R |= bit(b);
                grp.rbits = R;
                prem.erase(prem.begin());
                pass.groups.push_back(grp);
                continue;
            }
            if (lds_first) {
                grp.lds = true;
                grp.ops.push_back(prem[0]);
                const GateRec& gr = circ->gates[P.ops[prem[0]].gate];
                for (int j = 0; j < gr.k; ++j) R |= bit(tile_bit(gr.locs[j]));
                grp.rbits = R;
                prem.erase(prem.begin());
                pass.groups.push_back(grp);
                continue;
            }
            int nslot = 0;
            for (int oi : prem) {
                const HostOp& op = P.ops[oi];
                const GateRec& gr = circ->gates[op.gate];
                const int k1 = gr.k;
                const bool grad = reverse && is_param_kind(gr.kind) && gr.param >= 0;
                uint64_t rb = 0;
                for (int j = 0; j < k1; ++j) rb |= bit(tile_bit(gr.locs[j]));
                if ((op.tmask & gblocked) || (op.qmask & gblocked_t) || k1 > 1 || (grad && nslot >= max_slots)) {
                    gblocked |= op.qmask;
                    gblocked_t |= op.tmask;
                    grest.push_back(oi);
                    continue;
                }
                if (popc(R | rb) <= reg_bits) {
                    R |= rb;
                    gsel.push_back(oi);
                    nslot += grad ? 1 : 0;
                } else {
                    gblocked |= op.qmask;
                    gblocked_t |= op.tmask;
                    grest.push_back(oi);
                }
            }
            // Fill the register bits with the highest unused tile bits, which keeps the thread
            // bits on the low (contiguous) end of the tile.
            for (int b = t - 1; b >= cbits && popc(R) < reg_bits; --b) R |= bit(b);
            grp.rbits = R;
            grp.ops = gsel;
            pass.groups.push_back(grp);
            prem = grest;
        }
    }
    return P;
}

}  // namespace yao
