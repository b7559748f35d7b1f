// Host fusion of runs of gates into dense blocks of up to `width` qubits (forward sweeps only:
// a fused block has no per-parameter gradient).
//
// Gates are taken in order. Open blocks act on disjoint qubit sets, so they commute with each
// other; a gate whose qubits (targets and controls) fit in `width` qubits together with every
// open block it meets is multiplied into the union of those blocks (a chain is the matrix
// product in reverse order, Sec. "Representing Quantum Circuits"); a gate that meets no block
// opens one; any other gate first closes (emits) every block it meets. Products are formed in
// FP64.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "driver.h"

namespace yao {

namespace {

struct Block {
    std::vector<int> qubits;  // ascending; bit j of the matrix index <-> qubits[j]
    HostMat M;
};

int position(const std::vector<int>& qs, int q)
{
    for (size_t j = 0; j < qs.size(); ++j)
        if (qs[j] == q) return (int)j;
    return -1;
}

// Widen a block to the qubit set `qs` (a superset), as M (x) identity on the new qubits.
void widen(Block& b, const std::vector<int>& qs)
{
    const int k = (int)qs.size();
    HostMat W;
    W.resize(k);
    std::vector<int> map(b.qubits.size());
    for (size_t j = 0; j < b.qubits.size(); ++j) map[j] = position(qs, b.qubits[j]);
    uint64_t oldmask = 0;
    for (int p : map) oldmask |= uint64_t(1) << p;
    const int dn = 1 << k, dold = b.M.dim();
    for (int r = 0; r < dn; ++r)
        for (int c = 0; c < dn; ++c) {
            if ((r & ~oldmask) != (c & ~oldmask)) continue;
            int ro = 0, co = 0;
            for (size_t j = 0; j < map.size(); ++j) {
                ro |= ((r >> map[j]) & 1) << j;
                co |= ((c >> map[j]) & 1) << j;
            }
            W.re[(size_t)r * dn + c] = b.M.re[(size_t)ro * dold + co];
            W.im[(size_t)r * dn + c] = b.M.im[(size_t)ro * dold + co];
        }
    b.qubits = qs;
    b.M = W;
}

// Full operator of gate g (matrix U on its targets, identity where its controls fail) on
// the block's qubit set.
HostMat embed(const GateRec& g, const HostMat& U, const std::vector<int>& qs)
{
    const int k = (int)qs.size(), dn = 1 << k;
    HostMat F;
    F.resize(k);
    int tp[8], cp[8];
    for (int j = 0; j < g.k; ++j) tp[j] = position(qs, g.locs[j]);
    for (int m = 0; m < g.nctrl; ++m) cp[m] = position(qs, g.ctrls[m]);
    const int du = U.dim();
    for (int c = 0; c < dn; ++c) {
        bool pass = true;
        for (int m = 0; m < g.nctrl; ++m) pass &= ((c >> cp[m]) & 1) == g.cvals[m];
        if (!pass) {
            F.re[(size_t)c * dn + c] = 1.0;
            continue;
        }
        int sin = 0, clear = c;
        for (int j = 0; j < g.k; ++j) {
            sin |= ((c >> tp[j]) & 1) << j;
            clear &= ~(1 << tp[j]);
        }
        for (int sout = 0; sout < du; ++sout) {
            int r = clear;
            for (int j = 0; j < g.k; ++j) r |= ((sout >> j) & 1) << tp[j];
            F.re[(size_t)r * dn + c] += U.re[(size_t)sout * du + sin];
            F.im[(size_t)r * dn + c] += U.im[(size_t)sout * du + sin];
        }
    }
    return F;
}

GateRec dense_rec(const Block& b)
{
    GateRec r;
    r.kind = YAO_DENSE;
    r.param = -1;
    r.theta = 0;
    r.k = (int)b.qubits.size();
    for (int j = 0; j < r.k; ++j) r.locs[j] = b.qubits[j];
    r.nctrl = 0;
    r.G.resize(size_t(2) << (2 * r.k));
    for (size_t t = 0; t < b.M.re.size(); ++t) {
        r.G[2 * t] = b.M.re[t];
        r.G[2 * t + 1] = b.M.im[t];
    }
    return r;
}

std::vector<int> qubits_of(const GateRec& g)
{
    std::vector<int> q;
    for (int j = 0; j < g.k; ++j) q.push_back(g.locs[j]);
    for (int m = 0; m < g.nctrl; ++m) q.push_back(g.ctrls[m]);
    return q;
}

std::vector<int> merged(const std::vector<int>& a, const std::vector<int>& b)
{
    std::vector<int> m = a;
    for (int q : b)
        if (position(m, q) < 0) m.push_back(q);
    std::sort(m.begin(), m.end());
    return m;
}

bool meets(const std::vector<int>& a, const std::vector<int>& b)
{
    for (int q : b)
        if (position(a, q) >= 0) return true;
    return false;
}

struct Shadow {
    yao_circuit circ;
};

std::map<std::tuple<const yao_circuit*, uint64_t, int>, Shadow*> g_shadows;
std::mutex g_shadow_mu;

}  // namespace

std::vector<GateRec> fuse_gates(const yao_circuit* c, const double* params, int width)
{
    std::vector<GateRec> out;
    std::vector<Block> open;
    auto close_meeting = [&](const std::vector<int>& q) {
        for (size_t b = 0; b < open.size();) {
            if (meets(open[b].qubits, q)) {
                out.push_back(dense_rec(open[b]));
                open.erase(open.begin() + b);
            } else {
                ++b;
            }
        }
    };
    for (const GateRec& g : c->gates) {
        const std::vector<int> q = qubits_of(g);
        HostMat U;
        gate_matrix(g, gate_theta(g, params), U);
        std::vector<int> hits;
        std::vector<int> qs = merged({}, q);
        for (size_t b = 0; b < open.size(); ++b)
            if (meets(open[b].qubits, q)) {
                hits.push_back((int)b);
                qs = merged(qs, open[b].qubits);
            }
        if (!hits.empty() && (int)qs.size() <= width) {
            // The blocks it meets act on disjoint qubits, so they commute: their product on the
            // union is the product of the widened blocks, in any order.
            Block nb;
            nb.qubits = qs;
            nb.M.resize((int)qs.size());
            for (int d = 0; d < nb.M.dim(); ++d) nb.M.re[(size_t)d * nb.M.dim() + d] = 1.0;
            for (int h : hits) {
                Block w = open[h];
                widen(w, qs);
                nb.M = matmul(w.M, nb.M);
            }
            nb.M = matmul(embed(g, U, nb.qubits), nb.M);
            for (int i = (int)hits.size() - 1; i >= 0; --i) open.erase(open.begin() + hits[i]);
            open.push_back(nb);
            continue;
        }
        close_meeting(q);
        if ((int)q.size() <= width) {
            Block b;
            b.qubits = merged({}, q);
            b.M = embed(g, U, b.qubits);
            open.push_back(b);
        } else {
            // Kept as it is, with its angle fixed: the fused circuit takes no parameters.
            GateRec fixed = g;
            fixed.theta = gate_theta(g, params);
            fixed.param = -1;
            out.push_back(fixed);
        }
    }
    for (const Block& b : open) out.push_back(dense_rec(b));
    return out;
}

// A circuit holding the fused gates of c; its structure (and so its cached pass plans) is
// reused while c is unchanged, its matrices are refreshed on every call.
const yao_circuit* fused_circuit(const yao_circuit* c, const double* params, int width)
{
    std::vector<GateRec> gates = fuse_gates(c, params, width);
    std::lock_guard<std::mutex> lk(g_shadow_mu);
    auto key = std::make_tuple(c, c->version, width);
    auto it = g_shadows.find(key);
    Shadow* sh;
    if (it == g_shadows.end()) {
        sh = new Shadow;
        sh->circ.n = c->n;
        sh->circ.nparams = 0;
        sh->circ.version = 1;
        g_shadows[key] = sh;
    } else {
        sh = it->second;
    }
    bool same = sh->circ.gates.size() == gates.size();
    for (size_t t = 0; same && t < gates.size(); ++t) {
        const GateRec &a = sh->circ.gates[t], &b = gates[t];
        same = a.kind == b.kind && a.k == b.k && a.nctrl == b.nctrl &&
               std::equal(a.locs, a.locs + a.k, b.locs) && std::equal(a.ctrls, a.ctrls + a.nctrl, b.ctrls) &&
               std::equal(a.cvals, a.cvals + a.nctrl, b.cvals);
    }
    if (!same) sh->circ.version++;
    sh->circ.gates = std::move(gates);
    return &sh->circ;
}

void drop_fused(const yao_circuit* c)
{
    std::lock_guard<std::mutex> lk(g_shadow_mu);
    for (auto it = g_shadows.begin(); it != g_shadows.end();) {
        if (std::get<0>(it->first) == c) {
            drop_plans(&it->second->circ);
            delete it->second;
            it = g_shadows.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace yao
