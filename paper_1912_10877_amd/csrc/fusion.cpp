// Host fusion of runs of gates into dense blocks of up to `width` qubits (forward sweeps only:
// a fused block has no per-parameter gradient).
//
// Gates are taken in order. Open blocks act on disjoint qubit sets, so they commute with each
// other; a gate whose qubits (targets and controls) fit in `width` qubits together with every
// open block it meets joins the union of those blocks; a gate that meets no block opens one;
// any other gate first closes (emits) every block it meets. A block's matrix is the product of
// its gates in order (a chain is the matrix product in reverse order, Sec. "Representing
// Quantum Circuits"), formed in FP64 by applying each gate to the columns of the block matrix.
//
// The partition depends only on the circuit's structure and is kept per circuit and width;
// each call only recomputes the block matrices for its parameters.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "driver.h"

namespace yao {

namespace {

int position(const std::vector<int>& qs, int q)
{
    for (size_t j = 0; j < qs.size(); ++j)
        if (qs[j] == q) return (int)j;
    return -1;
}

std::vector<int> qubits_of(const GateRec& g)
{
    std::vector<int> q;
    for (int j = 0; j < g.k; ++j) q.push_back(g.locs[j]);
    for (int m = 0; m < g.nctrl; ++m) q.push_back(g.ctrls[m]);
    std::sort(q.begin(), q.end());
    return q;
}

bool meets(const std::vector<int>& a, const std::vector<int>& b)
{
    for (int q : b)
        if (position(a, q) >= 0) return true;
    return false;
}

std::vector<int> merged(const std::vector<int>& a, const std::vector<int>& b)
{
    std::vector<int> m = a;
    for (int q : b)
        if (position(m, q) < 0) m.push_back(q);
    std::sort(m.begin(), m.end());
    return m;
}

std::vector<FusedPart> partition(const yao_circuit* c, int width)
{
    std::vector<FusedPart> out, open;
    auto close_meeting = [&](const std::vector<int>& q) {
        for (size_t b = 0; b < open.size();) {
            if (meets(open[b].qubits, q)) {
                out.push_back(open[b]);
                open.erase(open.begin() + b);
            } else {
                ++b;
            }
        }
    };
    for (int gi = 0; gi < (int)c->gates.size(); ++gi) {
        const std::vector<int> q = qubits_of(c->gates[gi]);
        if ((int)q.size() > width) {
            close_meeting(q);
            FusedPart p;
            p.qubits = q;
            p.gates = {gi};
            p.single = true;
            out.push_back(p);
            continue;
        }
        std::vector<int> hits, qs = q;
        for (size_t b = 0; b < open.size(); ++b)
            if (meets(open[b].qubits, q)) {
                hits.push_back((int)b);
                qs = merged(qs, open[b].qubits);
            }
        if ((int)qs.size() <= width) {
            // The blocks it meets act on disjoint qubits and commute: their gates can follow
            // each other in any order.
            FusedPart nb;
            nb.qubits = qs;
            for (int h : hits) nb.gates.insert(nb.gates.end(), open[h].gates.begin(), open[h].gates.end());
            nb.gates.push_back(gi);
            for (int i = (int)hits.size() - 1; i >= 0; --i) open.erase(open.begin() + hits[i]);
            open.push_back(nb);
        } else {
            close_meeting(q);
            FusedPart nb;
            nb.qubits = q;
            nb.gates = {gi};
            open.push_back(nb);
        }
    }
    for (const FusedPart& b : open) out.push_back(b);
    return out;
}

// M <- (gate g with matrix U, identity where its controls fail) M, on the qubit set qs
// (index bit j <-> qs[j]): every column of M is updated as a state of |qs| qubits.
void apply_left(HostMat& M, const GateRec& g, const HostMat& U, const std::vector<int>& qs)
{
    const int D = M.dim(), du = U.dim();
    int tp[8], cp[kGateMaxCtrl];
    uint32_t tmask = 0, cmask = 0, cval = 0;
    for (int j = 0; j < g.k; ++j) {
        tp[j] = position(qs, g.locs[j]);
        tmask |= 1u << tp[j];
    }
    for (int m = 0; m < g.nctrl; ++m) {
        cp[m] = position(qs, g.ctrls[m]);
        cmask |= 1u << cp[m];
        if (g.cvals[m]) cval |= 1u << cp[m];
    }
    double inr[32], ini[32];
    int idx[32];
    for (int base = 0; base < D; ++base) {
        if (((uint32_t)base & tmask) || ((uint32_t)base & cmask) != cval) continue;
        for (int s = 0; s < du; ++s) {
            int e = base;
            for (int j = 0; j < g.k; ++j) e |= ((s >> j) & 1) << tp[j];
            idx[s] = e;
        }
        for (int col = 0; col < D; ++col) {
            for (int s = 0; s < du; ++s) {
                inr[s] = M.re[(size_t)idx[s] * D + col];
                ini[s] = M.im[(size_t)idx[s] * D + col];
            }
            for (int r = 0; r < du; ++r) {
                double xr = 0, xi = 0;
                for (int s = 0; s < du; ++s) {
                    const double ur = U.re[(size_t)r * du + s], ui = U.im[(size_t)r * du + s];
                    xr += ur * inr[s] - ui * ini[s];
                    xi += ur * ini[s] + ui * inr[s];
                }
                M.re[(size_t)idx[r] * D + col] = xr;
                M.im[(size_t)idx[r] * D + col] = xi;
            }
        }
    }
}

void part_matrix(const yao_circuit* c, const FusedPart& p, const double* params, HostMat& M)
{
    M.resize((int)p.qubits.size());
    for (int d = 0; d < M.dim(); ++d) M.re[(size_t)d * M.dim() + d] = 1.0;
    static thread_local HostMat U;
    for (int gi : p.gates) {
        const GateRec& g = c->gates[gi];
        gate_matrix(g, gate_theta(g, params), U);
        apply_left(M, g, U, p.qubits);
    }
}

GateRec dense_rec(const FusedPart& p)
{
    GateRec r;
    r.kind = YAO_DENSE;
    r.param = -1;
    r.theta = 0;
    r.k = (int)p.qubits.size();
    for (int j = 0; j < r.k; ++j) r.locs[j] = p.qubits[j];
    r.nctrl = 0;
    r.G.assign(size_t(2) << (2 * r.k), 0.0);
    for (int d = 0; d < (1 << r.k); ++d) r.G[2 * ((size_t)d * (1 << r.k) + d)] = 1.0;  // identity until bound
    return r;
}

struct Fused {
    std::vector<FusedPart> parts;
    yao_circuit host;   // gates with their matrices for the last parameters
    yao_circuit shape;  // structure only: multi-gate blocks as identity placeholders, single
                        // gates as they are (parameters kept)
};

std::map<std::tuple<const yao_circuit*, uint64_t, int>, Fused*> g_fused;
std::mutex g_fused_mu;

Fused* get_fused(const yao_circuit* c, int width)
{
    std::lock_guard<std::mutex> lk(g_fused_mu);
    auto key = std::make_tuple(c, c->version, width);
    auto it = g_fused.find(key);
    if (it != g_fused.end()) return it->second;
    Fused* f = new Fused;
    f->parts = partition(c, width);
    for (yao_circuit* x : {&f->host, &f->shape}) {
        x->n = c->n;
        x->version = 1;
    }
    f->host.nparams = 0;
    f->host.transient = true;
    f->shape.nparams = c->nparams;
    for (const FusedPart& p : f->parts) {
        const GateRec r = p.single ? c->gates[p.gates[0]] : dense_rec(p);
        f->shape.gates.push_back(r);
        f->host.gates.push_back(r);
    }
    g_fused[key] = f;
    return f;
}

}  // namespace

std::vector<GateRec> fuse_gates(const yao_circuit* c, const double* params, int width)
{
    return fused_circuit(c, params, width)->gates;
}

// A circuit holding the fused gates of c with matrices for these parameters; its structure (and
// so its cached pass plans) is reused while c is unchanged.
const yao_circuit* fused_circuit(const yao_circuit* c, const double* params, int width)
{
    Fused* f = get_fused(c, width);
    for (size_t i = 0; i < f->parts.size(); ++i) {
        const FusedPart& p = f->parts[i];
        GateRec& r = f->host.gates[i];
        if (p.single) {
            // Kept as it is, with its angle fixed: the fused circuit takes no parameters.
            r = c->gates[p.gates[0]];
            r.theta = gate_theta(r, params);
            r.param = -1;
            continue;
        }
        static thread_local HostMat M;
        part_matrix(c, p, params, M);
        for (size_t t = 0; t < M.re.size(); ++t) {
            r.G[2 * t] = M.re[t];
            r.G[2 * t + 1] = M.im[t];
        }
    }
    return &f->host;
}

const yao_circuit* fused_shape(const yao_circuit* c, int width, const std::vector<FusedPart>** parts)
{
    Fused* f = get_fused(c, width);
    if (parts) *parts = &f->parts;
    return &f->shape;
}

void drop_fused(const yao_circuit* c)
{
    std::lock_guard<std::mutex> lk(g_fused_mu);
    for (auto it = g_fused.begin(); it != g_fused.end();) {
        if (std::get<0>(it->first) == c) {
            drop_plans(&it->second->host);
            drop_plans(&it->second->shape);
            delete it->second;
            it = g_fused.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace yao
