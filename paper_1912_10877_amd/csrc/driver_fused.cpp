// Fused execution of circuits: plans are cached per circuit and geometry; each call lowers
// the current parameters to one device program (ops, groups, FP64 matrices) and launches one
// kernel per pass.
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "driver.h"
#include "fused.h"
#include "tuner.h"

namespace yao {

int launch_pass(bool bwd, int psi_dtype, int lam_dtype, void* psi, void* lam, const POp* ops, const PGroupDesc* groups,
                const double* mats, double* gpartial, int pstride, int mslots, int n, int B, int c, int t, int group0,
                int ngroups, const std::vector<int>& tile_qubits, const std::vector<int>& store_src, double flops,
                int op_first, int nops,
                const double* dmats, int dm_words);
int launch_fill(double* p, size_t count, double v);

using PlanKey = std::tuple<const yao_circuit*, uint64_t, int, int, int, int, int, int, bool, int, int, int>;
static std::map<PlanKey, Plan> g_plans;
static std::mutex g_plan_mu;

const Plan& get_plan_ex(const yao_circuit* c, int g0, int g1, int B, int t, int cb, int L, bool reverse, int reg_bits,
                        int max_ops, int max_slots)
{
    std::lock_guard<std::mutex> lk(g_plan_mu);
    PlanKey key{c, c->version, g0, g1, B, t, cb, L, reverse, reg_bits, max_ops, max_slots};
    auto it = g_plans.find(key);
    if (it != g_plans.end()) return it->second;
    return g_plans.emplace(key, make_plan(c, g0, g1, B, t, cb, L, reverse, reg_bits, max_ops, max_slots))
        .first->second;
}

const Plan& get_plan(const yao_circuit* c, int g0, int g1, int B, int t, int cb, int L, bool reverse, int lam_bytes)
{
    return get_plan_ex(c, g0, g1, B, t, cb, L, reverse, reverse ? kRegBitsBwd : kRegBitsFwd, kMaxPassOps,
                       reverse ? reverse_slot_limit(t, cb, lam_bytes) : kMaxGroupSlots);
}

int op_type_of(const HostMat& U)
{
    if (U.k != 1) return OT_LDSK;
    const auto& r = U.re;
    const auto& i = U.im;
    if (r[0] == 0 && i[0] == 0 && r[3] == 0 && i[3] == 0 && r[1] == 1 && i[1] == 0 && r[2] == 1 && i[2] == 0)
        return OT_SWAP;
    if (r[1] == 0 && i[1] == 0 && r[2] == 0 && i[2] == 0) return OT_DIAG;
    if (i[0] == 0 && i[1] == 0 && i[2] == 0 && i[3] == 0) return OT_REAL;
    if (i[0] == 0 && i[3] == 0 && r[1] == 0 && r[2] == 0 && r[0] == r[3] && i[1] == i[2]) return OT_RX;
    return OT_DENSE;
}

int gen_type_of(const GateRec& g)
{
    if (g.k != 1) return GEN_DENSE;
    switch (g.kind) {
    case YAO_RX: return GEN_X;
    case YAO_RY: return GEN_Y;
    case YAO_RZ: return GEN_Z;
    case YAO_SHIFT: return GEN_P1;
    default: return GEN_DENSE;
    }
}

// Real flops per state element of one op as the pass kernels execute it (complex multiply = 6,
// complex add = 2). diag_high: a reverse uncontrolled Z-generator diagonal, which multiplies only
// the second element of each pair (d1/d0) and leaves d0 to the pass's running phase.
double op_flops(const POp& op, bool bwd, bool diag_high)
{
    double f;
    switch (op.type) {
    case OT_SWAP: f = 0; break;
    case OT_DIAG: f = diag_high ? 3 : 6; break;
    case OT_REAL: case OT_RX: f = 6; break;
    case OT_LDSK: f = 8.0 * (1 << op.k) - 2.0; break;
    default: f = 14; break;
    }
    if (!bwd) return f;
    double g = 0;
    if (op.slot >= 0) g = op.gen == GEN_DENSE ? 16 : (op.gen == GEN_P1 ? 2 : 4);
    return 2 * f + g;
}

static void append(std::vector<double>& v, const std::vector<double>& a)
{
    v.insert(v.end(), a.begin(), a.end());
}

// One-qubit gate kinds k_bind evaluates from an angle (fixed kinds take none).
static bool bindable_kind(int kind)
{
    return kind == YAO_X || kind == YAO_Y || kind == YAO_Z || kind == YAO_H || kind == YAO_S || kind == YAO_SDAG ||
           kind == YAO_T || kind == YAO_TDAG || kind == YAO_RX || kind == YAO_RY || kind == YAO_RZ ||
           kind == YAO_SHIFT;
}

int build_program(const Plan& P, const yao_circuit* c, const double* params, bool bwd, int dtype, Program& prog,
                  const std::vector<FusedPart>* parts, const yao_circuit* orig)
{
    const int G = (int)c->gates.size();
    const bool bind = params == nullptr;
    // Factors of gate gi of c: the member gates of a fused placeholder, else the gate itself.
    auto placeholder = [&](int gi) { return parts && !(*parts)[gi].single; };
    auto param_dependent = [&](int gi) {
        if (placeholder(gi)) {
            for (int og : (*parts)[gi].gates)
                if (orig->gates[og].param >= 0 && is_param_kind(orig->gates[og].kind)) return true;
            return false;
        }
        return c->gates[gi].param >= 0 && is_param_kind(c->gates[gi].kind);
    };
    // Matrix of gate gi for the host when nothing in it depends on parameters.
    auto fixed_matrix = [&](int gi, HostMat& U) {
        if (!placeholder(gi)) return gate_matrix(c->gates[gi], c->gates[gi].theta, U);
        const FusedPart& fp = (*parts)[gi];
        U.resize((int)fp.qubits.size());
        for (int d = 0; d < U.dim(); ++d) U.re[(size_t)d * U.dim() + d] = 1.0;
        static thread_local HostMat F;
        for (int og : fp.gates) {
            const GateRec& h = orig->gates[og];
            if (!gate_matrix(h, h.theta, F) || h.k != 1 || h.nctrl) return false;
            HostMat T = matmul(F, U);
            U = T;
        }
        return true;
    };
    prog.slot_of_gate.assign(G, -1);
    if (bwd) {
        for (int g = 0; g < G; ++g)
            if (is_param_kind(c->gates[g].kind) && c->gates[g].param >= 0) prog.slot_of_gate[g] = prog.nslots++;
    }
    for (const HostPass& pass : P.passes) {
        prog.pass_group0.push_back((int)prog.groups.size());
        prog.pass_op0.push_back((int)prog.ops.size());
        prog.pass_nops.push_back(0);
        prog.pass_flops.push_back(0.0);
        prog.pass_mat.push_back(-1);
        prog.pass_dmat0.push_back(0);
        prog.pass_dmat_words.push_back(0);
        std::vector<double> dense;  // this pass's dense block matrices, in the order of their ops
        int ndense = 0;
        if (pass.standalone >= 0) {
            // A gate wider than a pass takes: its matrices go to the pool in the form its own
            // launch reads.
            const int gi = P.ops[pass.standalone].gate;
            const GateRec& g = c->gates[gi];
            if (bind && param_dependent(gi)) {
                prog.bindable = false;  // a wide parameterised gate: matrices from the host only
                continue;
            }
            const double th = bind ? g.theta : gate_theta(g, params);
            HostMat U;
            if (!(bind ? fixed_matrix(gi, U) : gate_matrix(g, th, U))) return set_error(YAO_EINVAL, "bad gate %d", gi);
            if (!bwd) {
                prog.pass_mat.back() = (int)encode_gate_matrix(dtype, P.n, P.B, U, prog.mats);
            } else {
                HostMat Ud = dagger(U), M;
                if (prog.slot_of_gate[gi] >= 0) gate_grad_matrix(g, th, M);
                else M.resize(g.k);
                prog.pass_mat.back() = (int)prog.mats.size();
                append(prog.mats, Ud.re);
                append(prog.mats, Ud.im);
                append(prog.mats, M.re);
                append(prog.mats, M.im);
            }
            continue;
        }
        // Tile index bits, and the index bit of each qubit in this pass's layout.
        uint64_t T = 0;
        for (int q : pass.tile_qubits) T |= uint64_t(1) << q;
        auto ph = [&](int q) { return pass.phys.empty() ? q : pass.phys[q]; };
        auto in_tile = [&](int q) { return ((T >> ph(q)) & 1) != 0; };
        auto tile_bit = [&](int q) {
            int r = 0;
            for (int j = 0; j < ph(q); ++j) r += (T >> j) & 1;
            return P.c + r;
        };
        for (const HostGroup& hg : pass.groups) {
            PGroupDesc gd;
            memset(&gd, 0, sizeof(gd));
            int nr = 0;
            for (int b = 0; b < P.t; ++b)
                if ((hg.rbits >> b) & 1) {
                    if (nr < P.reg_bits) gd.rpos[nr] = b;
                    ++nr;
                }
            gd.lds = hg.dense ? 2 : (hg.lds ? 1 : 0);
            gd.op0 = (int)prog.ops.size() - prog.pass_op0.back();
            prog.pass_nops.back() += (int)hg.ops.size();
            gd.nops = (int)hg.ops.size();
            gd.nslot = 0;
            for (int oi : hg.ops) {
                const HostOp& hop = P.ops[oi];
                const GateRec& g = c->gates[hop.gate];
                static thread_local HostMat U, Ud, M;  // reused across ops and calls
                const bool pdep = bind && param_dependent(hop.gate);
                double th = 0;
                if (!bind) {
                    th = gate_theta(g, params);
                    if (!gate_matrix(g, th, U)) return set_error(YAO_EINVAL, "bad gate %d", hop.gate);
                } else if (!pdep) {
                    th = g.theta;
                    if (!fixed_matrix(hop.gate, U)) return set_error(YAO_EINVAL, "bad gate %d", hop.gate);
                } else {
                    // Placeholder values: the matrix is written on the device by k_bind.
                    if (g.k != 1 || hg.dense) prog.bindable = false;
                    U.resize(g.k);
                    for (int d = 0; d < U.dim(); ++d) U.re[(size_t)d * U.dim() + d] = 1.0;
                }
                POp op;
                memset(&op, 0, sizeof(op));
                op.k = g.k;
                op.slot = bwd ? prog.slot_of_gate[hop.gate] : -1;
                op.mat = (int)prog.mats.size();
                if (!bwd) {
                    op.type = op_type_of(U);
                    op.gen = GEN_NONE;
                    append(prog.mats, U.re);
                    append(prog.mats, U.im);
                } else {
                    dagger_into(U, Ud);
                    op.type = op_type_of(Ud);
                    append(prog.mats, Ud.re);
                    append(prog.mats, Ud.im);
                    if (op.slot >= 0) {
                        gate_grad_matrix(g, th, M);
                        op.gen = gen_type_of(g);
                        if (gd.nslot >= std::min(kMaxGroupSlots, P.max_slots))
                            return set_error(YAO_EINVAL, "register group carries more than %d gradients",
                                             std::min(kMaxGroupSlots, P.max_slots));
                        gd.slots[gd.nslot++] = op.slot;
                    } else {
                        M.resize(g.k);
                        op.gen = GEN_NONE;
                    }
                    append(prog.mats, M.re);
                    append(prog.mats, M.im);
                }
                if (g.k > 1) op.type = OT_LDSK;
                if (hg.dense) {
                    // The gate as a 16 x 16 matrix on the group's register bits (index bit j <->
                    // tile bit gd.rpos[j]) with its controls on those bits folded in, stored in
                    // the state's precision: rows of re[16] then im[16].
                    int tp[kMaxDenseK], cpos[kGateMaxCtrl];
                    for (int j = 0; j < g.k; ++j) {
                        tp[j] = -1;
                        for (int r = 0; r < kRegBitsFwd; ++r)
                            if (gd.rpos[r] == tile_bit(g.locs[j])) tp[j] = r;
                        if (tp[j] < 0) return set_error(YAO_EINVAL, "dense block target outside its register bits");
                    }
                    for (int m = 0; m < g.nctrl; ++m) {
                        cpos[m] = -1;
                        if (in_tile(g.ctrls[m]))
                            for (int r = 0; r < kRegBitsFwd; ++r)
                                if (gd.rpos[r] == tile_bit(g.ctrls[m])) cpos[m] = r;
                    }
                    const int D = 1 << kRegBitsFwd, du = 1 << g.k;
                    std::vector<double> Fr((size_t)D * D, 0.0), Fi((size_t)D * D, 0.0);
                    for (int c = 0; c < D; ++c) {
                        bool pass_ok = true;
                        for (int m = 0; m < g.nctrl; ++m)
                            if (cpos[m] >= 0) pass_ok &= ((c >> cpos[m]) & 1) == g.cvals[m];
                        if (!pass_ok) {
                            Fr[(size_t)c * D + c] = 1.0;
                            continue;
                        }
                        int sin = 0, clear = c;
                        for (int j = 0; j < g.k; ++j) {
                            sin |= ((c >> tp[j]) & 1) << j;
                            clear &= ~(1 << tp[j]);
                        }
                        for (int so = 0; so < du; ++so) {
                            int r = clear;
                            for (int j = 0; j < g.k; ++j) r |= ((so >> j) & 1) << tp[j];
                            Fr[(size_t)r * D + c] += U.re[(size_t)so * du + sin];
                            Fi[(size_t)r * D + c] += U.im[(size_t)so * du + sin];
                        }
                    }
                    // op.mat is the block's ordinal among the pass's dense blocks. Complex64
                    // passes run the block on the FP32 matrix cores and take it row-major
                    // (16 x 16 complex); complex128 passes take it column-major: column c
                    // holds re[16] then im[16].
                    op.mat = ndense++;
                    if (dtype == YAO_C64) {
                        const size_t at = dense.size();
                        dense.resize(at + (size_t)D * D);  // 2 D^2 floats
                        float* f = (float*)(dense.data() + at);
                        for (int r = 0; r < D; ++r)
                            for (int c = 0; c < D; ++c) {
                                f[2 * (r * D + c)] = (float)Fr[(size_t)r * D + c];
                                f[2 * (r * D + c) + 1] = (float)Fi[(size_t)r * D + c];
                            }
                    } else {
                        for (int c = 0; c < D; ++c) {
                            for (int r = 0; r < D; ++r) dense.push_back(Fr[(size_t)r * D + c]);
                            for (int r = 0; r < D; ++r) dense.push_back(Fi[(size_t)r * D + c]);
                        }
                    }
                }
                if (pdep && g.k == 1) {
                    // Factors for k_bind, and the structure class the bound matrix will have.
                    BindRec br;
                    br.op = (int)prog.ops.size();
                    br.f0 = (int)prog.facs.size();
                    br.mode = bwd ? 2 : (dtype == YAO_C64 ? 0 : 1);
                    if (placeholder(hop.gate)) {
                        for (int og : (*parts)[hop.gate].gates) {
                            const GateRec& h = orig->gates[og];
                            prog.facs.push_back(BindFac{h.kind, is_param_kind(h.kind) ? h.param : -1, h.theta});
                        }
                    } else {
                        prog.facs.push_back(BindFac{g.kind, g.param, g.theta});
                    }
                    br.nf = (int)prog.facs.size() - br.f0;
                    for (int f = br.f0; f < br.f0 + br.nf; ++f) prog.bindable &= bindable_kind(prog.facs[f].kind);
                    prog.binds.push_back(br);
                    const int k1 = prog.facs[br.f0].kind;
                    op.type = br.nf > 1 ? OT_DENSE
                                        : (k1 == YAO_RX ? OT_RX : (k1 == YAO_RY ? OT_REAL : (k1 == YAO_RZ || k1 == YAO_SHIFT ? OT_DIAG : OT_DENSE)));
                }
                if (g.k == 1) {
                    // The forward kernel of complex64 states reads the 2x2 matrix as float[8].
                    if (!bwd && dtype == YAO_C64) {
                        float* f = (float*)op.u;
                        for (int e = 0; e < 8; ++e) f[e] = (float)prog.mats[op.mat + e];
                    } else {
                        for (int e = 0; e < 8; ++e) op.u[e] = prog.mats[op.mat + e];
                    }
                }
                for (int j = 0; j < g.k && j < 3; ++j) op.tpos[j] = tile_bit(g.locs[j]);
                op.rpos = 0;
                if (!hg.lds) {
                    for (int j = 0; j < P.reg_bits; ++j)
                        if (gd.rpos[j] == op.tpos[0]) op.rpos = j;
                }
                bool diag_high = false;
                for (int m = 0; m < g.nctrl; ++m) {
                    const int q = g.ctrls[m];
                    bool folded = false;  // a control on a dense block's register bit is in its matrix
                    if (hg.dense && in_tile(q))
                        for (int r = 0; r < kRegBitsFwd; ++r) folded |= gd.rpos[r] == tile_bit(q);
                    if (folded) continue;
                    if (in_tile(q)) {
                        op.cmask |= 1u << tile_bit(q);
                        if (g.cvals[m]) op.cval |= 1u << tile_bit(q);
                    } else {
                        op.omask |= uint64_t(1) << ph(q);
                        if (g.cvals[m]) op.oval |= uint64_t(1) << ph(q);
                    }
                }
                {
                    const bool plain = op.cmask == 0 && op.omask == 0;
                    const bool cswap = op.type == OT_SWAP && op.cmask != 0 && op.omask == 0;
                    int cls;
                    if (!bwd) {
                        cls = (plain && op.type == OT_RX)     ? 0
                              : (plain && op.type == OT_DIAG)  ? 1
                              : (plain && op.type == OT_DENSE) ? 2
                              : cswap                          ? 3
                                                               : kFwdGenericClass;
                    } else {
                        cls = (plain && op.slot >= 0 && op.type == OT_RX && op.gen == GEN_X)     ? 0
                              : (plain && op.slot >= 0 && op.type == OT_DIAG && op.gen == GEN_Z) ? 1
                              : (cswap && op.slot < 0)                                           ? 2
                                                                                                 : kBwdGenericClass;
                    }
                    op.var = g.k == 1 ? cls * P.reg_bits + op.rpos : 0;
                    // The reverse Z-generator diagonal class leaves d0 to a phase of the tile.
                    diag_high = bwd && g.k == 1 && cls == 1;
                    if (diag_high && !pdep) split_diag_phase(op.u);
                }
                prog.ops.push_back(op);
                prog.pass_flops.back() += op_flops(op, bwd, diag_high) / double(uint64_t(1) << g.nctrl);
            }
            prog.groups.push_back(gd);
        }
        if (ndense > kMaxPassDense) return set_error(YAO_EINVAL, "pass holds %d dense blocks", ndense);
        if (!dense.empty()) {
            prog.mats.resize((prog.mats.size() + 1) & ~size_t(1));  // 16-byte words
            prog.pass_dmat0.back() = (int)prog.mats.size();
            prog.pass_dmat_words.back() = (int)(dense.size() / 2);
            prog.mats.insert(prog.mats.end(), dense.begin(), dense.end());
        }
    }
    return 0;
}

static size_t al256(size_t v)
{
    return (v + 255) & ~size_t(255);
}

size_t program_blob_bytes(const Program& prog)
{
    return al256(prog.ops.size() * sizeof(POp)) + al256(prog.groups.size() * sizeof(PGroupDesc)) +
           al256(prog.mats.size() * sizeof(double)) + 256;
}

// Lay the program out at host (to be copied to dev); d receives the device addresses.
void pack_program(const Program& prog, char* host, char* dev, DevProgram& d)
{
    const size_t so = prog.ops.size() * sizeof(POp);
    const size_t sg = prog.groups.size() * sizeof(PGroupDesc);
    const size_t sm = prog.mats.size() * sizeof(double);
    memset(host, 0, program_blob_bytes(prog));
    if (so) memcpy(host, prog.ops.data(), so);
    if (sg) memcpy(host + al256(so), prog.groups.data(), sg);
    if (sm) memcpy(host + al256(so) + al256(sg), prog.mats.data(), sm);
    d.ops = (POp*)dev;
    d.groups = (PGroupDesc*)(dev + al256(so));
    d.mats = (double*)(dev + al256(so) + al256(sg));
}

// Pack a program into the slot's pinned buffer and queue its copy to the slot's device
// buffer; the host returns at once. The caller synchronises the stream before the slot is
// packed again.
static hipEvent_t g_copied[WS_COUNT] = {};

static int upload_program(const Program& prog, DevProgram& d, int slot = WS_MAT)
{
    // The previous copy out of this slot's pinned buffer has to be done before it is reused.
    if (!g_copied[slot]) YAO_HIP(hipEventCreateWithFlags(&g_copied[slot], hipEventDisableTiming));
    else YAO_HIP(hipEventSynchronize(g_copied[slot]));
    const size_t bytes = program_blob_bytes(prog);
    char* dev = (char*)workspace(slot, bytes);
    if (!dev) return YAO_ENOMEM;
    char* host = (char*)pinned(slot, bytes);
    if (!host) return YAO_ENOMEM;
    pack_program(prog, host, dev, d);
    YAO_HIP(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, stream()));
    YAO_HIP(hipEventRecord(g_copied[slot], stream()));
    return 0;
}

// A standalone gate's targets and controls on the index bits of the pass's layout.
static void layout_qubits(const HostPass& pass, const GateRec& g, int* locs, int* ctrls)
{
    auto ph = [&](int q) { return pass.phys.empty() ? q : pass.phys[q]; };
    for (int j = 0; j < g.k; ++j) locs[j] = ph(g.locs[j]);
    for (int m = 0; m < g.nctrl; ++m) ctrls[m] = ph(g.ctrls[m]);
}

int launch_forward_passes(const Plan& P, const Program& prog, const DevProgram& d, void* data, int dtype, int n, int B,
                          const yao_circuit* c, const double* params, const BoundProgram* bp)
{
    if (!P.valid) return set_error(YAO_EINVAL, "pass plan could not restore the qubit layout");
    const JitPasses* J = bp && &bp->prog == &prog ? jit_passes(bp, P, false, dtype, n, B) : nullptr;
    for (size_t p = 0; p < P.passes.size(); ++p) {
        const HostPass& pass = P.passes[p];
        if (jit_has(J, (int)p)) {
            const double N = (double)(uint64_t(1) << n) * B;
            YAO_TRY(jit_launch_forward(J, (int)p, data, d.ops, prog.pass_op0[p], 2.0 * N * (dtype == YAO_C64 ? 8 : 16),
                                       prog.pass_flops[p] * N));
            continue;
        }
        if (pass.standalone >= 0) {
            // The matrix is read from the program; the launch takes only its size from U.
            const GateRec& g = c->gates[P.ops[pass.standalone].gate];
            HostMat U;
            U.k = g.k;
            int locs[8], ctrls[kGateMaxCtrl];
            layout_qubits(pass, g, locs, ctrls);
            YAO_TRY(launch_gate(data, dtype, n, B, U, locs, make_ctrl(g.nctrl, ctrls, g.cvals),
                                d.mats + prog.pass_mat[p]));
            continue;
        }
        YAO_TRY(launch_pass(false, dtype, dtype, data, nullptr, d.ops, d.groups, d.mats, nullptr, 0, 0, n, B, P.c, P.t,
                            prog.pass_group0[p], (int)pass.groups.size(), pass.tile_qubits, pass.store_src,
                            prog.pass_flops[p] * (double)(uint64_t(1) << n) * B, prog.pass_op0[p],
                            prog.pass_nops[p], d.mats + prog.pass_dmat0[p], prog.pass_dmat_words[p]));
    }
    return 0;
}

int launch_backward_passes(const Plan& P, const Program& prog, const DevProgram& d, const yao_circuit* c,
                           const double* params, double* psi, void* lam, int lam_dtype, int n, int B, double* gpartial,
                           int W, const BoundProgram* bp)
{
    if (!P.valid) return set_error(YAO_EINVAL, "pass plan could not restore the qubit layout");
    const JitPasses* J = bp && &bp->prog == &prog ? jit_passes(bp, P, true, lam_dtype, n, B) : nullptr;
    for (size_t p = 0; p < P.passes.size(); ++p) {
        const HostPass& pass = P.passes[p];
        if (jit_has(J, (int)p)) {
            const double N = (double)(uint64_t(1) << n) * B;
            YAO_TRY(jit_launch_backward(J, (int)p, psi, lam, d.ops, prog.pass_op0[p], d.mats, gpartial, W,
                                        2.0 * N * (16 + (lam_dtype == YAO_C64 ? 8 : 16)), prog.pass_flops[p] * N));
            continue;
        }
        if (pass.standalone >= 0) {
            // Matrices come from the program; the launch takes only their size from Ud and M.
            const int gi = P.ops[pass.standalone].gate;
            const GateRec& g = c->gates[gi];
            HostMat Ud, M;
            Ud.k = M.k = g.k;
            const int slot = prog.slot_of_gate[gi];
            int locs[8], ctrls[kGateMaxCtrl];
            layout_qubits(pass, g, locs, ctrls);
            YAO_TRY(launch_adjoint_step_strided(psi, lam, lam_dtype, n, B, Ud, slot >= 0 ? &M : nullptr, locs,
                                                make_ctrl(g.nctrl, ctrls, g.cvals), d.mats + prog.pass_mat[p],
                                                slot >= 0 ? gpartial + (size_t)slot * B * W : nullptr, W));
            continue;
        }
        YAO_TRY(launch_pass(true, YAO_C128, lam_dtype, psi, lam, d.ops, d.groups, d.mats, gpartial, W, P.max_slots, n,
                            B, P.c, P.t,
                            prog.pass_group0[p], (int)pass.groups.size(), pass.tile_qubits, pass.store_src,
                            prog.pass_flops[p] * (double)(uint64_t(1) << n) * B, prog.pass_op0[p],
                            prog.pass_nops[p], nullptr, 0));
    }
    return 0;
}

// ---------------------------------------------------------------------- device-bound programs
// A plan's program built once without parameters and kept in device memory; each call only
// copies the parameters and runs k_bind over the parameter-dependent matrices.
static std::map<std::tuple<const Plan*, bool, int>, BoundProgram*> g_bound;
static std::mutex g_bound_mu;

static void free_bound(BoundProgram* b)
{
    jit_free(b->jit);
    if (b->dev) (void)hipFree(b->dev);
    if (b->dbinds) (void)hipFree(b->dbinds);
    if (b->dfacs) (void)hipFree(b->dfacs);
    delete b;
}

void drop_bound(const yao_circuit* c)
{
    std::lock_guard<std::mutex> lk(g_bound_mu);
    for (auto it = g_bound.begin(); it != g_bound.end();) {
        if (it->second->circ == c) {
            (void)hipDeviceSynchronize();
            free_bound(it->second);
            it = g_bound.erase(it);
        } else {
            ++it;
        }
    }
}

// The bound program of plan P over circuit c (with parts/orig for a fused structure), or
// nullptr when it cannot be bound on the device. Built and copied on first use.
const BoundProgram* bound_program(const Plan& P, const yao_circuit* c, bool bwd, int dtype,
                                  const std::vector<FusedPart>* parts, const yao_circuit* orig)
{
    std::lock_guard<std::mutex> lk(g_bound_mu);
    const auto key = std::make_tuple(&P, bwd, dtype);
    auto it = g_bound.find(key);
    if (it != g_bound.end()) return it->second->ok ? it->second : nullptr;
    BoundProgram* b = new BoundProgram;
    b->circ = orig ? orig : c;
    g_bound[key] = b;
    if (build_program(P, c, nullptr, bwd, dtype, b->prog, parts, orig) != 0 || !b->prog.bindable) return nullptr;
    const size_t bytes = program_blob_bytes(b->prog);
    std::vector<char> host(bytes);
    const size_t nb = std::max<size_t>(1, b->prog.binds.size()), nf = std::max<size_t>(1, b->prog.facs.size());
    if (hipMalloc((void**)&b->dev, bytes) != hipSuccess || hipMalloc((void**)&b->dbinds, nb * sizeof(BindRec)) != hipSuccess ||
        hipMalloc((void**)&b->dfacs, nf * sizeof(BindFac)) != hipSuccess) {
        set_error(YAO_ENOMEM, "bound program of %zu bytes", bytes);
        return nullptr;
    }
    pack_program(b->prog, host.data(), b->dev, b->d);
    if (hipMemcpy(b->dev, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        (!b->prog.binds.empty() && hipMemcpy(b->dbinds, b->prog.binds.data(), b->prog.binds.size() * sizeof(BindRec),
                                             hipMemcpyHostToDevice) != hipSuccess) ||
        (!b->prog.facs.empty() && hipMemcpy(b->dfacs, b->prog.facs.data(), b->prog.facs.size() * sizeof(BindFac),
                                            hipMemcpyHostToDevice) != hipSuccess)) {
        set_error(YAO_EHIP, "copying a bound program");
        return nullptr;
    }
    b->ok = true;
    return b;
}

// Copy the parameters to the device (queued; the pinned buffer is reused only after the copy
// is done). Returns the device array, or nullptr on failure.
const double* upload_params(const double* params, int nparams)
{
    static hipEvent_t done = nullptr;
    if (!done) {
        if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) return nullptr;
    } else if (hipEventSynchronize(done) != hipSuccess) {
        return nullptr;
    }
    const size_t bytes = sizeof(double) * (size_t)std::max(1, nparams);
    double* dev = (double*)workspace(WS_PARAMS, bytes);
    double* host = (double*)pinned(WS_PARAMS, bytes);
    if (!dev || !host) return nullptr;
    if (nparams > 0) {
        memcpy(host, params, sizeof(double) * (size_t)nparams);
        if (hipMemcpyAsync(dev, host, sizeof(double) * (size_t)nparams, hipMemcpyHostToDevice, stream()) != hipSuccess)
            return nullptr;
    }
    if (hipEventRecord(done, stream()) != hipSuccess) return nullptr;
    return dev;
}

int bind_program(const BoundProgram* b, const double* dparams)
{
    return launch_bind(b->d.ops, b->dbinds, (int)b->prog.binds.size(), b->dfacs, dparams);
}

namespace {

int run_forward_plan(const Plan& P, void* data, int dtype, int n, int B, const yao_circuit* c, const double* params)
{
    Program prog;
    YAO_TRY(build_program(P, c, params, false, dtype, prog));
    DevProgram d;
    YAO_TRY(upload_program(prog, d));
    return launch_forward_passes(P, prog, d, data, dtype, n, B, c, params);
}

// Reverse sweep over the gates of one plan: gradient partials into gpartial (row stride W).
int run_backward_plan(const Plan& P, const yao_circuit* c, const double* params, double* psi, void* lam,
                      int lam_dtype, int n, int B, double* gpartial, int W, std::vector<int>* slot_of_gate)
{
    Program prog;
    YAO_TRY(build_program(P, c, params, true, lam_dtype, prog));
    DevProgram d;
    YAO_TRY(upload_program(prog, d));
    if (slot_of_gate) *slot_of_gate = prog.slot_of_gate;
    return launch_backward_passes(P, prog, d, c, params, psi, lam, lam_dtype, n, B, gpartial, W);
}

int count_slots(const yao_circuit* c)
{
    int k = 0;
    for (const GateRec& g : c->gates) k += (is_param_kind(g.kind) && g.param >= 0) ? 1 : 0;
    return k;
}

}  // namespace

int forward_fused_range(void* data, int dtype, int n, int B, const yao_circuit* c, const double* params, int g0, int g1)
{
    if (g1 <= g0) return 0;
    int t, cb, L;
    tile_geometry(n, B, dtype, false, &t, &cb, &L);
    const Plan& P = get_plan(c, g0, g1, B, t, cb, L, false);
    const BoundProgram* bp = c->transient ? nullptr : bound_program(P, c, false, dtype, nullptr, nullptr);
    if (!bp) return run_forward_plan(P, data, dtype, n, B, c, params);
    const double* dp = c->nparams > 0 ? upload_params(params, c->nparams) : nullptr;
    if (c->nparams > 0 && !dp) return YAO_ENOMEM;
    YAO_TRY(bind_program(bp, dp));
    return launch_forward_passes(P, bp->prog, bp->d, data, dtype, n, B, c, params, bp);
}

int forward_fused(void* data, int dtype, int n, int B, const yao_circuit* c, const double* params)
{
    return forward_sweep(data, dtype, n, B, c, params, 0, options().tile_qubits, nullptr);
}

int forward_sweep(void* data, int dtype, int n, int B, const yao_circuit* c, const double* params, int width, int tq,
                  const double* dparams)
{
    if (c->gates.empty()) return 0;
    int t, cb, L;
    tile_geometry_tq(n, B, dtype, false, tq, &t, &cb, &L);
    if (!c->transient) {
        // Bound on the device: the circuit itself (width 0) or the structure of its fused form.
        const std::vector<FusedPart>* parts = nullptr;
        const yao_circuit* sc = width > 0 ? fused_shape(c, width, &parts) : c;
        const Plan& P = get_plan(sc, 0, (int)sc->gates.size(), B, t, cb, L, false);
        const BoundProgram* bp = bound_program(P, sc, false, dtype, parts, width > 0 ? c : nullptr);
        if (bp) {
            if (!dparams && c->nparams > 0) {
                dparams = upload_params(params, c->nparams);
                if (!dparams) return YAO_ENOMEM;
            }
            YAO_TRY(bind_program(bp, dparams));
            return launch_forward_passes(P, bp->prog, bp->d, data, dtype, n, B, sc, nullptr, bp);
        }
    }
    // Host-built program for these parameters (dense fused blocks, or gates the device cannot bind).
    const yao_circuit* hc = width > 0 && !c->transient ? fused_circuit(c, params, width) : c;
    const double* hp = hc == c ? params : nullptr;
    const Plan& P = get_plan(hc, 0, (int)hc->gates.size(), B, t, cb, L, false);
    return run_forward_plan(P, data, dtype, n, B, hc, hp);
}

// Sum the per-tile gradient partials of each gate slot into the caller's layout.
static void gather_gradients(const yao_circuit* c, const std::vector<int>& slot_of_gate, const double* sums, int B,
                             bool reduce_batch, double* grad)
{
    const int P_ = c->nparams;
    const size_t glen = reduce_batch ? (size_t)P_ : (size_t)P_ * B;
    for (size_t e = 0; e < glen; ++e) grad[e] = 0.0;
    for (int gi = (int)c->gates.size() - 1; gi >= 0; --gi) {
        const int slot = slot_of_gate.empty() ? -1 : slot_of_gate[gi];
        if (slot < 0) continue;
        const int p = c->gates[gi].param;
        for (int b = 0; b < B; ++b) {
            const double v = sums[(size_t)slot * B + b];
            if (reduce_batch) grad[p] += v;
            else grad[(size_t)b * P_ + p] += v;
        }
    }
}

// The reversible sweep as one plan. The forward sweep only has to produce the final state, so
// it may fold gates into dense blocks; the reverse program is built on the host while the
// device runs the forward sweep, and nothing waits for the device until the results are read.
static int backward_reversible(yao_state* s, const yao_circuit* c, const double* params, yao_pauli_sum* h,
                               bool reduce_batch, double* energy, double* grad, double* drift, const void* psi0,
                               bool check_drift)
{
    const int n = s->n, B = s->batch;
    const size_t elems = s->elems();
    const int G = (int)c->gates.size();
    hipStream_t st = stream();
    int t, cb, L;
    tile_geometry(n, B, s->dtype, true, &t, &cb, &L);
    const int ntiles = 1 << (n - (t - cb));
    const int W = std::max(ntiles, adjoint_nblk(n, 1, B));
    const int nslots = count_slots(c);
    double* psi = (double*)workspace(WS_PSI64, elems * 16);
    void* lam = workspace(WS_LAM, s->bytes());
    double* gpartial = (double*)workspace(WS_PARTIAL, sizeof(double) * (size_t)std::max(1, nslots) * B * W);
    const size_t hp = hpsi_partial_doubles(h, n, B, s->dtype);
    double* misc = (double*)workspace(WS_MISC, sizeof(double) * (hp + (size_t)B + (size_t)std::max(1, nslots) * B));
    if (!psi || !lam || !gpartial || !misc) return YAO_ENOMEM;
    double* edev = misc + hp;
    double* sums = edev + B;

    YAO_TRY(pauli_upload(h));
    int width = 0;
    YAO_TRY(pick_forward_width(c, params, s->data, s->dtype, n, B, &width));
    const double* dp = nullptr;
    if (c->nparams > 0) {
        dp = upload_params(params, c->nparams);
        if (!dp) return YAO_ENOMEM;
    }
    YAO_TRY(forward_sweep(s->data, s->dtype, n, B, c, params, width, options().tile_qubits, dp));

    const Plan& P = get_plan(c, 0, G, B, t, cb, L, true, s->dtype == YAO_C64 ? 8 : 16);
    const BoundProgram* bp = bound_program(P, c, true, s->dtype, nullptr, nullptr);
    Program hprog;
    if (!bp) YAO_TRY(build_program(P, c, params, true, s->dtype, hprog));
    YAO_TRY(launch_convert(s->data, s->dtype, psi, YAO_C128, elems));
    YAO_TRY(launch_hpsi_dev(s->data, s->dtype, lam, s->dtype, n, B, h, misc, edev));
    if (nslots) YAO_TRY(launch_fill(gpartial, (size_t)nslots * B * W, 0.0));
    DevProgram hd;
    if (bp) YAO_TRY(bind_program(bp, dp));
    else YAO_TRY(upload_program(hprog, hd, WS_MAT2));
    const Program& prog = bp ? bp->prog : hprog;
    YAO_TRY(launch_backward_passes(P, prog, bp ? bp->d : hd, c, params, psi, lam, s->dtype, n, B, gpartial, W, bp));
    if (nslots) YAO_TRY(launch_row_sums(gpartial, nslots * B, W, sums));
    const size_t nres = (size_t)B + (size_t)nslots * B;
    double* hres = (double*)pinned(WS_PARTIAL, sizeof(double) * nres);
    if (!hres) return YAO_ENOMEM;
    YAO_HIP(hipMemcpyAsync(hres, edev, sizeof(double) * nres, hipMemcpyDeviceToHost, st));
    double dend = 0;
    YAO_TRY(launch_maxdiff(psi, YAO_C128, psi0, s->dtype, elems, &dend));  // synchronises the stream
    for (int b = 0; b < B; ++b) energy[b] = hres[b];
    gather_gradients(c, prog.slot_of_gate, hres + B, B, reduce_batch, grad);
    if (drift) *drift = dend;
    if (check_drift && options().drift_tol > 0 && dend > options().drift_tol)
        return set_error(YAO_EDRIFT, "uncomputed input differs from the input by %.3g > %.3g", dend,
                         options().drift_tol);
    return 0;
}

static std::atomic<long> g_auto_fallbacks{0};

long auto_fallbacks()
{
    return g_auto_fallbacks.load();
}

int backward_fused(yao_state* s, const yao_circuit* c, const double* params, yao_pauli_sum* h, int mode,
                   bool reduce_batch, double* energy, double* grad, double* drift)
{
    const int n = s->n, B = s->batch;
    const size_t elems = s->elems();
    const int G = (int)c->gates.size();
    hipStream_t st = stream();
    const double tol = options().drift_tol > 0 ? options().drift_tol : (s->dtype == YAO_C64 ? 1e-5 : 1e-10);

    void* psi0 = workspace(WS_PSI0, s->bytes());
    if (!psi0) return YAO_ENOMEM;
    YAO_HIP(hipMemcpyAsync(psi0, s->data, s->bytes(), hipMemcpyDeviceToDevice, st));
    if (mode != YAO_GRAD_CHECKPOINT) {
        // Reversible sweep in constant memory. AUTO checks how far the uncomputed input strayed
        // from the kept input and, past the tolerance, restores the input and runs the
        // checkpointed sweep instead (its checkpoints are allocated only then).
        double d = 0;
        YAO_TRY(backward_reversible(s, c, params, h, reduce_batch, energy, grad, &d, psi0,
                                    mode == YAO_GRAD_REVERSIBLE));
        if (drift) *drift = d;
        if (mode == YAO_GRAD_REVERSIBLE || !(d > tol)) return 0;
        g_auto_fallbacks.fetch_add(1);
        YAO_HIP(hipMemcpyAsync(s->data, psi0, s->bytes(), hipMemcpyDeviceToDevice, st));
        return backward_fused(s, c, params, h, YAO_GRAD_CHECKPOINT, reduce_batch, energy, grad, nullptr);
    }

    // Checkpointed sweep: the circuit is cut into gate ranges whose end states the forward
    // keeps; the reverse sweep of each range restarts from the kept state.
    std::vector<int> cuts{0};
    if (G > 0) {
        int len = options().checkpoint_every;
        if (len <= 0) len = std::max((int)std::ceil(std::sqrt((double)G)), 4 * n);
        for (int g = len; g < G; g += len) cuts.push_back(g);
    }
    cuts.push_back(G);
    const int nseg = (int)cuts.size() - 1;

    if (nseg == 1)
        return backward_reversible(s, c, params, h, reduce_batch, energy, grad, drift, psi0, false);
    char* ckpt = (char*)workspace(WS_CKPT, s->bytes() * (size_t)(nseg - 1));
    if (!ckpt) return YAO_ENOMEM;
    for (int sg = 0; sg < nseg; ++sg) {
        YAO_TRY(forward_fused_range(s->data, s->dtype, n, B, c, params, cuts[sg], cuts[sg + 1]));
        if (sg + 1 < nseg)
            YAO_HIP(hipMemcpyAsync(ckpt + s->bytes() * sg, s->data, s->bytes(), hipMemcpyDeviceToDevice, st));
    }
    double* psi = (double*)workspace(WS_PSI64, elems * 16);
    void* lam = workspace(WS_LAM, s->bytes());
    if (!psi || !lam) return YAO_ENOMEM;
    YAO_TRY(launch_convert(s->data, s->dtype, psi, YAO_C128, elems));
    YAO_TRY(launch_hpsi(s->data, s->dtype, lam, s->dtype, n, B, h, energy));

    int t, cb, L;
    tile_geometry(n, B, s->dtype, true, &t, &cb, &L);
    const int ntiles = 1 << (n - (t - cb));
    const int W = std::max(ntiles, adjoint_nblk(n, 1, B));
    const int nslots = count_slots(c);
    double* gpartial = (double*)workspace(WS_PARTIAL, sizeof(double) * (size_t)std::max(1, nslots) * B * W);
    if (!gpartial) return YAO_ENOMEM;
    if (nslots) YAO_TRY(launch_fill(gpartial, (size_t)nslots * B * W, 0.0));
    std::vector<int> slot_of_gate;
    for (int sg = nseg - 1; sg >= 0; --sg) {
        if (sg + 1 < nseg) {
            // psi now stands at the end of segment sg, where the forward kept a copy.
            YAO_TRY(launch_convert(ckpt + s->bytes() * sg, s->dtype, psi, YAO_C128, elems));
        }
        const Plan& P = get_plan(c, cuts[sg], cuts[sg + 1], B, t, cb, L, true, s->dtype == YAO_C64 ? 8 : 16);
        YAO_TRY(run_backward_plan(P, c, params, psi, lam, s->dtype, n, B, gpartial, W, &slot_of_gate));
    }
    const int P_ = c->nparams;
    const size_t glen = reduce_batch ? (size_t)P_ : (size_t)P_ * B;
    for (size_t e = 0; e < glen; ++e) grad[e] = 0.0;
    if (nslots > 0) {
        double* sums = (double*)workspace(WS_PARTIAL2, sizeof(double) * (size_t)nslots * B);
        if (!sums) return YAO_ENOMEM;
        YAO_TRY(launch_row_sums(gpartial, nslots * B, W, sums));
        double* hs = (double*)host_staging(sizeof(double) * (size_t)nslots * B);
        if (!hs) return YAO_ENOMEM;
        YAO_HIP(hipMemcpyAsync(hs, sums, sizeof(double) * (size_t)nslots * B, hipMemcpyDeviceToHost, st));
        YAO_HIP(hipStreamSynchronize(st));
        for (int gi = G - 1; gi >= 0; --gi) {
            const int slot = slot_of_gate.empty() ? -1 : slot_of_gate[gi];
            if (slot < 0) continue;
            const int p = c->gates[gi].param;
            for (int b = 0; b < B; ++b) {
                const double v = hs[(size_t)slot * B + b];
                if (reduce_batch) grad[p] += v;
                else grad[(size_t)b * P_ + p] += v;
            }
        }
    }
    if (drift) *drift = 0;
    return 0;
}

void drop_plans(const yao_circuit* c)
{
    drop_bound(c);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (std::get<0>(it->first) == c) it = g_plans.erase(it);
        else ++it;
    }
}

}  // namespace yao
