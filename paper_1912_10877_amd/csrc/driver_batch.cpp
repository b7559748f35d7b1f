// Batches of independent circuits of uneven size (the batched registers of Sec. "Batched
// Quantum Registers", taken to circuits that differ): every circuit's reset, forward passes,
// H psi with its energy, reverse passes and gradient sums are recorded once into one HIP
// graph, spread over a few streams so that small circuits run beside large ones. Later calls
// with the same circuits rebuild only the parameter-dependent op records and matrices on the
// host, copy them to the device in one transfer and replay the graph.
//
// The forward sweep of each circuit may fold gates into dense blocks (fusion.cpp); the width
// of those blocks and the tile sizes of both sweeps are chosen per qubit count by timing the
// candidates on the first batch that has that qubit count (the autotuner below).
#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <tuple>

#include "driver.h"
#include "fused.h"
#include "tuner.h"

namespace yao {

int launch_fill(double* p, size_t count, double v);
void set_stream(hipStream_t s);
int prepare_pass_kernels();

namespace {

constexpr int kBanks = 16;  // streams of the graph

// Circuits are recorded in phases by state size, each phase waiting for the previous one on
// every stream: a pass over a tile takes about as long whatever the state size, so a small
// circuit's one-tile passes running beside a large circuit's passes (hundreds of tiles) hold
// CUs that the large pass waits for. Phases: >= 2^19 amplitudes, 2^16 .. 2^18, smaller.
int batch_phase(int n)
{
    return n >= 19 ? 0 : (n >= 16 ? 1 : 2);
}

struct Tune {
    int width = 0;  // fusion width of the forward sweep (0: none)
    int tq_f = 0;   // tile qubits of the forward passes (0: default)
    int tq_b = 0;   // of the reverse passes
};
std::map<std::pair<int, int>, Tune> g_tune;  // (n, dtype)

struct Item {
    int idx = 0;  // position in the caller's arrays
    const yao_circuit* c = nullptr;
    const yao_circuit* fc = nullptr;  // circuit of the forward sweep (c, or its fused form)
    uint64_t fc_version = 0;
    yao_state* s = nullptr;
    yao_pauli_sum* h = nullptr;
    Tune tune;
    const Plan* fwd = nullptr;
    const Plan* bwd = nullptr;
    Program pf, pb;
    DevProgram df{}, db{};
    const BoundProgram* bf = nullptr;  // programs bound on the device (null: built on the host)
    const BoundProgram* bb = nullptr;
    size_t poff = 0;                   // the circuit's parameters in the device parameter block
    size_t off_f = 0, off_b = 0, bytes_f = 0, bytes_b = 0;  // program blobs
    int bank = 0;
    int phase = 0;  // recording phase by state size (see record)
    bool small = false;  // run start to end by one workgroup (k_small_circuit)
    int nslots = 0;
    int W = 0;                    // partial-sum row stride of the reverse passes
    size_t out_e = 0, out_g = 0;  // positions in the output block
    double cost = 0;
    int unit = -1;  // recording unit (see Unit)
};

// Circuits recorded together. A z unit holds circuits of one structure (the same gates, the
// same observable, the same state shape) whose programs are bound on the device: every launch
// of the unit runs over all of them at once (grid z), each with its own state, records and
// scratch slice. Any other circuit is a unit of its own, recorded launch by launch.
struct Unit {
    int first = 0, count = 0;  // its items: C.items[first .. first + count)
    bool z = false;
    int bank = 0, phase = 0;
    double cost = 0;
    size_t zf = 0, zo = 0, zb = 0;  // its slot tables in C.d_zs (forward, H psi, reverse)
    size_t sp = 0;                  // its state pointers in C.d_ptrs
};

using Key = std::vector<std::tuple<const yao_circuit*, uint64_t, const yao_state*, const yao_pauli_sum*, int>>;

struct Cache {
    Key key;
    yao_options opt{};
    std::vector<Item> items;  // recording order
    char* d_prog = nullptr;
    char* h_prog = nullptr;
    size_t prog_bytes = 0;
    double* d_out = nullptr;
    double* h_out = nullptr;
    size_t nout = 0;
    double* d_params = nullptr;
    double* h_params = nullptr;
    size_t nparams = 0;
    double* psi64[kBanks] = {};
    void* lam[kBanks] = {};
    double* gpart[kBanks] = {};
    double* hpart[kBanks] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double algo_bytes = 0, algo_flops = 0;
    // Circuits run by k_small_circuit: their descriptors by qubit count (one launch per count)
    // and the bind jobs of their programs (one launch for all).
    SmallCircuit* d_small = nullptr;
    struct SmallLaunch {
        int n, first, count;
    };
    std::vector<SmallLaunch> small_launches;
    BindJob* d_jobs = nullptr;
    int njobs = 0, max_nb = 0;
    std::vector<Unit> units;  // recording order
    ZSlot* d_zs = nullptr;
    void** d_ptrs = nullptr;
};

// Recorded batches, most recently used first: a caller that alternates between a few batch
// lists replays each one's graph instead of recording it again. Each entry owns its scratch
// buffers, so the least recently used one is freed past kMaxCaches.
constexpr size_t kMaxCaches = 4;
std::vector<Cache*> g_caches;
hipStream_t g_capture = nullptr;
hipStream_t g_bank[kBanks] = {};
hipEvent_t g_fork = nullptr, g_join[kBanks] = {};

void free_cache(Cache* c)
{
    if (!c) return;
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->d_prog) (void)hipFree(c->d_prog);
    if (c->h_prog) (void)hipHostFree(c->h_prog);
    if (c->d_out) (void)hipFree(c->d_out);
    if (c->h_out) (void)hipHostFree(c->h_out);
    if (c->d_params) (void)hipFree(c->d_params);
    if (c->d_small) (void)hipFree(c->d_small);
    if (c->d_jobs) (void)hipFree(c->d_jobs);
    if (c->d_zs) (void)hipFree(c->d_zs);
    if (c->d_ptrs) (void)hipFree(c->d_ptrs);
    if (c->h_params) (void)hipHostFree(c->h_params);
    for (int b = 0; b < kBanks; ++b) {
        if (c->psi64[b]) (void)hipFree(c->psi64[b]);
        if (c->lam[b]) (void)hipFree(c->lam[b]);
        if (c->gpart[b]) (void)hipFree(c->gpart[b]);
        if (c->hpart[b]) (void)hipFree(c->hpart[b]);
    }
    delete c;
}

int dev_alloc(void** p, size_t bytes)
{
    if (hipMalloc(p, bytes ? bytes : 256) != hipSuccess) return set_error(YAO_ENOMEM, "batch buffer of %zu bytes", bytes);
    return 0;
}

int host_alloc(void** p, size_t bytes)
{
    if (hipHostMalloc(p, bytes ? bytes : 256, hipHostMallocDefault) != hipSuccess)
        return set_error(YAO_ENOMEM, "pinned batch buffer of %zu bytes", bytes);
    return 0;
}

int ensure_streams()
{
    if (g_fork) return 0;
    YAO_HIP(hipStreamCreateWithFlags(&g_capture, hipStreamNonBlocking));
    for (int b = 0; b < kBanks; ++b) {
        YAO_HIP(hipStreamCreateWithFlags(&g_bank[b], hipStreamNonBlocking));
        YAO_HIP(hipEventCreateWithFlags(&g_join[b], hipEventDisableTiming));
    }
    YAO_HIP(hipEventCreateWithFlags(&g_fork, hipEventDisableTiming));
    return 0;
}

int count_param_slots(const yao_circuit* c)
{
    int k = 0;
    for (const GateRec& g : c->gates) k += (is_param_kind(g.kind) && g.param >= 0) ? 1 : 0;
    return k;
}

const Plan& plan_for(const yao_circuit* c, int n, int dtype, bool bwd, int tq)
{
    int t, cb, L;
    tile_geometry_tq(n, 1, dtype, bwd, tq, &t, &cb, &L);
    return get_plan(c, 0, (int)c->gates.size(), 1, t, cb, L, bwd, dtype == YAO_C64 ? 8 : 16);
}

int reverse_stride(int n, int dtype, int tq)
{
    int t, cb, L;
    tile_geometry_tq(n, 1, dtype, true, tq, &t, &cb, &L);
    return std::max(1 << (n - (t - cb)), adjoint_nblk(n, 1, 1));
}

struct TrialBuffers {
    double* psi64 = nullptr;
    void* lam = nullptr;
    double* gpart = nullptr;
    double* hpart = nullptr;
    double* e = nullptr;
    ~TrialBuffers()
    {
        if (psi64) (void)hipFree(psi64);
        if (lam) (void)hipFree(lam);
        if (gpart) (void)hipFree(gpart);
        if (hpart) (void)hipFree(hpart);
        if (e) (void)hipFree(e);
    }
};

// Candidate tile qubit counts of a state: the default, and smaller tiles when the state has
// more qubits than a tile (more workgroups, more passes).
std::vector<int> tile_candidates(int n, int dtype, bool bwd)
{
    std::vector<int> out{0};
    int t0, cb, L;
    tile_geometry_tq(n, 1, dtype, bwd, 0, &t0, &cb, &L);
    if (t0 - cb >= n) return out;
    for (int tq = t0 - cb - 1; tq >= std::max(kMaxRegBits + 1, t0 - cb - 3); --tq) out.push_back(tq);
    return out;
}

// Pick the fusion width and tile sizes for circuits like c (on state s, observable h) by timing.
int autotune(const yao_circuit* c, const double* params, yao_state* s, yao_pauli_sum* h, Tune* best)
{
    hipStream_t st = g_capture;
    const int n = s->n, dt = s->dtype;
    set_stream(st);
    const size_t N = size_t(1) << n;
    // Forward: fusion width x tile.
    double best_f = 1e300;
    for (int w = 0; w <= std::min(5, n); ++w) {
        for (int tq : tile_candidates(n, dt, false)) {
            double ms = 0;
            YAO_TRY(time_forward(c, params, s->data, dt, n, 1, w, tq, &ms));
            if (ms < best_f) {
                best_f = ms;
                best->width = w;
                best->tq_f = tq;
            }
        }
    }
    // Reverse sweep: tile only (gradients need the gates one by one).
    const int nslots = count_param_slots(c);
    if (nslots == 0) return 0;
    TrialBuffers tb;
    size_t gp = 1;
    for (int tq : tile_candidates(n, dt, true)) gp = std::max(gp, (size_t)nslots * reverse_stride(n, dt, tq));
    YAO_TRY(dev_alloc((void**)&tb.psi64, 16 * N));
    YAO_TRY(dev_alloc(&tb.lam, s->elem_bytes() * N));
    YAO_TRY(dev_alloc((void**)&tb.gpart, sizeof(double) * gp));
    YAO_TRY(dev_alloc((void**)&tb.hpart, sizeof(double) * hpsi_partial_doubles(h, n, 1, dt)));
    YAO_TRY(dev_alloc((void**)&tb.e, sizeof(double)));
    double best_b = 1e300;
    for (int tq : tile_candidates(n, dt, true)) {
        const Plan& P = plan_for(c, n, dt, true, tq);
        Program prog;
        YAO_TRY(build_program(P, c, params, true, dt, prog));
        TrialProgram tp;
        YAO_TRY(tp.load(prog));
        const int W = reverse_stride(n, dt, tq);
        double ms = 0;
        YAO_TRY(launch_fill_basis(s->data, dt, n, 1));
        YAO_TRY(launch_convert(s->data, dt, tb.psi64, YAO_C128, N));
        YAO_TRY(launch_hpsi_dev(s->data, dt, tb.lam, dt, n, 1, h, tb.hpart, tb.e));
        YAO_TRY(time_ms(
            3,
            [&] {
                YAO_TRY(launch_fill(tb.gpart, (size_t)nslots * W, 0.0));
                return launch_backward_passes(P, prog, tp.dp, c, params, tb.psi64, tb.lam, dt, n, 1, tb.gpart, W);
            },
            &ms));
        if (ms < best_b) {
            best_b = ms;
            best->tq_b = tq;
        }
    }
    return 0;
}

// Host programs of every item for these parameters, packed into the pinned blob. Returns 1
// if a program no longer has the size the graph was recorded with.
int build_programs(Cache& C, const double* const* params, bool first)
{
    // A bound program holds one circuit's matrices at a time: a circuit listed twice binds
    // only in its first item and takes host-built programs in the others.
    std::set<const BoundProgram*> used;
    for (Item& it : C.items) {
        if (it.small) continue;  // programs bound at cache build
        const double* p = params[it.idx];
        const int dt = it.s->dtype;
        if (first) {
            // Programs bound on the device when possible: built once, nothing per call.
            const std::vector<FusedPart>* parts = nullptr;
            const yao_circuit* sc = it.tune.width > 0 ? fused_shape(it.c, it.tune.width, &parts) : it.c;
            const Plan& pf = plan_for(sc, it.s->n, dt, false, it.tune.tq_f);
            it.bf = bound_program(pf, sc, false, dt, parts, it.tune.width > 0 ? it.c : nullptr);
            if (it.bf && !used.insert(it.bf).second) it.bf = nullptr;
            if (it.bf) {
                it.fwd = &pf;
                it.fc = sc;
                it.fc_version = sc->version;
            }
            it.bwd = &plan_for(it.c, it.s->n, dt, true, it.tune.tq_b);
            if (it.nslots) it.bb = bound_program(*it.bwd, it.c, true, dt, nullptr, nullptr);
            if (it.bb && !used.insert(it.bb).second) it.bb = nullptr;
        }
        if (!it.bf) {
            const double* fp = nullptr;
            const yao_circuit* fc = forward_circuit(it.c, p, it.tune.width, &fp);
            if (!first && (fc != it.fc || fc->version != it.fc_version)) return 1;
            it.fc = fc;
            it.fc_version = fc->version;
            if (first) it.fwd = &plan_for(fc, it.s->n, dt, false, it.tune.tq_f);
            it.pf = Program();
            YAO_TRY(build_program(*it.fwd, fc, fp, false, dt, it.pf));
        }
        if (it.nslots && !it.bb) {
            it.pb = Program();
            YAO_TRY(build_program(*it.bwd, it.c, p, true, dt, it.pb));
        }
        const size_t bf = it.bf ? 0 : program_blob_bytes(it.pf), bb = (it.nslots && !it.bb) ? program_blob_bytes(it.pb) : 0;
        if (!first && (bf != it.bytes_f || bb != it.bytes_b)) return 1;
        it.bytes_f = bf;
        it.bytes_b = bb;
    }
    return 0;
}

const Program& fwd_prog(const Item& it)
{
    return it.bf ? it.bf->prog : it.pf;
}
const Program& bwd_prog(const Item& it)
{
    return it.bb ? it.bb->prog : it.pb;
}

void pack_all(Cache& C)
{
    for (Item& it : C.items) {
        if (!it.bf) pack_program(it.pf, C.h_prog + it.off_f, C.d_prog + it.off_f, it.df);
        if (it.nslots && !it.bb) pack_program(it.pb, C.h_prog + it.off_b, C.d_prog + it.off_b, it.db);
        if (it.bf) it.df = it.bf->d;
        if (it.bb) it.db = it.bb->d;
    }
}

void pack_params(Cache& C, const double* const* params)
{
    for (const Item& it : C.items)
        if (it.c->nparams > 0) memcpy(C.h_params + it.poff, params[it.idx], sizeof(double) * (size_t)it.c->nparams);
}

bool same_gates(const yao_circuit* a, const yao_circuit* b)
{
    if (a == b) return true;
    if (a->n != b->n || a->nparams != b->nparams || a->gates.size() != b->gates.size()) return false;
    for (size_t i = 0; i < a->gates.size(); ++i) {
        const GateRec &x = a->gates[i], &y = b->gates[i];
        if (x.kind != y.kind || x.param != y.param || x.theta != y.theta || x.k != y.k || x.nctrl != y.nctrl ||
            x.G != y.G)
            return false;
        for (int j = 0; j < x.k; ++j)
            if (x.locs[j] != y.locs[j]) return false;
        for (int m = 0; m < x.nctrl; ++m)
            if (x.ctrls[m] != y.ctrls[m] || x.cvals[m] != y.cvals[m]) return false;
    }
    return true;
}

bool same_observable(const yao_pauli_sum* a, const yao_pauli_sum* b)
{
    return a == b || (a->n == b->n && a->coef == b->coef && a->x == b->x && a->z == b->z);
}

// A circuit can share launches with others of its structure: both programs bound on the
// device (each circuit binds its own records), every pass a tile pass, H psi by tile passes.
bool z_capable(const Item& it)
{
    if (it.small || !it.bf || (it.nslots && !it.bb)) return false;
    for (const HostPass& p : it.fwd->passes)
        if (p.standalone >= 0) return false;
    if (it.nslots)
        for (const HostPass& p : it.bwd->passes)
            if (p.standalone >= 0) return false;
    return obs_passes_ok(it.h, it.s->n, 1, it.s->dtype);
}

// Scratch of one circuit of a z unit: psi in FP64, lambda, reverse and H psi partial sums.
size_t z_item_bytes(const Item& it)
{
    const size_t N = size_t(1) << it.s->n;
    return (16 + it.s->elem_bytes()) * N +
           sizeof(double) * ((size_t)std::max(1, it.nslots) * it.W + hpsi_partial_doubles(it.h, it.s->n, 1, it.s->dtype));
}
constexpr size_t kZUnitBytes = size_t(2) << 30;  // scratch of one z unit at most
constexpr int kZUnitMax = 1024;                   // circuits of one z unit at most

int build_cache(Cache& C, int ncirc, yao_state* const* states, const yao_circuit* const* circs,
                const double* const* params, yao_pauli_sum* const* h)
{
    C.opt = options();
    C.items.resize(ncirc);
    for (int i = 0; i < ncirc; ++i) {
        Item& it = C.items[i];
        it.idx = i;
        it.c = circs[i];
        it.s = states[i];
        it.h = h[i];
        const int n = it.s->n;
        if (!fused_supported(n, 1)) return set_error(YAO_EINVAL, "batch circuit %d has %d qubits; needs >= 5", i, n);
        YAO_TRY(pauli_upload(it.h));
        it.nslots = count_param_slots(it.c);
        it.cost = (double)(it.c->gates.size() + 1) * (double)(uint64_t(1) << n);
        it.phase = batch_phase(n);
    }
    // Circuits whose whole state fits one tile run start to end in one workgroup, from
    // programs of one pass each (3 register bits, FP64 matrices) bound on the device; a
    // circuit with a gate wider than an LDS op, or whose programs cannot be bound there (or are
    // already bound for an earlier entry of the same circuit), takes the pass path.
    {
        std::set<const BoundProgram*> used;
        for (Item& it : C.items) {
            const int n = it.s->n;
            if (n < 5 || n > kSmallMaxQubits) continue;
            bool narrow = true;
            for (const GateRec& g : it.c->gates) narrow &= g.k <= kMaxFusedK;
            const int G = (int)it.c->gates.size();
            if (!narrow || G == 0) continue;
            const Plan& pf = get_plan_ex(it.c, 0, G, 1, n, 0, 0, false, 3, 1 << 30);
            const Plan& pr = get_plan_ex(it.c, 0, G, 1, n, 0, 0, true, 3, 1 << 30);
            if (pf.passes.size() != 1 || pr.passes.size() != 1 || pf.passes[0].standalone >= 0 ||
                pr.passes[0].standalone >= 0)
                continue;
            const BoundProgram* bf = bound_program(pf, it.c, false, YAO_C128, nullptr, nullptr);
            const BoundProgram* bb = bound_program(pr, it.c, true, YAO_C128, nullptr, nullptr);
            if (!bf || !bb || used.count(bf) || used.count(bb)) continue;
            used.insert(bf);
            used.insert(bb);
            it.small = true;
            it.phase = -1;
            it.fwd = &pf;
            it.bwd = &pr;
            it.bf = bf;
            it.bb = bb;
            it.fc = it.c;
            it.fc_version = it.c->version;
        }
    }
    // Tuning per qubit count, on the deepest circuit of that count.
    std::map<std::pair<int, int>, int> rep;
    for (int i = 0; i < ncirc; ++i) {
        if (C.items[i].small) continue;
        auto k = std::make_pair(C.items[i].s->n, C.items[i].s->dtype);
        auto r = rep.find(k);
        if (r == rep.end() || C.items[r->second].c->gates.size() < C.items[i].c->gates.size()) rep[k] = i;
    }
    for (auto& kv : rep) {
        Tune t;
        t.width = C.opt.fuse_width;
        t.tq_f = t.tq_b = C.opt.tile_qubits;
        if (C.opt.autotune) {
            auto f = g_tune.find(kv.first);
            if (f != g_tune.end()) {
                t = f->second;
            } else {
                const Item& it = C.items[kv.second];
                YAO_TRY(autotune(it.c, params[it.idx], it.s, it.h, &t));
                g_tune[kv.first] = t;
            }
        }
        for (Item& it : C.items)
            if (!it.small && it.s->n == kv.first.first && it.s->dtype == kv.first.second) it.tune = t;
    }
    YAO_TRY(build_programs(C, params, true));
    for (Item& it : C.items)
        if (!it.small) it.W = reverse_stride(it.s->n, it.s->dtype, it.tune.tq_b);

    // Units: circuits of one structure with bound programs together (z units), every other
    // circuit alone; the small circuits stay outside the units.
    std::vector<std::vector<int>> members;
    std::vector<bool> zunit;
    {
        std::map<std::pair<int, int>, std::vector<int>> open;  // (n, dtype) -> z units
        for (int i = 0; i < (int)C.items.size(); ++i) {
            const Item& it = C.items[i];
            if (it.small) continue;
            if (!z_capable(it)) {
                members.push_back({i});
                zunit.push_back(false);
                continue;
            }
            std::vector<int>& cand = open[std::make_pair(it.s->n, it.s->dtype)];
            int u = -1;
            for (int v : cand) {
                const Item& lead = C.items[members[v][0]];
                if ((int)members[v].size() < kZUnitMax &&
                    z_item_bytes(lead) * (members[v].size() + 1) <= kZUnitBytes && lead.W == it.W &&
                    lead.nslots == it.nslots && same_gates(lead.c, it.c) && same_observable(lead.h, it.h)) {
                    u = v;
                    break;
                }
            }
            if (u < 0) {
                u = (int)members.size();
                members.emplace_back();
                zunit.push_back(true);
                cand.push_back(u);
            }
            members[u].push_back(i);
        }
    }
    // By phase, then largest units first, each on the least loaded stream of its phase; the
    // items are reordered so that each unit's circuits follow each other (their energies and
    // gradient sums then sit in consecutive output entries).
    std::vector<int> order(members.size());
    std::vector<double> ucost(members.size(), 0.0);
    for (size_t u = 0; u < members.size(); ++u) {
        order[u] = (int)u;
        for (int i : members[u]) ucost[u] += C.items[i].cost;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int pa = C.items[members[a][0]].phase, pb = C.items[members[b][0]].phase;
        return pa != pb ? pa < pb : ucost[a] > ucost[b];
    });
    {
        std::vector<Item> sorted;
        sorted.reserve(C.items.size());
        for (const Item& it : C.items)
            if (it.small) sorted.push_back(it);
        for (int u : order) {
            Unit U;
            U.first = (int)sorted.size();
            U.count = (int)members[u].size();
            U.z = zunit[u];
            U.phase = C.items[members[u][0]].phase;
            U.cost = ucost[u];
            for (int i : members[u]) {
                sorted.push_back(C.items[i]);
                sorted.back().unit = (int)C.units.size();
            }
            C.units.push_back(U);
        }
        C.items.swap(sorted);
    }
    double load[kBanks] = {};
    int cur_phase = -1;
    size_t psi_b[kBanks] = {}, lam_b[kBanks] = {}, gp_b[kBanks] = {}, hp_b[kBanks] = {};
    size_t nout = 0, off = 0, nzs = 0, nptr = 0;
    for (Item& it : C.items) {
        if (!it.small) continue;
        it.out_e = nout++;
        it.off_f = it.off_b = off;
    }
    for (Unit& U : C.units) {
        if (U.phase != cur_phase) {
            cur_phase = U.phase;
            for (double& l : load) l = 0;
        }
        int best = 0;
        for (int b = 1; b < kBanks; ++b)
            if (load[b] < load[best]) best = b;
        U.bank = best;
        load[best] += U.cost;
        const Item& lead = C.items[U.first];
        const size_t N = size_t(1) << lead.s->n, nz = (size_t)U.count;
        psi_b[best] = std::max(psi_b[best], nz * 16 * N);
        lam_b[best] = std::max(lam_b[best], nz * lead.s->elem_bytes() * N);
        gp_b[best] = std::max(gp_b[best], nz * sizeof(double) * (size_t)std::max(1, lead.nslots) * lead.W);
        hp_b[best] = std::max(hp_b[best], nz * sizeof(double) * hpsi_partial_doubles(lead.h, lead.s->n, 1, lead.s->dtype));
        if (U.z) {
            U.zf = nzs;
            U.zo = nzs + nz;
            U.zb = nzs + 2 * nz;
            nzs += 3 * nz;
            U.sp = nptr;
            nptr += nz;
        }
        for (int j = 0; j < U.count; ++j) {
            Item& it = C.items[U.first + j];
            it.bank = best;
            it.out_e = nout++;
            it.off_f = off;
            off += it.bytes_f;
            it.off_b = off;
            off += it.bytes_b;
        }
    }
    for (Item& it : C.items) {
        it.out_g = nout;
        nout += it.nslots;
        it.poff = C.nparams;
        C.nparams += (size_t)it.c->nparams;
    }
    C.nout = nout;
    C.prog_bytes = off;
    YAO_TRY(dev_alloc((void**)&C.d_prog, C.prog_bytes));
    YAO_TRY(host_alloc((void**)&C.h_prog, C.prog_bytes));
    YAO_TRY(dev_alloc((void**)&C.d_params, sizeof(double) * std::max<size_t>(1, C.nparams)));
    YAO_TRY(host_alloc((void**)&C.h_params, sizeof(double) * std::max<size_t>(1, C.nparams)));
    pack_params(C, params);
    YAO_TRY(dev_alloc((void**)&C.d_out, sizeof(double) * C.nout));
    YAO_TRY(host_alloc((void**)&C.h_out, sizeof(double) * C.nout));
    for (int b = 0; b < kBanks; ++b) {
        YAO_TRY(dev_alloc((void**)&C.psi64[b], psi_b[b]));
        YAO_TRY(dev_alloc(&C.lam[b], lam_b[b]));
        YAO_TRY(dev_alloc((void**)&C.gpart[b], gp_b[b]));
        YAO_TRY(dev_alloc((void**)&C.hpart[b], hp_b[b]));
    }
    pack_all(C);
    // Slot tables of the z units: each circuit's state, its slice of the unit's scratch (at
    // the bank's buffers) and its bound records.
    if (nzs) {
        std::vector<ZSlot> zs(nzs);
        std::vector<void*> ptrs(nptr);
        for (const Unit& U : C.units) {
            if (!U.z) continue;
            const Item& lead = C.items[U.first];
            const size_t N = size_t(1) << lead.s->n, es = lead.s->elem_bytes();
            const size_t wo = hpsi_partial_doubles(lead.h, lead.s->n, 1, lead.s->dtype);
            const size_t wg = (size_t)std::max(1, lead.nslots) * lead.W;
            for (int j = 0; j < U.count; ++j) {
                const Item& it = C.items[U.first + j];
                void* lam = (char*)C.lam[U.bank] + (size_t)j * es * N;
                ptrs[U.sp + j] = it.s->data;
                zs[U.zf + j] = ZSlot{it.s->data, nullptr, it.bf->d.ops, nullptr};
                zs[U.zo + j] = ZSlot{it.s->data, lam, nullptr, C.hpart[U.bank] + (size_t)j * wo};
                zs[U.zb + j] = ZSlot{C.psi64[U.bank] + (size_t)j * 2 * N, lam, it.nslots ? it.bb->d.ops : nullptr,
                                     C.gpart[U.bank] + (size_t)j * wg};
            }
        }
        YAO_TRY(dev_alloc((void**)&C.d_zs, sizeof(ZSlot) * nzs));
        YAO_TRY(dev_alloc((void**)&C.d_ptrs, sizeof(void*) * nptr));
        YAO_HIP(hipMemcpy(C.d_zs, zs.data(), sizeof(ZSlot) * nzs, hipMemcpyHostToDevice));
        YAO_HIP(hipMemcpy(C.d_ptrs, ptrs.data(), sizeof(void*) * nptr, hipMemcpyHostToDevice));
    }
    // Descriptors and bind jobs of the small circuits, by qubit count.
    {
        std::vector<const Item*> sm;
        for (const Item& it : C.items)
            if (it.small) sm.push_back(&it);
        std::stable_sort(sm.begin(), sm.end(), [](const Item* a, const Item* b) { return a->s->n < b->s->n; });
        std::vector<SmallCircuit> hs;
        std::vector<BindJob> jobs;
        for (const Item* it : sm) {
            SmallCircuit x;
            memset(&x, 0, sizeof(x));
            x.fops = it->bf->d.ops;
            x.fgroups = it->bf->d.groups;
            x.fmats = it->bf->d.mats;
            x.nfg = (int)it->fwd->passes[0].groups.size();
            x.rops = it->bb->d.ops;
            x.rgroups = it->bb->d.groups;
            x.rmats = it->bb->d.mats;
            x.nrg = (int)it->bwd->passes[0].groups.size();
            x.hgroups = (const PGroup*)it->h->d_groups;
            x.hterms = (const PTerm*)it->h->d_terms;
            x.nhg = it->h->ngroups;
            x.state = it->s->data;
            x.energy = C.d_out + it->out_e;
            x.grad = C.d_out + it->out_g;
            x.n = it->s->n;
            x.c64 = it->s->dtype == YAO_C64 ? 1 : 0;
            if (C.small_launches.empty() || C.small_launches.back().n != x.n)
                C.small_launches.push_back(Cache::SmallLaunch{x.n, (int)hs.size(), 0});
            C.small_launches.back().count++;
            hs.push_back(x);
            for (const BoundProgram* b : {it->bf, it->bb}) {
                const int nb = (int)b->prog.binds.size();
                if (nb == 0) continue;
                jobs.push_back(BindJob{b->d.ops, b->dbinds, b->dfacs, C.d_params + it->poff, nb, 0});
                C.max_nb = std::max(C.max_nb, nb);
            }
        }
        // The z units' circuits bind here too: one launch binds every such program.
        for (const Unit& U : C.units) {
            if (!U.z) continue;
            for (int j = 0; j < U.count; ++j) {
                const Item& it = C.items[U.first + j];
                for (const BoundProgram* b : {it.bf, it.nslots ? it.bb : nullptr}) {
                    const int nb = b ? (int)b->prog.binds.size() : 0;
                    if (nb == 0) continue;
                    jobs.push_back(BindJob{b->d.ops, b->dbinds, b->dfacs, C.d_params + it.poff, nb, 0});
                    C.max_nb = std::max(C.max_nb, nb);
                }
            }
        }
        if (!hs.empty()) {
            YAO_TRY(dev_alloc((void**)&C.d_small, sizeof(SmallCircuit) * hs.size()));
            YAO_HIP(hipMemcpy(C.d_small, hs.data(), sizeof(SmallCircuit) * hs.size(), hipMemcpyHostToDevice));
        }
        if (!jobs.empty()) {
            YAO_TRY(dev_alloc((void**)&C.d_jobs, sizeof(BindJob) * jobs.size()));
            YAO_HIP(hipMemcpy(C.d_jobs, jobs.data(), sizeof(BindJob) * jobs.size(), hipMemcpyHostToDevice));
        }
        C.njobs = (int)jobs.size();
    }
    // Algorithmic traffic and flops of one replay (every pass reads and writes its states once).
    for (const Item& it : C.items) {
        const double N = (double)(uint64_t(1) << it.s->n);
        const double s = (double)it.s->elem_bytes();
        for (size_t p = 0; p < it.fwd->passes.size(); ++p) {
            C.algo_bytes += 2.0 * s * N;
            C.algo_flops += fwd_prog(it).pass_flops[p] * N;
        }
        C.algo_bytes += 2.0 * s * N + 16.0 * N;  // H psi reads psi, writes lambda; FP64 copy
        if (!it.nslots) continue;
        for (size_t p = 0; p < it.bwd->passes.size(); ++p) {
            C.algo_bytes += 2.0 * (16.0 + s) * N;
            C.algo_flops += bwd_prog(it).pass_flops[p] * N;
        }
    }
    return 0;
}

// Restores single-circuit launches when a z unit's recording ends (also on errors).
struct ZBatchScope {
    ZBatchScope(const ZSlot* zs, int nz) { set_zbatch(zs, nz); }
    ~ZBatchScope() { set_zbatch(nullptr, 0); }
};

// One z unit: every launch runs over the unit's nz circuits (grid z); the leader's plans and
// programs give the shared part of each launch.
int record_z_unit(Cache& C, const Unit& U)
{
    const Item& it = C.items[U.first];
    const int n = it.s->n, dt = it.s->dtype, bk = U.bank, nz = U.count;
    YAO_TRY(launch_fill_basis_z(C.d_ptrs + U.sp, nz, dt, n));
    {
        ZBatchScope z(C.d_zs + U.zf, nz);
        YAO_TRY(launch_forward_passes(*it.fwd, fwd_prog(it), it.df, it.s->data, dt, n, 1, it.fc, nullptr, it.bf));
    }
    {
        ZBatchScope z(C.d_zs + U.zo, nz);
        YAO_TRY(launch_hpsi_dev(it.s->data, dt, C.lam[bk], dt, n, 1, it.h, C.hpart[bk], C.d_out + it.out_e));
    }
    if (it.nslots == 0) return 0;
    YAO_TRY(launch_convert_z(C.d_ptrs + U.sp, nz, dt, C.psi64[bk], n));
    YAO_TRY(launch_fill(C.gpart[bk], (size_t)nz * it.nslots * it.W, 0.0));
    {
        ZBatchScope z(C.d_zs + U.zb, nz);
        YAO_TRY(launch_backward_passes(*it.bwd, bwd_prog(it), it.db, it.c, nullptr, C.psi64[bk], C.lam[bk], dt, n, 1,
                                       C.gpart[bk], it.W, it.bb));
    }
    return launch_row_sums(C.gpart[bk], nz * it.nslots, it.W, C.d_out + it.out_g);
}

int record_item(Cache& C, Item& it)
{
    const int n = it.s->n, dt = it.s->dtype, bk = it.bank;
    YAO_TRY(launch_fill_basis(it.s->data, dt, n, 1));
    if (it.bf) YAO_TRY(bind_program(it.bf, C.d_params + it.poff));
    YAO_TRY(launch_forward_passes(*it.fwd, fwd_prog(it), it.df, it.s->data, dt, n, 1, it.fc, nullptr, it.bf));
    YAO_TRY(launch_hpsi_dev(it.s->data, dt, C.lam[bk], dt, n, 1, it.h, C.hpart[bk], C.d_out + it.out_e));
    if (it.nslots == 0) return 0;
    YAO_TRY(launch_convert(it.s->data, dt, C.psi64[bk], YAO_C128, size_t(1) << n));
    YAO_TRY(launch_fill(C.gpart[bk], (size_t)it.nslots * it.W, 0.0));
    if (it.bb) YAO_TRY(bind_program(it.bb, C.d_params + it.poff));
    YAO_TRY(launch_backward_passes(*it.bwd, bwd_prog(it), it.db, it.c, nullptr, C.psi64[bk], C.lam[bk], dt, n, 1,
                                   C.gpart[bk], it.W, it.bb));
    return launch_row_sums(C.gpart[bk], it.nslots, it.W, C.d_out + it.out_g);
}

int record(Cache& C)
{
    YAO_TRY(prepare_pass_kernels());
    hipStream_t cs = g_capture;
    YAO_HIP(hipStreamSynchronize(cs));
    YAO_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    prof_suspend(true);
    set_recording(true);
    int rc = 0;
    do {
        // One launch binds the programs of the small circuits and of the z units, before
        // any stream starts.
        set_stream(cs);
        if ((rc = launch_bind_jobs(C.d_jobs, C.njobs, C.max_nb))) break;
        if (hipEventRecord(g_fork, cs) != hipSuccess) {
            rc = set_error(YAO_EHIP, "fork record");
            break;
        }
        for (int b = 0; b < kBanks && !rc; ++b)
            if (hipStreamWaitEvent(g_bank[b], g_fork, 0) != hipSuccess) rc = set_error(YAO_EHIP, "fork wait");
        if (rc) break;
        // The small circuits: one launch per qubit count.
        for (const Cache::SmallLaunch& l : C.small_launches)
            if ((rc = launch_small_circuits(C.d_small + l.first, l.count, l.n))) break;
        if (rc) break;
        int phase = -1;
        for (const Unit& U : C.units) {
            if (U.phase != phase) {
                // Every stream finishes the previous phase before any starts this one.
                phase = U.phase;
                for (int b = 0; b < kBanks && !rc; ++b)
                    if (hipEventRecord(g_join[b], g_bank[b]) != hipSuccess || hipStreamWaitEvent(cs, g_join[b], 0) != hipSuccess)
                        rc = set_error(YAO_EHIP, "phase join");
                if (!rc && hipEventRecord(g_fork, cs) != hipSuccess) rc = set_error(YAO_EHIP, "phase fork record");
                for (int b = 0; b < kBanks && !rc; ++b)
                    if (hipStreamWaitEvent(g_bank[b], g_fork, 0) != hipSuccess) rc = set_error(YAO_EHIP, "phase fork wait");
                if (rc) break;
            }
            set_stream(g_bank[U.bank]);
            if (U.z) rc = record_z_unit(C, U);
            else rc = record_item(C, C.items[U.first]);
            if (rc) break;
        }
        if (rc) break;
        for (int b = 0; b < kBanks; ++b) {
            if (hipEventRecord(g_join[b], g_bank[b]) != hipSuccess || hipStreamWaitEvent(cs, g_join[b], 0) != hipSuccess) {
                rc = set_error(YAO_EHIP, "join");
                break;
            }
        }
    } while (0);
    prof_suspend(false);
    set_recording(false);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc ? rc : hip_fail(e, "hipStreamEndCapture");
    }
    C.graph = graph;
    YAO_HIP(hipGraphInstantiate(&C.exec, graph, nullptr, nullptr, 0));
    return 0;
}

// Same circuits, states, observables and types in the same order (circuit versions aside).
bool same_objects(const Key& a, const Key& b)
{
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i)
        if (std::get<0>(a[i]) != std::get<0>(b[i]) || std::get<2>(a[i]) != std::get<2>(b[i]) ||
            std::get<3>(a[i]) != std::get<3>(b[i]) || std::get<4>(a[i]) != std::get<4>(b[i]))
            return false;
    return true;
}

bool same_options(const yao_options& a, const yao_options& b)
{
    return a.tile_qubits == b.tile_qubits && a.fuse_width == b.fuse_width && a.mfma == b.mfma &&
           a.autotune == b.autotune;
}

}  // namespace

int batch_run(int ncirc, yao_state* const* states, const yao_circuit* const* circs, const double* const* params,
              yao_pauli_sum* const* h, double* energy, double* const* grad)
{
    YAO_TRY(ensure_streams());
    const hipStream_t origin = stream();
    Key key;
    for (int i = 0; i < ncirc; ++i) key.emplace_back(circs[i], circs[i]->version, states[i], h[i], states[i]->dtype);
    Cache* hit = nullptr;
    for (size_t i = 0; i < g_caches.size(); ++i)
        if (g_caches[i]->key == key && same_options(g_caches[i]->opt, options())) {
            hit = g_caches[i];
            g_caches.erase(g_caches.begin() + (long)i);
            g_caches.insert(g_caches.begin(), hit);
            break;
        }
    bool fresh = !hit;
    if (hit) {
        const int r = build_programs(*hit, params, false);
        if (r < 0) return r;
        if (r == 1) fresh = true;
        else {
            pack_all(*hit);
            pack_params(*hit, params);
        }
    }
    if (fresh) {
        YAO_HIP(hipStreamSynchronize(origin));
        // Drop the entry being replaced, entries for the same objects at older circuit versions
        // (they can never match again), and the least recently used one past the limit.
        for (size_t i = 0; i < g_caches.size();) {
            if (g_caches[i] == hit || same_objects(g_caches[i]->key, key)) {
                free_cache(g_caches[i]);
                g_caches.erase(g_caches.begin() + (long)i);
            } else ++i;
        }
        while (g_caches.size() >= kMaxCaches) {
            free_cache(g_caches.back());
            g_caches.pop_back();
        }
        Cache* c = new Cache;
        c->key = key;
        int rc = build_cache(*c, ncirc, states, circs, params, h);
        if (!rc) rc = record(*c);
        set_stream(origin);
        if (rc) {
            free_cache(c);
            return rc;
        }
        g_caches.insert(g_caches.begin(), c);
    }
    Cache& C = *g_caches.front();
    const int pi = prof_begin(YAO_KF_BATCH);
    if (C.prog_bytes) YAO_HIP(hipMemcpyAsync(C.d_prog, C.h_prog, C.prog_bytes, hipMemcpyHostToDevice, origin));
    if (C.nparams)
        YAO_HIP(hipMemcpyAsync(C.d_params, C.h_params, sizeof(double) * C.nparams, hipMemcpyHostToDevice, origin));
    YAO_HIP(hipGraphLaunch(C.exec, origin));
    prof_end(pi, C.algo_bytes, C.algo_flops);
    YAO_HIP(hipMemcpyAsync(C.h_out, C.d_out, sizeof(double) * C.nout, hipMemcpyDeviceToHost, origin));
    YAO_HIP(hipStreamSynchronize(origin));
    for (const Item& it : C.items) {
        energy[it.idx] = C.h_out[it.out_e];
        const int P = it.c->nparams;
        double* g = grad[it.idx];
        for (int p = 0; p < P; ++p) g[p] = 0.0;
        if (!it.nslots) continue;
        for (int gi = (int)it.c->gates.size() - 1; gi >= 0; --gi) {
            const int slot = bwd_prog(it).slot_of_gate[gi];
            if (slot >= 0) g[it.c->gates[gi].param] += C.h_out[it.out_g + slot];
        }
    }
    return 0;
}

void drop_batch(const void* obj)
{
    for (size_t i = 0; i < g_caches.size();) {
        bool uses = false;
        for (const Item& it : g_caches[i]->items)
            uses |= (const void*)it.c == obj || (const void*)it.s == obj || (const void*)it.h == obj;
        if (uses) {
            (void)hipDeviceSynchronize();
            free_cache(g_caches[i]);
            g_caches.erase(g_caches.begin() + (long)i);
        } else ++i;
    }
}

}  // namespace yao
