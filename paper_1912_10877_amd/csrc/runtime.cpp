// Host runtime: error state, stream binding, options, device workspace and the FP64 gate
// matrices that every kernel receives (the device code needs no transcendental functions).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "runtime.h"

namespace yao {

static thread_local std::string g_err;
static hipStream_t g_stream = nullptr;
static yao_options g_opts = {0, 0, 1, 0, 0.0, 1, 1, 3};
static int g_device_ok = -1;  // -1 unknown, 0 no gfx950, 1 ok

int set_error(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory) return set_error(YAO_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return set_error(YAO_EHIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error()
{
    return g_err.c_str();
}

hipStream_t stream()
{
    return g_stream;
}
void set_stream(hipStream_t s)
{
    g_stream = s;
}

const yao_options& options()
{
    return g_opts;
}
void set_options(const yao_options& o)
{
    g_opts = o;
}
void default_options(yao_options& o)
{
    o.plain = 0;
    o.tile_qubits = 0;
    o.fuse_width = 0;
    o.checkpoint_every = 0;
    o.drift_tol = 0.0;
    o.mfma = 1;
    o.autotune = 1;
    o.jit = 3;
}

int ensure_device()
{
    if (g_device_ok == 1) return 0;
    int dev = 0, count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
        g_device_ok = 0;
        return set_error(YAO_ENODEV, "no HIP device visible");
    }
    if (hipGetDevice(&dev) != hipSuccess) return set_error(YAO_ENODEV, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return set_error(YAO_ENODEV, "hipGetDeviceProperties failed");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_device_ok = 0;
        return set_error(YAO_ENODEV, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    }
    g_device_ok = 1;
    return 0;
}

// ---------------------------------------------------------------------------------- workspace
static void* g_ws[WS_COUNT] = {nullptr};
static size_t g_ws_size[WS_COUNT] = {0};
static void* g_stage = nullptr;
static size_t g_stage_size = 0;

void* workspace(int slot, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (g_ws_size[slot] >= bytes) return g_ws[slot];
    if (g_ws[slot]) {
        // hipFree waits for queued work that may still read the old buffer.
        (void)hipFree(g_ws[slot]);
        g_ws[slot] = nullptr;
        g_ws_size[slot] = 0;
    }
    size_t want = bytes + bytes / 8;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        set_error(YAO_ENOMEM, "workspace slot %d: %zu bytes: %s", slot, want, hipGetErrorString(e));
        return nullptr;
    }
    g_ws[slot] = p;
    g_ws_size[slot] = want;
    return p;
}

void* host_staging(size_t bytes)
{
    if (g_stage_size >= bytes) return g_stage;
    if (g_stage) (void)hipHostFree(g_stage);
    g_stage = nullptr;
    g_stage_size = 0;
    size_t want = bytes < 4096 ? 4096 : bytes;
    if (hipHostMalloc(&g_stage, want, hipHostMallocDefault) != hipSuccess) {
        set_error(YAO_ENOMEM, "pinned staging %zu bytes", want);
        return nullptr;
    }
    g_stage_size = want;
    return g_stage;
}

static void* g_pin[WS_COUNT] = {};
static size_t g_pin_size[WS_COUNT] = {};

void* pinned(int slot, size_t bytes)
{
    if (g_pin_size[slot] >= bytes) return g_pin[slot];
    if (g_pin[slot]) {
        (void)hipStreamSynchronize(g_stream);
        (void)hipHostFree(g_pin[slot]);
        g_pin[slot] = nullptr;
        g_pin_size[slot] = 0;
    }
    const size_t want = (bytes < 65536 ? 65536 : bytes) + bytes / 4;
    if (hipHostMalloc(&g_pin[slot], want, hipHostMallocDefault) != hipSuccess) {
        g_pin[slot] = nullptr;
        set_error(YAO_ENOMEM, "pinned slot %d: %zu bytes", slot, want);
        return nullptr;
    }
    g_pin_size[slot] = want;
    return g_pin[slot];
}

static constexpr size_t kRingSlot = 64 * 1024;
static constexpr int kRingSlots = 256;
static char* g_ring = nullptr;
static int g_ring_next = 0;
static bool g_recording = false;

void set_recording(bool on)
{
    g_recording = on;
}

bool recording()
{
    return g_recording;
}

void* ring_upload(const void* host, size_t bytes)
{
    if (g_recording) {
        // A captured copy would keep the host address and read it again at every replay.
        set_error(YAO_EINVAL, "ring upload while a graph is being recorded");
        return nullptr;
    }
    if (bytes > kRingSlot) {
        set_error(YAO_EINVAL, "ring upload of %zu bytes exceeds the slot size", bytes);
        return nullptr;
    }
    if (!g_ring) {
        if (hipMalloc((void**)&g_ring, kRingSlot * kRingSlots) != hipSuccess) {
            set_error(YAO_ENOMEM, "matrix ring");
            return nullptr;
        }
    }
    char* dst = g_ring + kRingSlot * (size_t)g_ring_next;
    g_ring_next = (g_ring_next + 1) % kRingSlots;
    // Pageable source: the call returns once the source has been staged.
    if (hipMemcpyAsync(dst, host, bytes, hipMemcpyHostToDevice, g_stream) != hipSuccess) {
        set_error(YAO_EHIP, "ring upload failed");
        return nullptr;
    }
    return dst;
}

void* upload_to(int slot, const void* host, size_t bytes)
{
    void* d = workspace(slot, bytes);
    if (!d) return nullptr;
    if (hipMemcpyAsync(d, host, bytes, hipMemcpyHostToDevice, g_stream) != hipSuccess) {
        set_error(YAO_EHIP, "upload failed");
        return nullptr;
    }
    return d;
}

// ---------------------------------------------------------------------------------- matrices
bool is_param_kind(int kind)
{
    return kind == YAO_RX || kind == YAO_RY || kind == YAO_RZ || kind == YAO_SHIFT || kind == YAO_ROT;
}

static void set_entry(HostMat& U, int r, int c, double re, double im)
{
    U.re[r * U.dim() + c] = re;
    U.im[r * U.dim() + c] = im;
}

// Generator of a rotation as a matrix (Pauli for Rx/Ry/Rz, the given G for rot).
static void generator(const GateRec& g, HostMat& S)
{
    S.resize(g.kind == YAO_ROT ? g.k : 1);
    switch (g.kind) {
    case YAO_RX: set_entry(S, 0, 1, 1, 0); set_entry(S, 1, 0, 1, 0); break;
    case YAO_RY: set_entry(S, 0, 1, 0, -1); set_entry(S, 1, 0, 0, 1); break;
    case YAO_RZ: set_entry(S, 0, 0, 1, 0); set_entry(S, 1, 1, -1, 0); break;
    default:
        for (size_t t = 0; t < S.re.size(); ++t) {
            S.re[t] = g.G[2 * t];
            S.im[t] = g.G[2 * t + 1];
        }
    }
}

bool gate_matrix(const GateRec& g, double theta, HostMat& U)
{
    const double h = 0.70710678118654752440;  // 1/sqrt(2)
    U.resize(g.k);
    switch (g.kind) {
    case YAO_X: set_entry(U, 0, 1, 1, 0); set_entry(U, 1, 0, 1, 0); return true;
    case YAO_Y: set_entry(U, 0, 1, 0, -1); set_entry(U, 1, 0, 0, 1); return true;
    case YAO_Z: set_entry(U, 0, 0, 1, 0); set_entry(U, 1, 1, -1, 0); return true;
    case YAO_H:
        set_entry(U, 0, 0, h, 0); set_entry(U, 0, 1, h, 0);
        set_entry(U, 1, 0, h, 0); set_entry(U, 1, 1, -h, 0);
        return true;
    case YAO_S: set_entry(U, 0, 0, 1, 0); set_entry(U, 1, 1, 0, 1); return true;
    case YAO_SDAG: set_entry(U, 0, 0, 1, 0); set_entry(U, 1, 1, 0, -1); return true;
    case YAO_T: set_entry(U, 0, 0, 1, 0); set_entry(U, 1, 1, h, h); return true;
    case YAO_TDAG: set_entry(U, 0, 0, 1, 0); set_entry(U, 1, 1, h, -h); return true;
    case YAO_SHIFT: set_entry(U, 0, 0, 1, 0); set_entry(U, 1, 1, std::cos(theta), std::sin(theta)); return true;
    case YAO_RX: case YAO_RY: case YAO_RZ: case YAO_ROT: {
        // cos(theta/2) 1 - i sin(theta/2) S
        static thread_local HostMat S;  // reused: programs are rebuilt for every call
        generator(g, S);
        const double c = std::cos(theta / 2), s = std::sin(theta / 2);
        for (int r = 0; r < U.dim(); ++r)
            for (int q = 0; q < U.dim(); ++q) {
                size_t t = (size_t)r * U.dim() + q;
                U.re[t] = (r == q ? c : 0.0) + s * S.im[t];
                U.im[t] = -s * S.re[t];
            }
        return true;
    }
    case YAO_DENSE:
        for (size_t t = 0; t < U.re.size(); ++t) {
            U.re[t] = g.G[2 * t];
            U.im[t] = g.G[2 * t + 1];
        }
        return true;
    default: return false;
    }
}

bool gate_grad_matrix(const GateRec& g, double theta, HostMat& M)
{
    (void)theta;
    if (g.kind == YAO_SHIFT) {
        // d/dtheta diag(1, e^{i theta}) times its adjoint: diag(0, i)
        M.resize(1);
        set_entry(M, 1, 1, 0, 1);
        return true;
    }
    if (g.kind == YAO_RX || g.kind == YAO_RY || g.kind == YAO_RZ || g.kind == YAO_ROT) {
        // d/dtheta exp(-i theta S/2) = (-i/2) S exp(-i theta S/2), so M = -(i/2) S
        static thread_local HostMat S;  // reused: programs are rebuilt for every call
        generator(g, S);
        M.resize(S.k);
        for (size_t t = 0; t < S.re.size(); ++t) {
            M.re[t] = 0.5 * S.im[t];
            M.im[t] = -0.5 * S.re[t];
        }
        return true;
    }
    return false;
}

void dagger_into(const HostMat& U, HostMat& D)
{
    D.resize(U.k);
    const int d = U.dim();
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            D.re[c * d + r] = U.re[r * d + c];
            D.im[c * d + r] = -U.im[r * d + c];
        }
}

HostMat dagger(const HostMat& U)
{
    HostMat D;
    D.resize(U.k);
    const int d = U.dim();
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            D.re[c * d + r] = U.re[r * d + c];
            D.im[c * d + r] = -U.im[r * d + c];
        }
    return D;
}

HostMat matmul(const HostMat& A, const HostMat& B)
{
    HostMat C;
    C.resize(A.k);
    const int d = A.dim();
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            double xr = 0, xi = 0;
            for (int t = 0; t < d; ++t) {
                double ar = A.re[r * d + t], ai = A.im[r * d + t];
                double br = B.re[t * d + c], bi = B.im[t * d + c];
                xr += ar * br - ai * bi;
                xi += ar * bi + ai * br;
            }
            C.re[r * d + c] = xr;
            C.im[r * d + c] = xi;
        }
    return C;
}

int classify(const HostMat& U)
{
    if (U.k != 1) return MC_DENSE;
    const bool off0 = U.re[1] == 0 && U.im[1] == 0 && U.re[2] == 0 && U.im[2] == 0;
    const bool diag0 = U.re[0] == 0 && U.im[0] == 0 && U.re[3] == 0 && U.im[3] == 0;
    if (off0) return (U.re[0] == 1 && U.im[0] == 0) ? MC_DIAG1 : MC_DIAG;
    if (diag0) return MC_ANTI;
    return MC_DENSE;
}

CtrlSpec make_ctrl(int nctrl, const int* ctrls, const int* cvals)
{
    CtrlSpec c;
    for (int m = 0; m < nctrl; ++m) {
        c.mask |= uint64_t(1) << ctrls[m];
        if (!cvals || cvals[m]) c.val |= uint64_t(1) << ctrls[m];
    }
    return c;
}

// ---------------------------------------------------------------------------------- profiler
namespace {
struct ProfRec {
    int family;
    int ev;  // index of the start event; the end event is ev + 1
    double bytes, flops;
};
bool g_prof_on = false;
std::vector<hipEvent_t> g_prof_events;
std::vector<ProfRec> g_prof_recs;
size_t g_prof_next_ev = 0;
}  // namespace

int prof_enable(bool on)
{
    g_prof_on = on;
    if (on) {
        g_prof_recs.clear();
        g_prof_next_ev = 0;
    }
    return 0;
}

static bool g_prof_suspended = false;

void prof_suspend(bool on)
{
    g_prof_suspended = on;
}

int prof_begin(int family)
{
    if (!g_prof_on || g_prof_suspended) return -1;
    if (g_prof_next_ev + 2 > g_prof_events.size()) {
        for (int i = 0; i < 256; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            g_prof_events.push_back(e);
        }
    }
    const int ev = (int)g_prof_next_ev;
    g_prof_next_ev += 2;
    if (hipEventRecord(g_prof_events[ev], g_stream) != hipSuccess) return -1;
    g_prof_recs.push_back(ProfRec{family, ev, 0.0, 0.0});
    return (int)g_prof_recs.size() - 1;
}

void prof_end(int idx, double bytes, double flops)
{
    if (idx < 0 || idx >= (int)g_prof_recs.size()) return;
    ProfRec& r = g_prof_recs[idx];
    (void)hipEventRecord(g_prof_events[r.ev + 1], g_stream);
    r.bytes = bytes;
    r.flops = flops;
}

int prof_read(int family, int* launches, double* total_ms, double* bytes, double* flops)
{
    int n = 0;
    double ms = 0, by = 0, fl = 0;
    for (const ProfRec& r : g_prof_recs) {
        if (r.family != family) continue;
        YAO_HIP(hipEventSynchronize(g_prof_events[r.ev + 1]));
        float t = 0;
        YAO_HIP(hipEventElapsedTime(&t, g_prof_events[r.ev], g_prof_events[r.ev + 1]));
        ++n;
        ms += t;
        by += r.bytes;
        fl += r.flops;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    if (bytes) *bytes = by;
    if (flops) *flops = fl;
    return 0;
}

}  // namespace yao
