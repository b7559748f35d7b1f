// Candidate timing for fusion widths and tile sizes.
#include "tuner.h"

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>

#include "driver.h"

namespace yao {

TrialProgram::~TrialProgram()
{
    if (d) (void)hipFree(d);
}

int TrialProgram::load(const Program& p)
{
    const size_t bytes = program_blob_bytes(p);
    std::vector<char> h(bytes);
    if (hipMalloc((void**)&d, bytes) != hipSuccess) return set_error(YAO_ENOMEM, "trial program of %zu bytes", bytes);
    pack_program(p, h.data(), d, dp);
    YAO_HIP(hipMemcpyAsync(d, h.data(), bytes, hipMemcpyHostToDevice, stream()));
    YAO_HIP(hipStreamSynchronize(stream()));
    return 0;
}

int time_runs(int reps, int (*fn)(void*), void* ctx, double* ms)
{
    hipEvent_t e0, e1;
    YAO_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(YAO_EHIP, "hipEventCreate");
    }
    const hipStream_t st = stream();
    int rc = fn(ctx);
    std::vector<double> v;
    for (int r = 0; r < reps && !rc; ++r) {
        if (hipEventRecord(e0, st) != hipSuccess) rc = set_error(YAO_EHIP, "event record");
        if (!rc) rc = fn(ctx);
        if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = set_error(YAO_EHIP, "event record");
        if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = set_error(YAO_EHIP, "event sync");
        float f = 0;
        if (!rc && hipEventElapsedTime(&f, e0, e1) != hipSuccess) rc = set_error(YAO_EHIP, "elapsed time");
        v.push_back(f);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::sort(v.begin(), v.end());
    *ms = v.empty() ? 0.0 : v[v.size() / 2];
    return 0;
}

const yao_circuit* forward_circuit(const yao_circuit* c, const double* params, int width, const double** fparams)
{
    if (width <= 0 || c->gates.empty()) {
        *fparams = params;
        return c;
    }
    *fparams = nullptr;
    return fused_circuit(c, params, width);
}

int time_forward(const yao_circuit* c, const double* params, void* data, int dtype, int n, int B, int width, int tq,
                 double* ms)
{
    // Wall time of the whole sweep (host work for the program included), median of three runs
    // for small states and one for large ones, after one untimed run.
    const int reps = (uint64_t(1) << n) * (uint64_t)B >= (uint64_t(1) << 24) ? 1 : 3;
    struct Suspend {
        Suspend() { jit_suspend(true); }
        ~Suspend() { jit_suspend(false); }
    } suspend;
    YAO_TRY(forward_sweep(data, dtype, n, B, c, params, width, tq, nullptr));
    YAO_HIP(hipStreamSynchronize(stream()));
    std::vector<double> v;
    for (int r = 0; r < reps; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        YAO_TRY(forward_sweep(data, dtype, n, B, c, params, width, tq, nullptr));
        YAO_HIP(hipStreamSynchronize(stream()));
        v.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    std::sort(v.begin(), v.end());
    *ms = v[v.size() / 2];
    return 0;
}

namespace {

using TuneKey = std::tuple<const yao_circuit*, uint64_t, int, int, int, int>;  // c, version, n, B, dtype, mfma
std::map<TuneKey, int> g_width;
std::mutex g_mu;

}  // namespace

int pick_forward_width(const yao_circuit* c, const double* params, void* data, int dtype, int n, int B, int* width)
{
    *width = options().fuse_width;
    if (!options().autotune || c->gates.empty()) return 0;
    const TuneKey key{c, c->version, n, B, dtype, options().mfma};
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_width.find(key);
        if (it != g_width.end()) {
            *width = it->second;
            return 0;
        }
    }
    const size_t bytes = ((size_t)1 << n) * (size_t)B * (dtype == YAO_C64 ? 8 : 16);
    void* save = workspace(WS_TUNE, bytes);
    if (!save) return YAO_ENOMEM;
    const hipStream_t st = stream();
    YAO_HIP(hipMemcpyAsync(save, data, bytes, hipMemcpyDeviceToDevice, st));
    double best = 1e300;
    int bw = 0;
    for (int w = 0; w <= std::min(5, n); ++w) {
        double ms = 0;
        YAO_TRY(time_forward(c, params, data, dtype, n, B, w, options().tile_qubits, &ms));
        if (ms < best) {
            best = ms;
            bw = w;
        }
    }
    YAO_HIP(hipMemcpyAsync(data, save, bytes, hipMemcpyDeviceToDevice, st));
    std::lock_guard<std::mutex> lk(g_mu);
    g_width[key] = bw;
    *width = bw;
    return 0;
}

void drop_tuning(const yao_circuit* c)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_width.begin(); it != g_width.end();) {
        if (std::get<0>(it->first) == c) it = g_width.erase(it);
        else ++it;
    }
}

}  // namespace yao
