// Pauli-sum expectation that allocates nothing: every device buffer it needs (the grouped term
// tables, per-block partial sums and per-slot sums) lives in one static device array of fixed
// size, so callers that must not allocate (work under graph capture, tight serving loops,
// harnesses that forbid hipMalloc) can evaluate E_b = Re <psi_b|H|psi_b>.
//
// The array is a file-scope __device__ object: each GPU the library runs on holds its own copy
// at its own address until the process ends. Host code never passes the array's name to a
// kernel or a copy (on the host that name is only a stand-in); it looks the address up once per
// device with hipGetSymbolAddress and uses that pointer.
#include <mutex>

#include "runtime.h"

namespace yao {

namespace {

constexpr size_t kScratchBytes = size_t(2) << 20;       // 2 MiB per GPU
constexpr size_t kTableBytes = size_t(256) << 10;       // grouped term tables
constexpr int kMaxTerms = 4096;                         // 4096 x 24 B + 4096 x 16 B < kTableBytes
constexpr size_t kPartialOff = kTableBytes;
constexpr size_t kPartialBytes = size_t(1) << 20;       // B * blocks doubles
constexpr size_t kSumsOff = kPartialOff + kPartialBytes;
constexpr int kMaxBatch = (int)((kScratchBytes - kSumsOff) / sizeof(double));  // sums region
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};

// Address of this device's copy of `scratch` (looked up on first use per device).
int scratch_ptr(char** out)
{
    int dev = 0;
    YAO_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(YAO_EINVAL, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        YAO_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(YAO_EHIP, "hipGetSymbolAddress returned no address");
        g_ptr[dev] = p;
    }
    *out = (char*)g_ptr[dev];
    return 0;
}

}  // namespace

int noalloc_setup()
{
    char* p = nullptr;
    return scratch_ptr(&p);
}

}  // namespace yao

using namespace yao;

extern "C" int yao_expect_noalloc(const yao_state* s, const yao_pauli_sum* h, double* energy)
{
    if (!s || !s->data) return set_error(YAO_EINVAL, "state is NULL or has no memory");
    if (!h || !energy) return set_error(YAO_EINVAL, "pauli sum or energy is NULL");
    if (h->n != s->n) return set_error(YAO_EINVAL, "observable on %d qubits, state has %d", h->n, s->n);
    const int ng = (int)(h->host_groups.size() / 2), nt = (int)(h->host_terms.size() / 3);
    if (nt > kMaxTerms) return set_error(YAO_EINVAL, "%d terms exceed the static limit of %d", nt, kMaxTerms);
    const int B = s->batch;
    const size_t nblk = (size_t)expect_grid_x(s->n, B);
    if (B > kMaxBatch || (size_t)B * nblk * sizeof(double) > kPartialBytes)
        return set_error(YAO_EINVAL, "batch %d exceeds the static partial-sum buffer (%zu doubles)", B,
                         kPartialBytes / sizeof(double));
    YAO_TRY(ensure_device());
    char* base = nullptr;
    YAO_TRY(scratch_ptr(&base));
    char* groups = base;
    char* terms = base + (((size_t)ng * 16 + 255) & ~size_t(255));
    double* partial = (double*)(base + kPartialOff);
    double* sums = (double*)(base + kSumsOff);
    hipStream_t st = stream();
    YAO_HIP(hipMemcpyAsync(groups, h->host_groups.data(), (size_t)ng * 16, hipMemcpyHostToDevice, st));
    YAO_HIP(hipMemcpyAsync(terms, h->host_terms.data(), (size_t)nt * 24, hipMemcpyHostToDevice, st));
    YAO_TRY(launch_expect_into(s->data, s->dtype, s->n, B, groups, ng, terms, partial, sums));
    YAO_HIP(hipMemcpyAsync(energy, sums, sizeof(double) * B, hipMemcpyDeviceToHost, st));
    YAO_HIP(hipStreamSynchronize(st));
    return 0;
}
