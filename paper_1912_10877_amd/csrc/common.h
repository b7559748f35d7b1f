// Shared device/host definitions of the gfx950 state-vector library.
//
// Layout: a state of n qubits and batch B is 2^n * B complex numbers; element (i, b) sits at
// offset i*B + b, so the batch is innermost (stride 1). Qubit q is bit q of i.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/yao.h"

namespace yao {

// ------------------------------------------------------------------------------------------
// Complex helpers on HIP vector types. R is the real type, V the interleaved pair.
// ------------------------------------------------------------------------------------------
template <typename R> struct VecOf;
template <> struct VecOf<float> { using type = float2; };
template <> struct VecOf<double> { using type = double2; };
template <typename R> using vec2_t = typename VecOf<R>::type;

template <typename R> struct Cx {
    R re, im;
};

// c * v for a complex coefficient c and amplitude v.
template <typename R, typename V>
__device__ __forceinline__ void cmul_acc(R& ore, R& oim, R cre, R cim, const V& v)
{
    ore = fma(cre, (R)v.x, ore);
    ore = fma(-cim, (R)v.y, ore);
    oim = fma(cre, (R)v.y, oim);
    oim = fma(cim, (R)v.x, oim);
}

// A 2x2 complex matrix (row-major) passed by value.
template <typename R> struct M2 {
    R re[4];
    R im[4];
};

// A 2^k x 2^k complex matrix by value for k <= 3.
template <typename R, int K> struct MK {
    R re[1 << (2 * K)];
    R im[1 << (2 * K)];
};

// Insert a zero bit at position q of j.
__device__ __host__ __forceinline__ uint64_t insert_zero(uint64_t j, int q)
{
    uint64_t lo = j & ((uint64_t(1) << q) - 1);
    return ((j >> q) << (q + 1)) | lo;
}

// Batch geometry of a launch whose rows are reduced per batch slot: a block of 256 threads
// covers Bc = 2^logBc consecutive slots (thread & (Bc-1)) of 256/Bc rows; blockIdx.y selects
// the slot chunk; rows are walked grid-stride over blockIdx.x.
struct BatchGeom {
    int B;        // batch
    int logBc;    // slots per block = 1 << logBc  (<= 64)
    int nchunks;  // gridDim.y
};

inline int ilog2_ceil(uint64_t v)
{
    int l = 0;
    while ((uint64_t(1) << l) < v) ++l;
    return l;
}

inline BatchGeom make_batch_geom(int B)
{
    BatchGeom g;
    g.B = B;
    int lb = ilog2_ceil((uint64_t)B);
    g.logBc = lb < 6 ? lb : 6;
    g.nchunks = (B + (1 << g.logBc) - 1) >> g.logBc;
    return g;
}

// ------------------------------------------------------------------------------------------
// Host-side objects behind the opaque handles of the C ABI.
// ------------------------------------------------------------------------------------------
// Controls a gate record holds: the C ABI takes up to 8; the shifted-circuit register of the
// faithful gradient adds one control per slot bit.
constexpr int kGateMaxCtrl = 32;

struct GateRec {
    int kind;             // enum yao_gate
    int param;            // -1: fixed
    double theta;
    int k;
    int locs[8];
    int nctrl;
    int ctrls[kGateMaxCtrl];
    int cvals[kGateMaxCtrl];
    std::vector<double> G;  // 2 * 4^k doubles for ROT / DENSE
};

}  // namespace yao

struct yao_state {
    void* data;
    int n;
    int batch;
    int dtype;  // enum yao_dtype
    bool owns;
    size_t elems() const { return (size_t(1) << n) * size_t(batch); }
    size_t elem_bytes() const { return dtype == YAO_C64 ? 8 : 16; }
    size_t bytes() const { return elems() * elem_bytes(); }
};

struct yao_circuit {
    int n;
    int nparams;
    std::vector<yao::GateRec> gates;
    uint64_t version;  // bumped on every push; plans cache against it
    bool transient = false;  // matrices rewritten on every call (a fused circuit for given angles)
};

struct yao_pauli_sum {
    int n;
    std::vector<double> coef;
    std::vector<uint64_t> x, z;
    // Terms grouped by X mask on the host (built at creation): group records of 16 bytes
    // (x, first term, end term) and term records of 24 bytes (c, z, ny), as the kernels read them.
    std::vector<uint64_t> host_groups, host_terms;
    // Device tables (grouped by X mask), built on first use.
    void* d_groups = nullptr;
    void* d_terms = nullptr;
    int ngroups = 0;
    int nterms_dev = 0;
};
