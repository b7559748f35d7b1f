// Run-time compiled pass kernels (hipRTC). The generic pass kernels read every op record at run
// time and dispatch on its variant: per op, scalar loads, a compare tree, loop control and, at
// the merge of the variants, register copies. With one wave per SIMD (a 20-qubit state gives
// each CU one 2^12 tile) that scalar work is not hidden behind another wave's vector work. A
// device-bound program's structure (which ops, on which register bits, under which controls)
// is fixed; only its matrices change with the parameters, and they stay in the op records that
// k_bind rewrites. So each pass of such a program can be emitted as straight-line code: the
// tile mapping and the register-group layouts become constants, a SWAP on register bits whose
// controls are register bits is a renaming of registers at compile time (no instructions),
// and the matrix entries are read from the records at constant offsets.
//
// Supported: single-slot states (B = 1), passes whose groups are all register groups (no
// LDS-applied k = 2, 3 ops and no dense blocks); the LDS of a compiled pass is a static
// allocation of the sizes the pass needs. Any other pass of the program runs the generic
// kernel. A compile failure switches the program back to the generic kernels for good.
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstdio>
#include <atomic>
#include <cstddef>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "fused.h"

namespace yao {

namespace {

std::string I(long long v)
{
    return std::to_string(v);
}
std::string U(unsigned long long v)
{
    return std::to_string(v) + "ull";
}

// Bank swizzle of LDS tile rows, the generic kernels' layout (linear over GF(2): the swizzle
// of a ^ b is the XOR of the swizzles).
uint32_t swz_host(uint32_t e)
{
    return e ^ (((e >> 4) ^ (e >> 8)) & 15u);
}

// Pointers in the generated code carry their address space: global memory for states and
// partials (global instead of flat loads) and constant for the op records (scalar loads).
const char* kPrelude = R"YAO(
typedef unsigned long long u64;
#define GLB __attribute__((address_space(1)))
#define CST __attribute__((address_space(4)))
__device__ __forceinline__ unsigned swz(unsigned e) { return e ^ (((e >> 4) ^ (e >> 8)) & 15u); }
)YAO";

// Code of one forward pass, or an empty string when the pass is not supported.
std::string gen_forward_pass(const Plan& P, const Program& prog, int p, int n, int dtype, const std::string& name,
                             int* nthr_out, size_t* lds_out)
{
    const HostPass& pass = P.passes[p];
    const int RB = P.reg_bits, N = 1 << RB, t = P.t;
    if (P.c != 0 || pass.standalone >= 0 || prog.pass_dmat_words[p] != 0) return "";
    if (t - RB < 0 || t - RB > 9 || (int)pass.tile_qubits.size() != t) return "";
    const int g0 = prog.pass_group0[p], ng = (int)pass.groups.size();
    for (int g = 0; g < ng; ++g)
        if (prog.groups[g0 + g].lds) return "";
    const bool c64 = dtype == YAO_C64;
    const size_t lds = (size_t)(c64 ? 8 : 16) << t;
    if (lds > 160 * 1024) return "";
    const int nthr = 1 << (t - RB);
    const std::string V = c64 ? "float2" : "double2", R = c64 ? "float" : "double";
    const std::string MK = c64 ? "make_float2" : "make_double2";
    std::ostringstream o;
    o << "extern \"C\" __global__ void __launch_bounds__(" << nthr << ") " << name
      << "(void* psi_, const char* ops_, const char* zs_, int op_first) {\n";
    // LDS sized at compile time (static allocations may exceed the 64 KiB of a dynamic one):
    // the tile, and the pass's one-qubit matrices (8 entries per record), copied in with the
    // tile so that the ops read them from LDS instead of waiting on a scalar load each.
    const int nrec = prog.pass_nops[p];
    o << "  __shared__ __align__(16) " << V << " lp[" << (1 << t) << "];\n";
    o << "  __shared__ __align__(16) " << R << " um[" << std::max(1, nrec) * 8 << "];\n";
    o << "  const unsigned th = threadIdx.x;\n";
    o << "  GLB " << V << "* gp = (GLB " << V << "*)psi_;\n  const CST char* ops = (const CST char*)ops_;\n";
    o << "  if (zs_) { const CST u64* z = (const CST u64*)(zs_ + 32 * blockIdx.z); gp = (GLB " << V
      << "*)z[0]; ops = (const CST char*)z[2] + (u64)op_first * " << sizeof(POp) << "; }\n";
    // Tile base: the tile index bits on the qubits outside the tile, ascending.
    uint64_t T = 0;
    for (int q : pass.tile_qubits) T |= uint64_t(1) << q;
    o << "  const u64 tid = blockIdx.x;\n  u64 base = 0;\n";
    {
        int j = 0;
        for (int q = 0; q < n; ++q) {
            if ((T >> q) & 1) continue;
            o << "  base |= ((tid >> " << j << ") & 1ull) << " << q << ";\n";
            ++j;
        }
    }
    // Load mapping: element e = th + r * nthr; bits of th on tile qubits 0 .. t-RB-1, bits of r
    // on the next RB tile qubits.
    o << "  u64 toff = base;\n";
    for (int j = 0; j < t - RB; ++j) o << "  toff |= (u64)((th >> " << j << ") & 1u) << " << pass.tile_qubits[j] << ";\n";
    std::vector<uint64_t> rofs(N);
    for (int r = 0; r < N; ++r) {
        uint64_t d = 0;
        for (int b = 0; b < RB; ++b)
            if ((r >> b) & 1) d |= uint64_t(1) << pass.tile_qubits[t - RB + b];
        rofs[r] = d;
    }
    o << "  {\n";
    for (int r = 0; r < N; ++r) o << "    const " << V << " v" << r << " = gp[toff | " << U(rofs[r]) << "];\n";
    {
        const int W = c64 ? 8 : 16;  // dwords of a record's matrix
        o << "    { const CST unsigned* src = (const CST unsigned*)ops; unsigned* dst = (unsigned*)um;\n"
          << "      for (unsigned i = th; i < " << nrec * W << "u; i += " << nthr << "u) dst[i] = src[(i / " << W << "u) * "
          << sizeof(POp) / 4 << "u + " << offsetof(POp, u) / 4 << "u + i % " << W << "u]; }\n";
    }
    for (int r = 0; r < N; ++r) o << "    lp[swz(th + " << r * nthr << "u)] = v" << r << ";\n";
    o << "  }\n  __syncthreads();\n";
    // Register groups (records are addressed relative to the pass's first record).
    for (int g = 0; g < ng; ++g) {
        const PGroupDesc& G = prog.groups[g0 + g];
        uint32_t rmask = 0;
        for (int j = 0; j < RB; ++j) rmask |= 1u << G.rpos[j];
        std::vector<uint32_t> er(N);
        for (int r = 0; r < N; ++r) {
            uint32_t e = 0;
            for (int j = 0; j < RB; ++j)
                if ((r >> j) & 1) e |= 1u << G.rpos[j];
            er[r] = e;
        }
        o << "  {\n    unsigned ethr = 0;\n";
        {
            int k = 0;
            for (int b = 0; b < t; ++b) {
                if ((rmask >> b) & 1) continue;
                o << "    ethr |= ((th >> " << k << ") & 1u) << " << b << ";\n";
                ++k;
            }
        }
        o << "    const unsigned sw = swz(ethr);\n";
        std::vector<int> perm(N);
        for (int r = 0; r < N; ++r) {
            perm[r] = r;
            o << "    " << V << " x" << r << " = lp[sw ^ " << swz_host(er[r]) << "u];\n";
        }
        for (int i = 0; i < G.nops; ++i) {
            const int oi = G.op0 + i;
            const POp& op = prog.ops[prog.pass_op0[p] + oi];
            const int J = op.rpos;
            const int cls = op.var / RB;
            const uint32_t tm = op.cmask & ~rmask, rm = op.cmask & rmask;
            // Generic class: the outer controls decide per tile; fast classes have none.
            const bool outer = cls >= kFwdGenericClass && op.omask != 0;
            const bool swap = cls == 3;
            const bool lane_pred = (cls == 3 || cls >= kFwdGenericClass) && tm != 0;
            const bool cond = lane_pred || outer;
            o << "    {\n";
            if (!swap) o << "      const " << R << "* u = um + " << oi * 8 << ";\n";
            if (cond) {
                o << "      const bool pc = true";
                if (lane_pred) o << " && ((ethr & " << tm << "u) == " << (op.cval & tm) << "u)";
                if (outer) o << " && ((base & " << U(op.omask) << ") == " << U(op.oval) << ")";
                o << ";\n";
            }
            for (int a = 0; a < N; ++a) {
                if ((a >> J) & 1) continue;
                if ((cls == 3 || cls >= kFwdGenericClass) && (er[a] & rm) != (op.cval & rm)) continue;
                const std::string X = "x" + I(perm[a]), Y = "x" + I(perm[a | (1 << J)]);
                if (swap) {
                    if (!cond) {
                        std::swap(perm[a], perm[a | (1 << J)]);
                    } else {
                        o << "      { const " << V << " p = " << X << ", q = " << Y << "; " << X << " = pc ? q : p; " << Y
                          << " = pc ? p : q; }\n";
                    }
                    continue;
                }
                std::string np, nq;
                if (cls == 0) {  // (c a + i s b, i s a + c b), c = u[0], s = u[5]
                    np = MK + "(u[0] * p.x - u[5] * q.y, u[0] * p.y + u[5] * q.x)";
                    nq = MK + "(u[0] * q.x - u[5] * p.y, u[0] * q.y + u[5] * p.x)";
                } else if (cls == 1) {  // diag(u0 + i u4, u3 + i u7)
                    np = MK + "(u[0] * p.x - u[4] * p.y, u[0] * p.y + u[4] * p.x)";
                    nq = MK + "(u[3] * q.x - u[7] * q.y, u[3] * q.y + u[7] * q.x)";
                } else {  // dense: mr = u[0..3], mi = u[4..7], row-major
                    np = MK + "(u[0] * p.x - u[4] * p.y + u[1] * q.x - u[5] * q.y, u[0] * p.y + u[4] * p.x + u[1] * q.y + u[5] * q.x)";
                    nq = MK + "(u[2] * p.x - u[6] * p.y + u[3] * q.x - u[7] * q.y, u[2] * p.y + u[6] * p.x + u[3] * q.y + u[7] * q.x)";
                }
                o << "      { const " << V << " p = " << X << ", q = " << Y << "; ";
                if (cond) o << X << " = pc ? " << np << " : p; " << Y << " = pc ? " << nq << " : q; }\n";
                else o << X << " = " << np << "; " << Y << " = " << nq << "; }\n";
            }
            o << "    }\n";
        }
        for (int r = 0; r < N; ++r) o << "    lp[sw ^ " << swz_host(er[r]) << "u] = x" << perm[r] << ";\n";
        o << "  }\n  __syncthreads();\n";
    }
    // Store: element e = th + r * nthr of the stored tile comes from LDS tile element
    // sth | sreg[r], thread bit i moving to tile bit store_src[i].
    o << "  unsigned sth = 0;\n";
    for (int i = 0; i < t - RB; ++i) {
        const int src = pass.store_src.empty() ? i : pass.store_src[i];
        o << "  sth |= ((th >> " << i << ") & 1u) << " << src << ";\n";
    }
    o << "  const unsigned ssw = swz(sth);\n";
    for (int r = 0; r < N; ++r) {
        uint32_t v = 0;
        for (int j = 0; j < RB; ++j)
            if ((r >> j) & 1) v |= 1u << (pass.store_src.empty() ? t - RB + j : pass.store_src[t - RB + j]);
        o << "  gp[toff | " << U(rofs[r]) << "] = lp[ssw ^ " << swz_host(v) << "u];\n";
    }
    o << "}\n";
    *nthr_out = nthr;
    *lds_out = lds;
    return o.str();
}

// Gradient term of one pair for generator class gen (Re or Im of lambda^dagger M psi on the
// pair, the generic kernels' formulas): p0, p1 psi and l0, l1 lambda of the pair.
std::string grad_expr(int gen, const std::string& p0, const std::string& p1, const std::string& l0,
                      const std::string& l1)
{
    switch (gen) {
    case GEN_X: return "fma(" + l0 + ".x, " + p1 + ".y, fma(-" + l0 + ".y, " + p1 + ".x, fma(" + l1 + ".x, " + p0 + ".y, -" + l1 + ".y * " + p0 + ".x)))";
    case GEN_Y: return "fma(" + l1 + ".x, " + p0 + ".x, fma(" + l1 + ".y, " + p0 + ".y, fma(-" + l0 + ".x, " + p1 + ".x, -" + l0 + ".y * " + p1 + ".y)))";
    case GEN_Z: return "fma(" + l0 + ".x, " + p0 + ".y, fma(-" + l0 + ".y, " + p0 + ".x, fma(-" + l1 + ".x, " + p1 + ".y, " + l1 + ".y * " + p1 + ".x)))";
    case GEN_P1: return "(-2.0 * fma(" + l1 + ".x, " + p1 + ".y, -" + l1 + ".y * " + p1 + ".x))";
    default:
        return "dense_grad(gm, " + p0 + ", " + p1 + ", " + l0 + ", " + l1 + ")";
    }
}

const char* kBwdPrelude = R"YAO(
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v)
{
    const u64 b = __builtin_bit_cast(u64, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((u64)hi << 32) | lo);
}
// Sum over the 16 lanes of a DPP row (single-slot tiles): lane 0 of the row holds it.
__device__ __forceinline__ double row_sum16(double v)
{
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x124>(v);
    v += dpp_f64<0x128>(v);
    return v;
}
// Exchanges two double2 registers in place (v_swap_b32 on each 32-bit half), so that a swap
// under a lane mask needs neither selects nor copies where the lanes rejoin.
__device__ __forceinline__ void swap_d2(double2& a, double2& b)
{
    unsigned* x = reinterpret_cast<unsigned*>(&a);
    unsigned* y = reinterpret_cast<unsigned*>(&b);
    asm volatile("v_swap_b32 %0, %1\n\tv_swap_b32 %2, %3\n\tv_swap_b32 %4, %5\n\tv_swap_b32 %6, %7"
                 : "+v"(x[0]), "+v"(y[0]), "+v"(x[1]), "+v"(y[1]), "+v"(x[2]), "+v"(y[2]), "+v"(x[3]), "+v"(y[3]));
}
// 2 Re(conj(l) M p) for a dense 2 x 2 generator M (re[4], im[4], row-major).
__device__ __forceinline__ double dense_grad(const CST double* m, double2 p0, double2 p1, double2 l0, double2 l1)
{
    const double m0x = m[0] * p0.x - m[4] * p0.y + m[1] * p1.x - m[5] * p1.y;
    const double m0y = m[0] * p0.y + m[4] * p0.x + m[1] * p1.y + m[5] * p1.x;
    const double m1x = m[2] * p0.x - m[6] * p0.y + m[3] * p1.x - m[7] * p1.y;
    const double m1y = m[2] * p0.y + m[6] * p0.x + m[3] * p1.y + m[7] * p1.x;
    return 2.0 * (l0.x * m0x + l0.y * m0y + l1.x * m1x + l1.y * m1y);
}
)YAO";

// Code of one reverse pass (psi in FP64, lambda in the state's precision), or an empty
// string when the pass is not supported.
std::string gen_backward_pass(const Plan& P, const Program& prog, int p, int n, int dtype, const std::string& name,
                              int* nthr_out, size_t* lds_out)
{
    const HostPass& pass = P.passes[p];
    const int RB = P.reg_bits, N = 1 << RB, t = P.t;
    if (P.c != 0 || pass.standalone >= 0) return "";
    if (t - RB < 4 || t - RB > 9 || (int)pass.tile_qubits.size() != t) return "";
    const int g0 = prog.pass_group0[p], ng = (int)pass.groups.size();
    int maxslots = 0;
    for (int g = 0; g < ng; ++g) {
        if (prog.groups[g0 + g].lds) return "";
        maxslots = std::max(maxslots, prog.groups[g0 + g].nslot);
    }
    const bool c64 = dtype == YAO_C64;
    const int nthr = 1 << (t - RB);
    const int lb = c64 ? 8 : 16;
    // Gradient partials: each gradient is summed over lane pairs (one DPP step) and the pair sums
    // go to LDS, E = nthr / 2 entries per gradient, two buffers of the group's gradients; when
    // that does not fit, over rows of 16 lanes (E = nthr / 16).
    auto lds_for = [&](int e) {
        return ((size_t)(16 + lb) << t) + sizeof(double) * 2 * (size_t)std::max(1, maxslots) * e;
    };
    const int red_lanes = lds_for(nthr >> 1) <= 160 * 1024 ? 2 : 16;
    const int E = nthr / red_lanes;
    const size_t lds = lds_for(E);
    if (lds > 160 * 1024) return "";
    const std::string VL = c64 ? "float2" : "double2", RL = c64 ? "float" : "double";
    std::ostringstream o;
    // Workgroups per CU that the LDS allows; when that is more than the registers would
    // allow at the compiler's choice, ask for the register budget that fits them.
    const int wg_lds = (int)std::min<size_t>(8, (160 * 1024) / lds);
    const int waves = std::max(1, wg_lds * (nthr / 64) / 4);  // per SIMD
    o << "extern \"C\" __global__ void __launch_bounds__(" << nthr << ") __attribute__((amdgpu_waves_per_eu("
      << std::min(waves, 8) << "))) " << name
      << "(void* psi_, void* lam_, const char* ops_, const double* mats, double* gpart_, const char* zs_, int op_first, "
         "int pstride) {\n";
    o << "  __shared__ __align__(16) unsigned char smem[" << lds << "];\n";
    o << "  double2* lp = (double2*)smem;\n  " << VL << "* ll = (" << VL << "*)(smem + " << (16 << t) << ");\n";
    o << "  double* red0 = (double*)(smem + " << ((16 + lb) << t) << ");\n";
    o << "  const unsigned th = threadIdx.x;\n";
    o << "  GLB double2* gp = (GLB double2*)psi_;\n  GLB " << VL << "* gl = (GLB " << VL << "*)lam_;\n";
    o << "  const CST char* ops = (const CST char*)ops_;\n  GLB double* gpart = (GLB double*)gpart_;\n";
    o << "  if (zs_) { const CST u64* z = (const CST u64*)(zs_ + 32 * blockIdx.z); gp = (GLB double2*)z[0]; gl = (GLB "
      << VL << "*)z[1]; ops = (const CST char*)z[2] + (u64)op_first * " << sizeof(POp)
      << "; gpart = (GLB double*)z[3]; }\n";
    uint64_t T = 0;
    for (int q : pass.tile_qubits) T |= uint64_t(1) << q;
    o << "  const u64 tid = blockIdx.x;\n  u64 base = 0;\n";
    {
        int j = 0;
        for (int q = 0; q < n; ++q) {
            if ((T >> q) & 1) continue;
            o << "  base |= ((tid >> " << j << ") & 1ull) << " << q << ";\n";
            ++j;
        }
    }
    o << "  u64 toff = base;\n";
    for (int j = 0; j < t - RB; ++j) o << "  toff |= (u64)((th >> " << j << ") & 1u) << " << pass.tile_qubits[j] << ";\n";
    std::vector<uint64_t> rofs(N);
    for (int r = 0; r < N; ++r) {
        uint64_t d = 0;
        for (int b = 0; b < RB; ++b)
            if ((r >> b) & 1) d |= uint64_t(1) << pass.tile_qubits[t - RB + b];
        rofs[r] = d;
    }
    o << "  {\n";
    for (int r = 0; r < N; ++r)
        o << "    const double2 v" << r << " = gp[toff | " << U(rofs[r]) << "]; const " << VL << " w" << r << " = gl[toff | "
          << U(rofs[r]) << "];\n";
    for (int r = 0; r < N; ++r)
        o << "    lp[swz(th + " << r * nthr << "u)] = v" << r << "; ll[swz(th + " << r * nthr << "u)] = w" << r << ";\n";
    o << "  }\n  __syncthreads();\n";
    o << "  double phr = 1.0, phi = 0.0;\n";
    // Matrix entries each op reads (cls 0: u0, u5; cls 1: u3, u7 and the phase's u0, u4;
    // swaps none; generic: all eight). They come through the scalar cache a batch ahead:
    // batches of up to 8 consecutive ops (at most 16 entries); at the first op of batch b the
    // kernel waits for batch b's loads and issues batch b + 1's, so records that miss the
    // scalar cache are fetched while batch b computes. The loads are volatile so that the
    // compiler keeps them where they are issued instead of next to their uses.
    std::vector<std::pair<int, int>> seq;  // (group, op within group) in pass order
    for (int g = 0; g < ng; ++g)
        for (int i = 0; i < prog.groups[g0 + g].nops; ++i) seq.push_back({g, i});
    auto coeffs = [&](int oi) -> std::vector<int> {
        const int cls = prog.ops[prog.pass_op0[p] + oi].var / RB;
        if (cls == 0) return {0, 5};
        if (cls == 1) return {3, 7, 0, 4};
        if (cls == 2) return {};
        return {0, 1, 2, 3, 4, 5, 6, 7};
    };
    auto op_index = [&](size_t i) { return prog.groups[g0 + seq[i].first].op0 + seq[i].second; };
    std::vector<size_t> batch_first;  // first op (in seq) of each batch
    {
        int cnt = 0, ent = 0;
        for (size_t i = 0; i < seq.size(); ++i) {
            const int c = (int)coeffs(op_index(i)).size();
            if (batch_first.empty() || cnt == 8 || ent + c > 16) {
                batch_first.push_back(i);
                cnt = 0;
                ent = 0;
            }
            ++cnt;
            ent += c;
        }
        batch_first.push_back(seq.size());
    }
    auto emit_loads = [&](size_t b) {
        if (b + 1 >= batch_first.size()) return;
        for (size_t i = batch_first[b]; i < batch_first[b + 1]; ++i)
            for (int k : coeffs(op_index(i)))
                o << "    U" << i << "_" << k << " = ((const volatile CST double*)(ops + "
                  << (size_t)op_index(i) * sizeof(POp) + offsetof(POp, u) << "))[" << k << "];\n";
    };
    for (size_t i = 0; i < seq.size(); ++i)
        for (int k : coeffs(op_index(i))) o << "  double U" << i << "_" << k << ";\n";
    size_t si = 0, bi = 0;
    emit_loads(0);
    int buf = 0;
    for (int g = 0; g < ng; ++g) {
        const PGroupDesc& G = prog.groups[g0 + g];
        uint32_t rmask = 0;
        for (int j = 0; j < RB; ++j) rmask |= 1u << G.rpos[j];
        std::vector<uint32_t> er(N);
        for (int r = 0; r < N; ++r) {
            uint32_t e = 0;
            for (int j = 0; j < RB; ++j)
                if ((r >> j) & 1) e |= 1u << G.rpos[j];
            er[r] = e;
        }
        o << "  {\n    unsigned ethr = 0;\n";
        {
            int k = 0;
            for (int b = 0; b < t; ++b) {
                if ((rmask >> b) & 1) continue;
                o << "    ethr |= ((th >> " << k << ") & 1u) << " << b << ";\n";
                ++k;
            }
        }
        o << "    const unsigned sw = swz(ethr);\n";
        o << "    double* red = red0 + " << buf * std::max(1, maxslots) * E << ";\n";
        std::vector<int> perm(N);
        for (int r = 0; r < N; ++r) {
            perm[r] = r;
            o << "    double2 x" << r << " = lp[sw ^ " << swz_host(er[r]) << "u]; double2 y" << r << "; { const " << VL
              << " q = ll[sw ^ " << swz_host(er[r]) << "u]; y" << r << " = make_double2((double)q.x, (double)q.y); }\n";
        }
        int nslot = 0;
        for (int i = 0; i < G.nops; ++i) {
            const int oi = G.op0 + i;
            const POp& op = prog.ops[prog.pass_op0[p] + oi];
            const int J = op.rpos;
            const int cls = op.var / RB;
            const uint32_t tm = op.cmask & ~rmask, rm = op.cmask & rmask;
            const bool generic = cls >= kBwdGenericClass;
            const bool outer = generic && op.omask != 0;
            const bool lane_pred = (cls == 2 || generic) && tm != 0;
            const bool cond = lane_pred || outer;
            // Reverse ops read their matrices through the scalar cache (in LDS they would occupy
            // VGPRs, and the reverse kernel has none to spare), prefetched one op ahead.
            if (si == batch_first[bi]) {
                o << "    __builtin_amdgcn_s_waitcnt(0xC07F);\n    __builtin_amdgcn_sched_barrier(0);\n";
                emit_loads(++bi);
                o << "    __builtin_amdgcn_sched_barrier(0);\n";
            }
            const size_t cur = si++;
            std::ostringstream enclosing;
            std::swap(o, enclosing);  // the op's code goes to its own stream first
            o << "    {\n";
            if (generic && op.slot >= 0 && op.gen == GEN_DENSE)
                o << "      const CST double* gm = (const CST double*)mats + " << op.mat + 8 << ";\n";
            if (cond) {
                o << "      const bool pc = true";
                if (lane_pred) o << " && ((ethr & " << tm << "u) == " << (op.cval & tm) << "u)";
                if (outer) o << " && ((base & " << U(op.omask) << ") == " << U(op.oval) << ")";
                o << ";\n";
            }
            // Pairs whose register-bit controls hold.
            std::vector<int> pairs;
            for (int a = 0; a < N; ++a) {
                if ((a >> J) & 1) continue;
                if ((cls == 2 || generic) && (er[a] & rm) != (op.cval & rm)) continue;
                pairs.push_back(a);
            }
            // Gradient from psi and lambda before the update.
            if (op.slot >= 0) {
                const int gen = cls == 0 ? GEN_X : cls == 1 ? GEN_Z : op.gen;
                o << "      double g = 0.0;\n";
                for (int a : pairs) {
                    const std::string e = grad_expr(gen, "x" + I(perm[a]), "x" + I(perm[a | (1 << J)]), "y" + I(perm[a]),
                                                    "y" + I(perm[a | (1 << J)]));
                    if (cond) o << "      g += pc ? " << e << " : 0.0;\n";
                    else o << "      g += " << e << ";\n";
                }
                if (red_lanes == 2)
                    o << "      g += dpp_f64<0xB1>(g);\n      if ((th & 1u) == 0) red[" << nslot * E << " + (th >> 1)] = g;\n";
                else
                    o << "      g = row_sum16(g);\n      if ((th & 15u) == 0) red[" << nslot * E << " + (th >> 4)] = g;\n";
                ++nslot;
            }
            for (int a : pairs) {
                const std::string X = "x" + I(perm[a]), Y = "x" + I(perm[a | (1 << J)]);
                const std::string LX = "y" + I(perm[a]), LY = "y" + I(perm[a | (1 << J)]);
                if (cls == 2) {
                    if (!cond) {
                        std::swap(perm[a], perm[a | (1 << J)]);
                    } else {
                        // Swapped in place under the lane mask: one branch around the op's pairs,
                        // no selects and no copies where the lanes rejoin.
                        if (a == pairs.front()) o << "      if (pc) {\n";
                        o << "        swap_d2(" << X << ", " << Y << "); swap_d2(" << LX << ", " << LY << ");\n";
                        if (a == pairs.back()) o << "      }\n";
                    }
                    continue;
                }
                for (const auto& pr : {std::make_pair(X, Y), std::make_pair(LX, LY)}) {
                    const std::string& A = pr.first;
                    const std::string& B = pr.second;
                    if (cls == 0) {  // (c a + i s b, i s a + c b)
                        o << "      { const double2 p = " << A << ", q = " << B << "; " << A
                          << " = make_double2(u[0] * p.x - u[5] * q.y, u[0] * p.y + u[5] * q.x); " << B
                          << " = make_double2(u[0] * q.x - u[5] * p.y, u[0] * q.y + u[5] * p.x); }\n";
                    } else if (cls == 1) {  // diag(1, u3 + i u7); the first entry goes to the phase
                        o << "      { const double2 q = " << B << "; " << B
                          << " = make_double2(u[3] * q.x - u[7] * q.y, u[3] * q.y + u[7] * q.x); }\n";
                    } else {
                        const std::string np = "make_double2(u[0] * p.x - u[4] * p.y + u[1] * q.x - u[5] * q.y, u[0] * p.y + u[4] * p.x + u[1] * q.y + u[5] * q.x)";
                        const std::string nq = "make_double2(u[2] * p.x - u[6] * p.y + u[3] * q.x - u[7] * q.y, u[2] * p.y + u[6] * p.x + u[3] * q.y + u[7] * q.x)";
                        o << "      { const double2 p = " << A << ", q = " << B << "; ";
                        if (cond) o << A << " = pc ? " << np << " : p; " << B << " = pc ? " << nq << " : q; }\n";
                        else o << A << " = " << np << "; " << B << " = " << nq << "; }\n";
                    }
                }
            }
            if (cls == 1) o << "      { const double pr = phr * u[0] - phi * u[4]; phi = phr * u[4] + phi * u[0]; phr = pr; }\n";
            o << "    }\n";
            // The op's u[k] are the prefetched U<cur>_k.
            std::string body = o.str();
            for (int k = 0; k < 8; ++k) {
                const std::string from = "u[" + I(k) + "]", to = "U" + I((long long)cur) + "_" + I(k);
                for (size_t pos = body.find(from); pos != std::string::npos; pos = body.find(from, pos + to.size()))
                    body.replace(pos, from.size(), to);
            }
            std::swap(o, enclosing);
            o << body;
        }
        if (nslot != G.nslot) return "";  // the record's slots and the group's list disagree
        for (int r = 0; r < N; ++r)
            o << "    lp[sw ^ " << swz_host(er[r]) << "u] = x" << perm[r] << "; ll[sw ^ " << swz_host(er[r]) << "u] = make_"
              << VL << "((" << RL << ")y" << perm[r] << ".x, (" << RL << ")y" << perm[r] << ".y);\n";
        o << "  }\n  __syncthreads();\n";
        if (nslot > 0) {
            // Partials of each gradient over the tile: 16 tasks per gradient, E entries each.
            o << "  {\n    const double* red = red0 + " << buf * std::max(1, maxslots) * E << ";\n";
            o << "    for (unsigned task = th; task < " << nslot * 16 << "u; task += " << nthr << "u) {\n";
            o << "      const unsigned s = task >> 4, j = task & 15u;\n      double v = 0.0;\n";
            o << "      for (unsigned e = j; e < " << E << "u; e += 16u) v += red[s * " << E << "u + e];\n";
            o << "      for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off, 16);\n";
            o << "      int slot = " << G.slots[0] << ";\n";
            for (int k = 1; k < nslot; ++k) o << "      if (s == " << k << "u) slot = " << G.slots[k] << ";\n";
            o << "      if (j == 0) gpart[(u64)slot * (u64)pstride + blockIdx.x] = v;\n    }\n  }\n";
            buf ^= 1;
        }
    }
    // Store with the accumulated phase.
    o << "  unsigned sth = 0;\n";
    for (int i = 0; i < t - RB; ++i) {
        const int src = pass.store_src.empty() ? i : pass.store_src[i];
        o << "  sth |= ((th >> " << i << ") & 1u) << " << src << ";\n";
    }
    o << "  const unsigned ssw = swz(sth);\n";
    for (int r = 0; r < N; ++r) {
        uint32_t v = 0;
        for (int j = 0; j < RB; ++j)
            if ((r >> j) & 1) v |= 1u << (pass.store_src.empty() ? t - RB + j : pass.store_src[t - RB + j]);
        o << "  { const double2 v = lp[ssw ^ " << swz_host(v) << "u]; const " << VL << " w = ll[ssw ^ " << swz_host(v)
          << "u]; const double wx = (double)w.x, wy = (double)w.y;\n";
        o << "    gp[toff | " << U(rofs[r]) << "] = make_double2(phr * v.x - phi * v.y, phr * v.y + phi * v.x);\n";
        o << "    gl[toff | " << U(rofs[r]) << "] = make_" << VL << "((" << RL << ")(phr * wx - phi * wy), (" << RL
          << ")(phr * wy + phi * wx)); }\n";
    }
    o << "}\n";
    *nthr_out = nthr;
    *lds_out = lds;
    return o.str();
}

std::mutex g_jit_mu;
int g_suspend = 0;
std::atomic<long long> g_compiled_programs{0}, g_compiled_passes{0}, g_failures{0};
std::atomic<long long> g_launches_fwd{0}, g_launches_bwd{0};

// A program that could not be compiled keeps the generic kernels; say why, once per program.
void report_failure(const char* what, const std::string& detail)
{
    ++g_failures;
    fprintf(stderr, "yao: run-time compiled passes unavailable (%s): %.300s; using the generic kernels\n", what,
            detail.c_str());
}

}  // namespace

struct JitPasses {
    std::vector<hipModule_t> mod;   // per pass
    std::vector<hipFunction_t> fn;  // per pass; null: the generic kernel
    std::vector<int> nthr;
    std::vector<size_t> lds;
    std::vector<int> ntiles;
};

void jit_suspend(bool on)
{
    std::lock_guard<std::mutex> lk(g_jit_mu);
    g_suspend += on ? 1 : -1;
}

namespace {

// Source of each supported pass of a program (empty for passes left to the generic kernel),
// every pass a program of its own so that the passes compile in parallel.
int jit_source(const Plan& P, const Program& prog, bool bwd, int dtype, int n, std::vector<std::string>& src,
               std::vector<int>& nthr, std::vector<size_t>& lds)
{
    src.assign(P.passes.size(), "");
    nthr.assign(P.passes.size(), 0);
    lds.assign(P.passes.size(), 0);
    int count = 0;
    for (size_t p = 0; p < P.passes.size(); ++p) {
        const std::string code = bwd ? gen_backward_pass(P, prog, (int)p, n, dtype, "yao_pass_bwd", &nthr[p], &lds[p])
                                     : gen_forward_pass(P, prog, (int)p, n, dtype, "yao_pass_fwd", &nthr[p], &lds[p]);
        if (code.empty()) continue;
        src[p] = std::string(kPrelude) + (bwd ? kBwdPrelude : "") + code;
        ++count;
    }
    return count;
}

// Compile the non-empty sources on a few host threads; code[p] stays empty for a failure, and
// logs[p] then holds the compiler log.
std::vector<char> jit_build(const std::string& src, std::string* log);
void jit_build_all(const std::vector<std::string>& src, std::vector<std::vector<char>>& code,
                   std::vector<std::string>& logs)
{
    code.assign(src.size(), {});
    logs.assign(src.size(), "");
    std::atomic<size_t> next{0};
    auto work = [&] {
        for (size_t p; (p = next.fetch_add(1)) < src.size();)
            if (!src[p].empty()) code[p] = jit_build(src[p], &logs[p]);
    };
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned i = 1; i < hw && i < src.size(); ++i) th.emplace_back(work);
    work();
    for (std::thread& x : th) x.join();
}

// hipRTC compile for gfx950 with the library's own code-generation flags. Returns the code
// object, or an empty vector with the compiler log in *log.
std::vector<char> jit_build(const std::string& src, std::string* log)
{
    std::vector<char> code;
    hiprtcProgram rp;
    if (hiprtcCreateProgram(&rp, src.c_str(), "yao_pass.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        if (log) *log = "hiprtcCreateProgram failed";
        return code;
    }
    // The load/store vectorizer finds nothing to merge here (LDS rows are XOR-swizzled, tile
    // rows far apart) and costs a sixth of the compile time.
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-ffp-contract=fast", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-load-store-vectorizer=false"};
    if (hiprtcCompileProgram(rp, (int)(sizeof(opts) / sizeof(opts[0])), opts) == HIPRTC_SUCCESS) {
        size_t cs = 0;
        if (hiprtcGetCodeSize(rp, &cs) == HIPRTC_SUCCESS && cs > 0) {
            code.resize(cs);
            if (hiprtcGetCode(rp, code.data()) != HIPRTC_SUCCESS) code.clear();
        }
    } else if (log) {
        size_t ls = 0;
        if (hiprtcGetProgramLogSize(rp, &ls) == HIPRTC_SUCCESS && ls > 0) {
            std::string l(ls, '\0');
            if (hiprtcGetProgramLog(rp, &l[0]) == HIPRTC_SUCCESS) *log = l;
        }
    }
    (void)hiprtcDestroyProgram(&rp);
    return code;
}

}  // namespace

// Compile every supported pass of a bound program into one module. Returns nullptr (and
// leaves the program on the generic kernels) when nothing is supported or compiling fails.
static JitPasses* jit_compile(const Plan& P, const Program& prog, bool bwd, int dtype, int n)
{
    std::vector<std::string> src, logs;
    std::vector<int> nthr;
    std::vector<size_t> lds;
    if (jit_source(P, prog, bwd, dtype, n, src, nthr, lds) == 0) return nullptr;
    std::vector<std::vector<char>> code;
    jit_build_all(src, code, logs);
    for (size_t p = 0; p < src.size(); ++p)
        if (!src[p].empty() && code[p].empty()) {
            report_failure("compile", logs[p]);
            return nullptr;
        }
    JitPasses* J = new JitPasses;
    J->mod.assign(P.passes.size(), nullptr);
    J->fn.assign(P.passes.size(), nullptr);
    J->nthr = nthr;
    J->lds = lds;
    J->ntiles.assign(P.passes.size(), 0);
    for (size_t p = 0; p < P.passes.size(); ++p) {
        if (code[p].empty()) continue;
        hipError_t e = hipModuleLoadData(&J->mod[p], code[p].data());
        if (e == hipSuccess) e = hipModuleGetFunction(&J->fn[p], J->mod[p], bwd ? "yao_pass_bwd" : "yao_pass_fwd");
        if (e != hipSuccess) {
            report_failure("module load", hipGetErrorString(e));
            jit_free(J);
            return nullptr;
        }
        J->ntiles[p] = 1 << (n - P.t);
        ++g_compiled_passes;
    }
    ++g_compiled_programs;
    return J;
}

const JitPasses* jit_passes(const BoundProgram* bp, const Plan& P, bool bwd, int dtype, int n, int B)
{
    if (!bp || B != 1) return nullptr;
    const int when = options().jit;
    std::lock_guard<std::mutex> lk(g_jit_mu);
    if (bp->jit || bp->jit_failed) return bp->jit;
    if (when <= 0 || g_suspend > 0 || recording()) return nullptr;
    if (++bp->uses < when) return nullptr;
    bp->jit = jit_compile(P, bp->prog, bwd, dtype, n);
    if (!bp->jit) bp->jit_failed = true;
    return bp->jit;
}

bool jit_has(const JitPasses* J, int p)
{
    return J && p < (int)J->fn.size() && J->fn[p];
}

int jit_launch_forward(const JitPasses* J, int p, void* psi, const POp* ops, int op_first, double bytes,
                       double flops)
{
    const ZSlot* zs = zbatch_slots();
    const int nz = zs ? zbatch_count() : 1;
    struct {
        void* psi;
        const void* ops;
        const void* zs;
        int op_first;
        int pad;
    } args{psi, ops + op_first, zs, op_first, 0};
    size_t asz = sizeof(args);
    void* cfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &args, HIP_LAUNCH_PARAM_BUFFER_SIZE, &asz, HIP_LAUNCH_PARAM_END};
    ++g_launches_fwd;
    const int pi = prof_begin(YAO_KF_PASS_FWD);
    YAO_HIP(hipModuleLaunchKernel(J->fn[p], (unsigned)J->ntiles[p], 1, (unsigned)nz, (unsigned)J->nthr[p], 1, 1, 0,
                                  stream(), nullptr, cfg));
    prof_end(pi, bytes * nz, flops * nz);
    return 0;
}

int jit_selfcheck(const yao_circuit* c, int dtype, int reverse, int tile_qubits, int* npasses, int* njit)
{
    const int n = c->n;
    const bool bwd = reverse != 0;
    int t, cb, L;
    tile_geometry_tq(n, 1, dtype, bwd, tile_qubits, &t, &cb, &L);
    if (t - cb < kMaxRegBits + 1) return set_error(YAO_EINVAL, "circuit too small for tile passes");
    const Plan& P = get_plan(c, 0, (int)c->gates.size(), 1, t, cb, L, bwd, dtype == YAO_C64 ? 8 : 16);
    if (!P.valid) return set_error(YAO_EINVAL, "pass plan could not restore the qubit layout");
    Program prog;
    YAO_TRY(build_program(P, c, nullptr, bwd, dtype, prog));
    if (!prog.bindable) return set_error(YAO_EINVAL, "circuit cannot be bound on the device");
    std::vector<std::string> src, logs;
    std::vector<int> nthr;
    std::vector<size_t> lds;
    *npasses = (int)P.passes.size();
    *njit = jit_source(P, prog, bwd, dtype, n, src, nthr, lds);
    std::vector<std::vector<char>> code;
    jit_build_all(src, code, logs);
    for (size_t p = 0; p < src.size(); ++p)
        if (!src[p].empty() && code[p].empty())
            return set_error(YAO_EHIP, "run-time compile of pass %zu failed: %.400s", p, logs[p].c_str());
    return 0;
}

int jit_launch_backward(const JitPasses* J, int p, double* psi, void* lam, const POp* ops, int op_first,
                        const double* mats, double* gpartial, int pstride, double bytes, double flops)
{
    const ZSlot* zs = zbatch_slots();
    const int nz = zs ? zbatch_count() : 1;
    const int ps = std::max(pstride, J->ntiles[p]);
    struct {
        void* psi;
        void* lam;
        const void* ops;
        const double* mats;
        double* gpart;
        const void* zs;
        int op_first;
        int pstride;
    } args{psi, lam, ops + op_first, mats, gpartial, zs, op_first, ps};
    size_t asz = sizeof(args);
    void* cfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &args, HIP_LAUNCH_PARAM_BUFFER_SIZE, &asz, HIP_LAUNCH_PARAM_END};
    ++g_launches_bwd;
    const int pi = prof_begin(YAO_KF_PASS_BWD);
    YAO_HIP(hipModuleLaunchKernel(J->fn[p], (unsigned)J->ntiles[p], 1, (unsigned)nz, (unsigned)J->nthr[p], 1, 1, 0,
                                  stream(), nullptr, cfg));
    prof_end(pi, bytes * nz, flops * nz);
    return 0;
}

void jit_stats(long long* out)
{
    out[0] = g_compiled_programs.load();
    out[1] = g_compiled_passes.load();
    out[2] = g_failures.load();
    out[3] = g_launches_fwd.load();
    out[4] = g_launches_bwd.load();
}

void jit_free(JitPasses* J)
{
    if (!J) return;
    for (hipModule_t m : J->mod)
        if (m) (void)hipModuleUnload(m);
    delete J;
}

}  // namespace yao
