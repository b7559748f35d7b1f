// Drivers behind the C ABI: per-gate and fused execution of circuits, the reverse sweep and
// batches of circuits. Arguments are validated by the caller.
#pragma once

#include "runtime.h"

namespace yao {

int apply_one(yao_state* s, const GateRec& g, double theta);
int forward(yao_state* s, const yao_circuit* c, const double* params);
int backward(yao_state* s, const yao_circuit* c, const double* params, yao_pauli_sum* h, int mode, bool reduce_batch,
             double* energy, double* grad, double* drift);
// Graph-recorded batch of circuits (driver_batch.cpp); drop_batch forgets a recorded batch
// that uses the circuit, state or observable obj.
int batch_run(int ncirc, yao_state* const* states, const yao_circuit* const* circs, const double* const* params,
              yao_pauli_sum* const* h, double* energy, double* const* grad);
void drop_batch(const void* obj);
void drop_plans(const yao_circuit* c);

// Dense-block fusion for forward sweeps (fusion.cpp).
struct FusedPart {
    std::vector<int> qubits;  // ascending: the fused gate's locs
    std::vector<int> gates;   // member gates of the circuit, in application order
    bool single = false;      // one gate kept as it is (wider than the width)
};
std::vector<GateRec> fuse_gates(const yao_circuit* c, const double* params, int width);
const yao_circuit* fused_circuit(const yao_circuit* c, const double* params, int width);
// The fused circuit's structure (cached): one gate per part, multi-gate parts as placeholders
// whose matrices are bound later, single gates as in c (with their parameters).
const yao_circuit* fused_shape(const yao_circuit* c, int width, const std::vector<FusedPart>** parts);
void drop_fused(const yao_circuit* c);

// Host run of a circuit's pass plan against gate-by-gate application (plan_check.cpp).
int plan_selfcheck(const yao_circuit* c, const double* params, int dtype, int reverse, int tile_qubits, double* max_err,
                   int* npasses);

// Per-gate form.
int forward_plain(void* data, int dtype, int n, int B, const yao_circuit* c, const double* params);
int backward_plain(yao_state* s, const yao_circuit* c, const double* params, yao_pauli_sum* h, bool reduce_batch,
                   double* energy, double* grad, double* drift);

inline double gate_theta(const GateRec& g, const double* params)
{
    return g.param >= 0 ? params[g.param] : g.theta;
}

}  // namespace yao
