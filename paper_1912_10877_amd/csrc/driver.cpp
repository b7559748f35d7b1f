// Choice between the per-gate form and the fused tile passes, and batches of circuits.
#include "driver.h"
#include "fused.h"

namespace yao {

static bool use_fused(const yao_state* s)
{
    return !options().plain && fused_supported(s->n, s->batch);
}

int forward(yao_state* s, const yao_circuit* c, const double* params)
{
    // Forward-only sweeps may fold runs of gates into dense blocks of up to fuse_width qubits.
    const int width = options().fuse_width;
    if (width > 1 && !c->gates.empty()) {
        c = fused_circuit(c, params, width);
        params = nullptr;
    }
    if (use_fused(s)) return forward_fused(s->data, s->dtype, s->n, s->batch, c, params);
    return forward_plain(s->data, s->dtype, s->n, s->batch, c, params);
}

int backward(yao_state* s, const yao_circuit* c, const double* params, yao_pauli_sum* h, int mode, bool reduce_batch,
             double* energy, double* grad, double* drift)
{
    if (use_fused(s)) return backward_fused(s, c, params, h, mode, reduce_batch, energy, grad, drift);
    return backward_plain(s, c, params, h, reduce_batch, energy, grad, drift);
}

}  // namespace yao
