// Choice between the per-gate form and the fused tile passes, and batches of circuits.
#include "driver.h"
#include "fused.h"
#include "tuner.h"

namespace yao {

static bool use_fused(const yao_state* s)
{
    return !options().plain && fused_supported(s->n, s->batch);
}

int forward(yao_state* s, const yao_circuit* c, const double* params)
{
    // Forward-only sweeps may fold gates into dense blocks (fusion.cpp): at options().fuse_width,
    // or at the width the autotuner found fastest for this circuit and state shape.
    const bool fused = use_fused(s);
    int width = options().fuse_width;
    if (fused) {
        YAO_TRY(pick_forward_width(c, params, s->data, s->dtype, s->n, s->batch, &width));
        return forward_sweep(s->data, s->dtype, s->n, s->batch, c, params, width, options().tile_qubits, nullptr);
    }
    const double* fp = params;
    c = forward_circuit(c, params, width, &fp);
    return forward_plain(s->data, s->dtype, s->n, s->batch, c, fp);
}

int backward(yao_state* s, const yao_circuit* c, const double* params, yao_pauli_sum* h, int mode, bool reduce_batch,
             double* energy, double* grad, double* drift)
{
    if (use_fused(s)) return backward_fused(s, c, params, h, mode, reduce_batch, energy, grad, drift);
    return backward_plain(s, c, params, h, reduce_batch, energy, grad, drift);
}

}  // namespace yao
