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
    if (use_fused(s)) return forward_fused(s->data, s->dtype, s->n, s->batch, c, params);
    return forward_plain(s->data, s->dtype, s->n, s->batch, c, params);
}

int backward(yao_state* s, const yao_circuit* c, const double* params, yao_pauli_sum* h, int mode, bool reduce_batch,
             double* energy, double* grad, double* drift)
{
    if (use_fused(s)) return backward_fused(s, c, params, h, mode, reduce_batch, energy, grad, drift);
    return backward_plain(s, c, params, h, reduce_batch, energy, grad, drift);
}

int batch_run(int ncirc, yao_state* const* states, const yao_circuit* const* circs, const double* const* params,
              yao_pauli_sum* const* h, double* energy, double* const* grad)
{
    for (int c = 0; c < ncirc; ++c) {
        YAO_TRY(launch_reset(states[c]));
        YAO_TRY(backward(states[c], circs[c], params[c], h[c], YAO_GRAD_REVERSIBLE, false, energy + c, grad[c], nullptr));
    }
    return 0;
}

}  // namespace yao
