"""torch.autograd face of the reverse sweep: expect'(H, reg => circuit) (Sec. "Reverse Mode").

`expectation(params, circuit, H, ...)` returns E[b] = <psi_b|H|psi_b> as a torch tensor whose
gradient with respect to `params` comes from the library's reversible adjoint sweep: the
forward call runs yao_backward once (forward sweep, H psi, reverse sweep) and keeps the
per-slot gradients; the autograd backward only applies the chain rule with the incoming
dL/dE. No state or intermediate is kept in torch.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as yb


class _Expectation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, circuit, H, n, batch, dtype, mode, psi0):
        p = params.detach().to("cpu", torch.float64).numpy()
        dev = torch.device("cuda", torch.cuda.current_device())
        cdt = torch.complex64 if dtype == yb.C64 else torch.complex128
        buf = torch.empty((1 << n) * batch, dtype=cdt, device=dev)
        state = yb.State(n, batch, dtype, tensor=buf)
        yb.use_torch_stream()
        if psi0 is None:
            state.reset()
        else:
            buf.copy_(psi0.reshape(-1).to(dev, cdt))
        e, g, _ = yb.backward(state, circuit, p, H, mode=mode)
        ctx.save_for_backward(torch.as_tensor(np.asarray(g), dtype=torch.float64))
        ctx.param_device = params.device
        ctx.param_dtype = params.dtype
        ctx.state = buf.reshape(1 << n, batch)
        return torch.as_tensor(e, dtype=torch.float64, device=params.device)

    @staticmethod
    def backward(ctx, grad_e):
        (g,) = ctx.saved_tensors  # [batch][nparams]
        ge = grad_e.detach().to("cpu", torch.float64).reshape(-1, 1)
        gp = (ge * g).sum(0)
        return gp.to(ctx.param_device, ctx.param_dtype), None, None, None, None, None, None, None


def expectation(params: torch.Tensor, circuit: "yb.Circuit", H: "yb.PauliSum", n: int, batch: int = 1,
                dtype: int = yb.C64, mode: int = yb.GRAD_REVERSIBLE, psi0: torch.Tensor | None = None):
    """Energy per batch slot of circuit(params) applied to psi0 (default |0...0>); differentiable
    in `params` through the library's adjoint sweep."""
    return _Expectation.apply(params, circuit, H, n, batch, dtype, mode, psi0)
