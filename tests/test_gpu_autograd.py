"""torch.autograd through the library's reverse sweep, checked against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

yb = ag = torch = None


@pytest.fixture(scope="module", autouse=True)
def gpu():
    global yb, ag, torch
    import torch as _torch

    assert _torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_10877_amd import autograd as _ag
    from paper_1912_10877_amd import binding as _yb

    torch, yb, ag = _torch, _yb, _ag
    yb.init()
    yield


@pytest.mark.parametrize("dtype", [0, 1])
def test_autograd_gradient_matches_oracle(dtype):
    n, depth = 8, 3
    circ = w.hea_circuit(n, depth)
    H = w.heisenberg(n)
    p0 = w.angles(3, circ.nparams)
    e_ref, g_ref, _ = oracle.adjoint(H, circ, p0, w.zero_state(n))
    params = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    e = ag.expectation(params, yb.Circuit.from_workload(circ), yb.PauliSum.from_workload(H), n, dtype=dtype)
    e.sum().backward()
    tol = 1e-10 if dtype == 1 else 1e-4
    assert abs(e.item() - e_ref[0]) <= (1e-10 if dtype == 1 else 1e-5)
    assert np.abs(params.grad.numpy() - g_ref[0]).max() <= tol * max(1, np.abs(g_ref).max())


def test_autograd_batched_chain_rule():
    """L = sum_b w_b E_b for a batch of random inputs: dL/dtheta = sum_b w_b dE_b/dtheta."""
    n, B = 7, 3
    circ = w.random_gate_list(n, 30, seed=77, kmax=2)
    H = w.heisenberg(n)
    p0 = w.angles(4, circ.nparams)
    psi0 = w.random_state(n, B, 8)
    e_ref, g_ref, _ = oracle.adjoint(H, circ, p0, psi0)
    wts = np.array([0.5, -2.0, 1.5])
    params = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    e = ag.expectation(params, yb.Circuit.from_workload(circ), yb.PauliSum.from_workload(H), n, batch=B,
                       dtype=yb.C128, psi0=torch.tensor(psi0))
    (torch.tensor(wts) * e).sum().backward()
    np.testing.assert_allclose(e.detach().numpy(), e_ref, atol=1e-10)
    np.testing.assert_allclose(params.grad.numpy(), wts @ g_ref, atol=1e-10)


def test_vqe_descent_lowers_energy():
    """A few gradient-descent steps of the VQE loop (Listing "10000-layer VQE", small)."""
    n, depth = 6, 3
    circ = w.hea_circuit(n, depth)
    H = w.heisenberg(n)
    c, h = yb.Circuit.from_workload(circ), yb.PauliSum.from_workload(H)
    params = torch.tensor(w.angles(5, circ.nparams), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.SGD([params], lr=0.05)
    energies = []
    for _ in range(25):
        opt.zero_grad()
        e = ag.expectation(params, c, h, n, dtype=yb.C128)
        e.sum().backward()
        opt.step()
        energies.append(e.item())
    assert energies[-1] < energies[0] - 0.5
    assert energies[-1] >= -11.2111025509 - 1e-9  # ground energy of the 6-site ring


def test_deep_circuit_reversible_sweep():
    """10 qubits, depth 500 (15000 parameters): the reversible sweep needs no stored states."""
    n, depth = 10, 500
    circ = w.hea_circuit(n, depth)
    H = w.heisenberg(n)
    p = w.angles(6, circ.nparams)
    e_ref, g_ref, _ = oracle.adjoint(H, circ, p, w.zero_state(n))
    s = yb.State(n, 1, yb.C128)
    e, g, drift = yb.backward(s, yb.Circuit.from_workload(circ), p, yb.PauliSum.from_workload(H))
    assert abs(e[0] - e_ref[0]) <= 1e-9
    assert np.abs(g[0] - g_ref[0]).max() <= 1e-9 * max(1, np.abs(g_ref).max())
    assert drift < 1e-10
