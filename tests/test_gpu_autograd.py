"""LKSFunction: torch.autograd wrapper of the C-ABI forward and adjoint."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_2411_03090_amd import autograd, lks, workloads as W  # noqa: E402

DEV = torch.device("cuda:0")


def _wl():
    wl = W.steady_channel_uniform(40, 24, Re=10.0, seed=5, n_fwd=2500, n_adj=2500)
    wl.alpha_max = 0.5
    wl.gamma = 0.2 + 0.6 * W.gamma_grf(40, 24, 3.0, 1)   # strictly inside (0, 1)
    return wl


def test_function_matches_oracle_and_chain_rule():
    print("[gpu] autograd 40x24", flush=True)
    wl = _wl()
    solver = lks.LKS(wl, precision="fp64", device=DEV)
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=DEV, requires_grad=True)
    J = autograd.objective(g, solver)
    loss = 3.0 * J + J * J
    loss.backward()
    Jo, so, _, _ = O.gradient(wl)
    assert abs(J.item() - Jo) / abs(Jo) < 1e-12
    want = (3.0 + 2.0 * Jo) * so.reshape(-1)
    got = g.grad.cpu().numpy()
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-12


def test_backward_recomputes_a_stale_forward():
    print("[gpu] autograd stale forward", flush=True)
    wl = _wl()
    solver = lks.LKS(wl, precision="fp64", device=DEV)
    g1 = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=DEV, requires_grad=True)
    g2 = torch.tensor(np.clip(wl.gamma.reshape(-1) * 0.8, 0, 1), dtype=torch.float64, device=DEV,
                      requires_grad=True)
    J1 = autograd.objective(g1, solver)
    J2 = autograd.objective(g2, solver)
    J1.backward()
    ref = torch.empty_like(g1)
    solver.forward(g1.detach())
    solver.backward(1.0, ref)
    torch.cuda.synchronize()
    assert torch.equal(g1.grad, ref)
    assert J2.item() != J1.item()


def test_directional_fd_through_the_function():
    """Central differences of J through LKSFunction.forward along a smooth
    direction agree with the oracle's; the ALKS directional derivative agrees
    with them within 10 % (the paper's approximate adjoint boundary treatment;
    the oracle gives 0.5-4 % on these directions)."""
    print("[gpu] autograd directional FD", flush=True)
    wl = _wl()
    solver = lks.LKS(wl, precision="fp64", device=DEV)
    dirs = [W.gaussian_random_field((wl.ny, wl.nx), 3.0, s).reshape(-1) for s in range(3)]
    base = wl.gamma.reshape(-1)
    g = torch.tensor(base, dtype=torch.float64, device=DEV, requires_grad=True)
    J = autograd.objective(g, solver)
    J.backward()
    grad = g.grad.cpu().numpy()
    eps = 1e-4
    adj, fd = [], []
    for d in dirs:
        d = d * (np.arange(base.size) % wl.nx > 0)  # leave the ring untouched
        vals = []
        for sgn in (1.0, -1.0):
            gg = torch.tensor(base + sgn * eps * d, dtype=torch.float64, device=DEV)
            vals.append(autograd.objective(gg, solver).item())
        fd.append((vals[0] - vals[1]) / (2 * eps))
        adj.append(grad @ d)
        w2 = W.steady_channel_uniform(40, 24, Re=10.0, seed=5, n_fwd=2500, n_adj=2500)
        w2.alpha_max = 0.5
        jp = O.objective(w2, (base + eps * d).reshape(wl.ny, wl.nx))
        jm = O.objective(w2, (base - eps * d).reshape(wl.ny, wl.nx))
        assert abs((jp - jm) / (2 * eps) - fd[-1]) < 1e-6 * abs(fd[-1]) + 1e-12
    ratio = np.array(adj) / np.array(fd)
    assert np.all(np.abs(ratio - 1.0) < 0.1), ratio
