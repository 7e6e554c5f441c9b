"""The allocation-free entry point lks_bind_static_workspace: a context
bound to the library's static per-device array gives the same objective and
gradient as the same context on caller-owned (torch) memory, on two calls in
a row with the second on a smaller problem, and a context that lost the
array to another one refuses further calls."""
import numpy as np
import pytest
import torch

from paper_2411_03090_amd import lks, workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def _gradient(ctx, wl, steps=None):
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=DEV)
    out = torch.full_like(g, float("nan"))
    ctx.forward(g, steps)
    J = ctx.objective()
    ctx.backward(1.0, out, steps)
    torch.cuda.synchronize()
    return J, out.cpu().numpy(), ctx.read("ux").cpu().numpy()


def _pair(wl, precision):
    ref = lks.LKS(wl, precision=precision, device=DEV)
    J0, d0, u0 = _gradient(ref, wl)
    st = lks.LKS(wl, precision=precision, device=DEV, bind=False)
    st.bind_static()
    J1, d1, u1 = _gradient(st, wl)
    return (J0, d0, u0), (J1, d1, u1), st


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_workspace_matches_caller_workspace_on_two_calls(precision):
    say(f"[gpu] static workspace, steady 200x120 then unsteady thermal 96x48, {precision}")
    first = W.steady_channel_grf(200, 120, Re=50.0, sigma=6.0, seed=3, n_fwd=300, n_adj=300)
    a, b, c1 = _pair(first, precision)
    assert b[0] == a[0]
    assert np.array_equal(b[1], a[1]) and np.array_equal(b[2], a[2])
    # the second call: a smaller problem on the same array (unsteady,
    # checkpointed inside the array)
    second = W.unsteady_thermal_channel(96, 48, n_steps=60, period=30.0)
    a2, b2, c2 = _pair(second, precision)
    assert b2[0] == a2[0]
    assert np.array_equal(b2[1], a2[1]) and np.array_equal(b2[2], a2[2])
    assert np.all(np.isfinite(b2[1]))
    # the first context lost the array to the second one
    g = torch.tensor(first.gamma.reshape(-1), dtype=torch.float64, device=DEV)
    with pytest.raises(lks.LKSError) as e:
        c1.forward(g, 10)
    assert e.value.status == lks.LKS_E_STATE
    # bound again, it works as before
    c1.bind_static()
    J, d, u = _gradient(c1, first)
    assert J == a[0] and np.array_equal(d, a[1])
