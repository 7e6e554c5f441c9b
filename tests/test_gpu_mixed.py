"""Mixed precision (LKS_MIXED): the forward sweep and the objective of an
FP64 context, the adjoint sweep of an FP32 one from the final forward state
rounded to float. The forward fields and J are bitwise those of the FP64
path; the gradient agrees with the FP64 oracle within the FP32 gradient
tolerance (1e-3 relative L2) and with the FP32 path's adjoint run from the
same rounded state bitwise."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_2411_03090_amd import lks, workloads as W  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _run(ctx, g, wl):
    out = torch.full_like(g, float("nan"))
    ctx.forward(g, wl.n_fwd)
    J = ctx.objective()
    ctx.backward(1.0, out, wl.n_adj)
    torch.cuda.synchronize()
    fields = {n: ctx.read(n).cpu().numpy() for n in ("drho", "ux", "uy", "adj_rho", "adj_vx")}
    return J, out.cpu().numpy(), fields


@pytest.mark.parametrize("nx,ny,shape", [(70, 37, None), (256, 131, (8, 1, 2)), (129, 64, (4, 1, 1))])
def test_mixed_forward_is_fp64_and_gradient_is_within_fp32_tolerance(nx, ny, shape):
    say(f"[gpu] mixed precision {nx}x{ny} shape {shape}")
    wl = W.steady_channel_grf(nx, ny, Re=40.0, sigma=4.0, seed=2, n_fwd=600, n_adj=600)
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=DEV)
    c64 = lks.LKS(wl, precision="fp64", device=DEV)
    cm = lks.LKS(wl, precision="mixed", device=DEV)
    if shape is not None:
        for c in (c64, cm):
            c.set_tile_rows(shape[0])
        cm.set_steps_per_launch(shape[1], shape[2])
    J64, d64, f64 = _run(c64, g, wl)
    Jm, dm, fm = _run(cm, g, wl)
    assert Jm == J64
    for n in ("drho", "ux", "uy"):
        assert np.array_equal(fm[n], f64[n]), n
    Jo, so, _, _ = O.gradient(wl)
    assert abs(Jm - Jo) / abs(Jo) < 1e-12
    assert rel(dm, so) < 1e-3
    assert rel(dm, d64) < 1e-3
    # the adjoint part is the FP32 path's adjoint from the same rounded state
    c32 = lks.LKS(wl, precision="fp32", device=DEV)
    if shape is not None:
        c32.set_tile_rows(shape[0])
        c32.set_steps_per_launch(1, shape[2])
    c32.forward(g, 0)
    for n in ("drho", "ux", "uy"):
        c32.write(n, torch.tensor(f64[n], device=DEV))
    out = torch.full_like(g, float("nan"))
    c32.backward(1.0, out, wl.n_adj)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), dm)
    cm.gradient_status()


def test_mixed_refuses_unsteady_and_batches():
    say("[gpu] mixed precision refusals")
    wl = W.unsteady_thermal_channel(40, 24, n_steps=10)
    with pytest.raises(lks.LKSError) as e:
        lks.LKS(wl, precision="mixed", device=DEV)
    assert e.value.status == lks.LKS_E_UNSUPPORTED
    st = W.steady_channel_uniform(40, 24, Re=10.0, seed=0, n_fwd=10, n_adj=10)
    with pytest.raises(lks.LKSError):
        lks.Batch([st, st], precision="mixed", device=DEV)
