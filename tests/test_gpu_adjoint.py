"""The hand-written adjoint behind torch.autograd: finite differences and the
FP64 oracle gradient (the differentiable workload)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_08555_amd import workloads
from tests.losses import grad_energy, loss_grad_u

pytestmark = pytest.mark.gpu


def _announce(msg):
    print("[case]", msg, flush=True)


def _setup(n, prec, seed=5):
    from paper_2512_08555_amd.lengths import auto_pad
    from paper_2512_08555_amd.solver import Plan
    h = 1.0 / n
    f = workloads.config_blobs_noise(n, seed)
    w = workloads.weight_field(n, h, seed=55)
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = Plan((n, n, n), h, prec, pad=auto_pad((n, n, n), prec))
    return plan, h, torch.from_numpy(f).to("cuda", dt), torch.from_numpy(w).to("cuda", dt)


@pytest.mark.parametrize("n", [32, 64])
def test_autograd_gradient_matches_central_difference_f64(n):
    from paper_2512_08555_amd.autograd import poisson_solve
    _announce("adjoint FD f64 %d^3" % n)
    plan, h, f, w = _setup(n, "f64")
    fr = f.clone().requires_grad_(True)
    L = grad_energy(poisson_solve(fr, plan), w, h)
    L.backward()
    g = fr.grad.detach()
    rng = np.random.default_rng(7)
    for _ in range(2):
        v = torch.from_numpy(rng.standard_normal(f.shape)).to("cuda", torch.float64)
        eps = 1e-3 * float(f.abs().max()) / float(v.abs().max())
        with torch.no_grad():
            lp = grad_energy(plan.solve((f + eps * v).contiguous()), w, h)
            lm = grad_energy(plan.solve((f - eps * v).contiguous()), w, h)
        fd = float((lp - lm) / (2 * eps))
        an = float((g * v).sum())
        assert abs(fd - an) <= 1e-8 * abs(an), (fd, an)


def test_autograd_gradient_matches_oracle_f64():
    from paper_2512_08555_amd.autograd import poisson_solve
    n = 56   # padded to 128 per axis
    _announce("adjoint vs oracle f64 %d^3" % n)
    plan, h, f, w = _setup(n, "f64")
    fr = f.clone().requires_grad_(True)
    grad_energy(poisson_solve(fr, plan), w, h).backward()
    g = fr.grad.detach().cpu().numpy()
    fh = f.cpu().numpy()
    M = plan.padded
    u = oracle.solve(fh, h, M=M)
    gu = loss_grad_u(torch.from_numpy(u), torch.from_numpy(w.cpu().numpy()), h).numpy()
    ref = oracle.adjoint(gu, h, M=M)
    assert np.abs(g - ref).max() / np.abs(ref).max() < 1e-11


def test_c5_fp32_gradient_vs_fp64_oracle():
    """256^3 FP32 forward + backward through autograd, against the FP64
    oracle gradient of the same (FP32-rounded) source and weight."""
    from paper_2512_08555_amd.autograd import poisson_solve
    n = 256
    _announce("c5 fp32 gradient %d^3" % n)
    plan, h, f, w = _setup(n, "f32")
    fr = f.clone().requires_grad_(True)
    L = grad_energy(poisson_solve(fr, plan), w, h)
    L.backward()
    g = fr.grad.detach().double().cpu().numpy()
    fh = f.double().cpu().numpy()
    wh = w.double().cpu().numpy()
    u = oracle.solve(fh, h)
    gu = loss_grad_u(torch.from_numpy(u), torch.from_numpy(wh), h).numpy()
    ref = oracle.adjoint(gu, h)
    linf = np.abs(g - ref).max() / np.abs(ref).max()
    l2 = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    lref = float(grad_energy(torch.from_numpy(u), torch.from_numpy(wh), h))
    print("c5 fp32 grad rel Linf %.3e rel L2 %.3e loss rel err %.3e"
          % (linf, l2, abs(float(L) - lref) / abs(lref)), flush=True)
    # measured 6.1e-7 and 3.3e-7: about 8x and 6x headroom
    assert linf < 5e-6 and l2 < 2e-6
