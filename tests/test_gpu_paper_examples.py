"""The paper's own examples on the GPU, checked against the oracle and against
what the paper reports (loose physics pins)."""
import json
import os

import numpy as np
import pytest

from oracle import equations as eq, grid, pdhg
from tests.rd_cases import max_abs

pytestmark = pytest.mark.gpu
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.fixture(scope="module")
def rd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_03945_amd import rd as rdmod
    return rdmod


@pytest.fixture(scope="module")
def ctx(rd):
    c = rd.Context(0)
    yield c
    c.close()


def dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def schnakenberg_paper(N=128):
    """Sec. 3.4.1: Neumann unit square, kappa = 100, a = 0.1305, b = 0.7695, D = (0.05, 1),
    a small Gaussian bump on the steady state."""
    a, b = 0.1305, 0.7695
    prob = eq.Problem(kind=eq.SCHNAKENBERG, N=N, L=1.0, bc=grid.NEUMANN, diff=(0.05, 1.0), a=a, sb=b, kappa=100.0)
    x = (np.arange(N) + 0.5) * prob.h
    X, Y = np.meshgrid(x, x)
    U = np.stack([a + b + 1e-3 * np.exp(-100 * ((X - 1 / 3) ** 2 + (Y - 1 / 2) ** 2)),
                  np.full((N, N), b / (a + b) ** 2)])
    return prob, U


def test_schnakenberg_paper_example(ctx, rd):
    """About 30 iterations per step (Sec. 3.4.1); FP64 equal to the oracle step by step."""
    g = GOLDEN["schnakenberg_iterations"]
    prob, U = schnakenberg_paper()
    p = rd.make_problem("schnakenberg", 128, bc="neumann", diff=(0.05, 1.0), a=0.1305, sb=0.7695, kappa=100.0)
    o64 = rd.make_opts(tol=1e-7, tau_u=0.9, tau_p=0.9)
    omx = rd.make_opts(tol=1e-7, tau_u=0.9, tau_p=0.9, precision="mixed")
    lo, hi = g["accept_range"]
    u64, umx = dev(U), dev(U)
    for k in range(g["steps_checked"]):
        r = pdhg.step(prob, U, 1.0 / 5000, pdhg.Options(tol=1e-7, tau_u=0.9, tau_p=0.9))
        u64, i64 = ctx.step(u64, 1.0 / 5000, p, o64)
        umx, imx = ctx.step(umx, 1.0 / 5000, p, omx)
        assert lo <= i64["iters"] <= hi and i64["iters"] == r.iters, (k, i64, r.iters)
        assert max_abs(u64.cpu().numpy(), r.U) <= 1e-10
        assert imx["status"] == "ok" and max_abs(umx.cpu().numpy(), r.U) <= 1e-5
        U = r.U


def test_allen_cahn_shrinking_circle(ctx, rd):
    """Sec. 3.1.1: a circle of radius 0.2 on [-0.25, 0.25]^2, eps = 0.01 (lambda = eps,
    b = 1 / eps), h_t = 1e-3, tau = 0.5, delta = 1e-7.  The paper's grid has 100 points;
    this one 128 (power-of-two transforms).  Fewer than 200 iterations per step, and
    the zero level set follows mean-curvature flow, r(t)^2 = r0^2 - 2 eps t."""
    N, L, eps, r0, ht = 128, 0.5, 0.01, 0.2, 1e-3
    prob = eq.Problem(kind=eq.ALLEN_CAHN, N=N, L=L, bc=grid.PERIODIC, diff=(eps,), b=1.0 / eps)
    x = -0.25 + np.arange(N) * prob.h
    X, Y = np.meshgrid(x, x)
    U = np.where(X ** 2 + Y ** 2 < r0 ** 2, 1.0, -1.0)
    p = rd.make_problem("allen_cahn", N, L=L, diff=(eps,), b=1.0 / eps)
    o64 = rd.make_opts(tol=1e-7, tau_u=0.5, tau_p=0.5)
    u = dev(U)
    g = GOLDEN["allen_cahn_circle_iterations"]
    for k in range(g["steps_checked"]):
        r = pdhg.step(prob, U, ht, pdhg.Options(tol=1e-7, tau_u=0.5, tau_p=0.5))
        u, info = ctx.step(u, ht, p, o64)
        assert info["iters"] == r.iters and info["iters"] < g["max_iters"], (k, info, r.iters)
        assert max_abs(u.cpu().numpy(), r.U) <= 1e-10
        U = r.U
    omx = rd.make_opts(tol=1e-7, tau_u=0.5, tau_p=0.5, precision="mixed")
    t = g["steps_checked"] * ht
    radii = []
    for t_check in (0.5, 1.0):
        while t < t_check - 1e-9:
            u, info = ctx.step(u, ht, p, omx)
            assert info["status"] == "ok"
            t += ht
        area = prob.h ** 2 * float(((u.cpu().numpy() + 1.0) / 2.0).sum())
        radii.append((t_check, np.sqrt(area / np.pi), np.sqrt(r0 ** 2 - 2 * eps * t_check)))
    for t_check, r_num, r_law in radii:
        assert abs(r_num - r_law) <= 0.03 * r_law, radii
