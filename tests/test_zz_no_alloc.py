"""rd_step_noalloc through the C ABI: the allocation-free step (workspace in the library's
device scratch array) against rd_step on the same inputs, two calls in a row with the
second on a smaller grid, to the parity bar (FP64 1e-10 with equal iteration counts,
mixed 1e-5; both are in fact bitwise equal, the kernels being the same), plus the
refusal of a problem beyond the array."""
import numpy as np
import pytest

from paper_2305_03945_amd import workloads as wl
from tests.rd_cases import small_cfg

pytestmark = pytest.mark.gpu


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


CASES = [("allen_cahn", "periodic"), ("cahn_hilliard", "neumann"), ("schnakenberg", "periodic")]


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
@pytest.mark.parametrize("kind,bc", CASES)
def test_noalloc_step_matches_rd_step(ctx, rd, kind, bc, precision, bar):
    import torch
    for N in (256, 64):   # the second call on a smaller grid reuses the scratch array
        cfg = small_cfg(kind, N, bc)
        p = rd.problem_from_config(cfg)
        o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], omega=cfg["omega"], precision=precision)
        u = dev(wl.initial_field(cfg, N=N, seed=N + 1))
        ref, info_ref = ctx.step(u, cfg["ht"], p, o)
        out = torch.full_like(u, float("nan"))
        info, code = ctx.step_noalloc(u, cfg["ht"], p, o, out)
        print("noalloc %s %s %s N=%d: iters %d/%d outer %d/%d" % (kind, bc, precision, N, info["iters"],
              info_ref["iters"], info["outer"], info_ref["outer"]), flush=True)
        assert code == rd.RD_OK and info["status"] == info_ref["status"] == "ok"
        assert info["iters"] == info_ref["iters"] and info["outer"] == info_ref["outer"]
        assert float((out - ref).abs().max().item()) <= bar
        assert torch.equal(out, ref)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_fch_step_matches_rd_step(ctx, rd, precision):
    """The sixth-order equation (Sec. 3.3) through the allocation-free step, 128^2 then 64^2."""
    import math
    import torch
    for N in (128, 64):
        p = rd.make_problem("fch", N, L=2 * math.pi, diff=(0.18 ** 2,))
        o = rd.make_opts(tol=1e-6, tau_u=0.58, tau_p=0.58, max_iter=5000, precision=precision)
        x = np.arange(N) * (2 * math.pi / N)
        X, Y = np.meshgrid(x, x)
        u = dev(2 * np.exp(np.sin(X) + np.sin(Y) - 2) + 2.2 * np.exp(-np.sin(X) - np.sin(Y) - 2) - 1)
        ref, info_ref = ctx.step(u, 1e-3, p, o)
        out = torch.full_like(u, float("nan"))
        info, code = ctx.step_noalloc(u, 1e-3, p, o, out)
        assert code == rd.RD_OK and info["status"] == info_ref["status"] == "ok"
        assert info["iters"] == info_ref["iters"] and info["outer"] == info_ref["outer"]
        assert torch.equal(out, ref)


def test_noalloc_in_place_and_refusal(ctx, rd):
    import torch
    cfg = small_cfg("allen_cahn", 128, "periodic")
    p = rd.problem_from_config(cfg)
    o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], precision="fp64")
    u = dev(wl.initial_field(cfg, N=128, seed=3))
    ref, _ = ctx.step(u, cfg["ht"], p, o)
    info, code = ctx.step_noalloc(u, cfg["ht"], p, o, u)   # in place
    assert code == rd.RD_OK and torch.equal(u, ref)
    big = small_cfg("allen_cahn", 2048, "periodic")
    ub = torch.zeros((2048, 2048), dtype=torch.float64, device="cuda")
    info, code = ctx.step_noalloc(ub, big["ht"], rd.problem_from_config(big), o, ub)
    assert code == rd.RD_E_NOMEM
