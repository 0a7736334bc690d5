"""Entry points called on a caller's stream (a torch side stream, default priority) while
that stream is still busy with the work that produces their input: every call orders its
own work after the caller's, so its results are bitwise those of the same call made on the
current stream after a synchronisation."""
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


def busy_copy(torch, src, stream):
    """src copied on `stream` behind about a millisecond of other work on that stream, with
    no host synchronisation: a call that did not wait for the stream would read the copy
    before it is written."""
    src_ready = torch.cuda.Event()
    src_ready.record()
    with torch.cuda.stream(stream):
        stream.wait_event(src_ready)
        a = torch.ones(4096, 4096, dtype=torch.float32, device="cuda")
        for _ in range(3):
            a = a @ a * (1.0 / 4096)
        out = src.clone()
        out.record_stream(stream)
    return out


def opts(rd, cfg, precision):
    return rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], omega=cfg["omega"], precision=precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("N", [64, 256])
def test_step_on_a_busy_side_stream(ctx, rd, N, precision):
    import torch
    cfg = small_cfg("allen_cahn", N, "periodic")
    p, o = rd.problem_from_config(cfg), opts(rd, cfg, precision)
    u0 = dev(wl.initial_field(cfg, N=N))
    ref, ref_info = ctx.step(u0, cfg["ht"], p, o)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    u_s = busy_copy(torch, u0, s)
    with torch.cuda.stream(s):
        out = torch.full_like(u0, float("nan"))
    out_s, info = ctx.step(u_s, cfg["ht"], p, o, out=out, stream=s)
    torch.cuda.synchronize()
    assert (info["iters"], info["outer"], info["status"]) == (ref_info["iters"], ref_info["outer"], "ok")
    assert torch.equal(out_s, ref)


def test_kernel_level_calls_on_a_busy_side_stream(ctx, rd):
    import torch
    cfg = small_cfg("allen_cahn", 256, "neumann")
    p = rd.problem_from_config(cfg)
    u0 = dev(wl.initial_field(cfg, N=256))
    uk = u0 * 0.5
    w_ref, r_ref = ctx.residual(u0, uk, cfg["ht"], p)
    y_ref = ctx.precond_solve(w_ref, cfg["ht"], p)
    x_ref = ctx.prox(u0, cfg["ht"], p)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    w, r = ctx.residual(busy_copy(torch, u0, s), busy_copy(torch, uk, s), cfg["ht"], p, stream=s)
    y = ctx.precond_solve(busy_copy(torch, w_ref, s), cfg["ht"], p, stream=s)
    x = ctx.prox(busy_copy(torch, u0, s), cfg["ht"], p, stream=s)
    torch.cuda.synchronize()
    assert r == r_ref and torch.equal(w, w_ref)
    assert torch.equal(y, y_ref) and torch.equal(x, x_ref)


def test_advance_on_a_busy_side_stream(ctx, rd):
    import torch
    cfg = small_cfg("allen_cahn", 128, "periodic")
    p, o = rd.problem_from_config(cfg), opts(rd, cfg, "fp64")
    u0 = dev(wl.initial_field(cfg, N=128))
    a = rd.make_adapt(cfg["ht"], 0.5, 40, 10)
    ref = u0.clone()
    ref_info, ref_trace = ctx.advance(ref, 4 * cfg["ht"], p, o, a)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    u = busy_copy(torch, u0, s)
    info, trace = ctx.advance(u, 4 * cfg["ht"], p, o, a, stream=s)
    torch.cuda.synchronize()
    assert info == ref_info and trace == ref_trace
    assert torch.equal(u, ref)


def test_trajectory_open_and_read_on_a_busy_side_stream(ctx, rd):
    import torch
    cfg = small_cfg("allen_cahn", 256, "periodic")
    p, o = rd.problem_from_config(cfg), opts(rd, cfg, "fp64")
    u0 = dev(wl.initial_field(cfg, N=256))
    ref, _ = ctx.step(u0, cfg["ht"], p, o)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    t = ctx.open(p, o, busy_copy(torch, u0, s), stream=s)
    try:
        tk = t.submit(cfg["ht"])
        for _ in range(20000):
            if ctx.poll(tk) is not None:
                break
            ctx.pump()
        assert ctx.poll(tk)["status"] == "ok"
        with torch.cuda.stream(s):
            out = torch.full_like(u0, float("nan"))
        got = t.read(out=busy_copy(torch, out, s), stream=s)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
    finally:
        t.close()
