"""GPU parity of the 3-D grids (7-point Laplacian, N^3 points) against the oracle."""
import numpy as np
import pytest

from oracle import equations as oeq, grid, pdhg, spectral
from paper_2305_03945_amd import workloads as wl
from tests.rd_cases import max_abs, oracle_opts, oracle_problem

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


def cfg3(kind, N, bc):
    if kind == "schnakenberg":
        return dict(kind=kind, dim=3, N=N, L=1.0, bc=bc, diff=(1.0, 10.0), a=0.1, sb=0.9, kappa=1.0, ht=1e-3,
                    init=("steady_plus_uniform", -0.05, 0.05), seed=13, tol=1e-6, tau=0.9, omega=1.0)
    return dict(kind=kind, dim=3, N=N, L=1.0, bc=bc, diff=(0.05 ** 2,), b=1.0, ht=1e-2,
                init=("uniform", -0.9, 0.9), seed=12, tol=1e-8, tau=0.9, omega=1.0)


KINDS = ["allen_cahn", "heat", "schnakenberg"]
BCS = ["periodic", "neumann"]


@pytest.mark.parametrize("kind", ["allen_cahn", "schnakenberg"])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("N", [16, 32, 64, 128])
def test_precond_3d(ctx, rd, kind, bc, N):
    cfg = cfg3(kind, N, bc)
    op = oracle_problem(cfg)
    W = np.random.default_rng(N).standard_normal((op.ncomp,) + op.shape if op.ncomp > 1 else op.shape)
    coeffs = oeq.precond_coeffs(op, cfg["ht"])
    if op.ncomp == 1:
        Y_ref = spectral.precond_solve(W, op.h, bc, *coeffs[0])
    else:
        Y_ref = np.stack([spectral.precond_solve(W[c], op.h, bc, *coeffs[c]) for c in range(2)])
    p = rd.problem_from_config(cfg)
    Y = ctx.precond_solve(dev(W), cfg["ht"], p, "fp64").cpu().numpy()
    scale = np.abs(Y_ref).max()
    assert max_abs(Y, Y_ref) <= 1e-12 * scale
    Y32 = ctx.precond_solve(dev(W), cfg["ht"], p, "mixed").cpu().numpy()
    assert max_abs(Y32, Y_ref) <= 2e-6 * scale


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("N", [16, 32, 64])
def test_step_3d_fp64_and_mixed(ctx, rd, kind, bc, N):
    cfg = cfg3(kind, N, bc)
    op = oracle_problem(cfg)
    U = wl.initial_field(cfg)
    p = rd.problem_from_config(cfg)
    o64 = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"])
    omx = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], precision="mixed")
    u64, umx = dev(U), dev(U)
    for k in range(2):
        r = pdhg.step(op, U, cfg["ht"], oracle_opts(cfg))
        u64, i64 = ctx.step(u64, cfg["ht"], p, o64)
        umx, imx = ctx.step(umx, cfg["ht"], p, omx)
        assert r.status == pdhg.OK and i64["status"] == "ok" and imx["status"] == "ok"
        assert i64["iters"] == r.iters, (k, i64, r.iters)
        assert max_abs(u64.cpu().numpy(), r.U) <= 1e-10
        assert max_abs(umx.cpu().numpy(), r.U) <= 1e-5
        U = r.U


@pytest.mark.parametrize("bc", BCS)
def test_z_invariant_3d_step_equals_2d_step(ctx, rd, bc):
    N = 32
    v = wl.uniform_field(N, -0.9, 0.9, 21)
    p2 = rd.make_problem("allen_cahn", N, bc=bc, diff=(0.05 ** 2,))
    p3 = rd.make_problem("allen_cahn", N, bc=bc, diff=(0.05 ** 2,), dim=3)
    u2, i2 = ctx.step(dev(v), 1e-2, p2, rd.make_opts(tol=1e-9))
    u3, i3 = ctx.step(dev(np.broadcast_to(v, (N, N, N))), 1e-2, p3, rd.make_opts(tol=1e-9 * np.sqrt(N)))
    assert i2["iters"] == i3["iters"]
    a3 = u3.cpu().numpy()
    for z in (0, 7, N - 1):
        assert max_abs(a3[z], u2.cpu().numpy()) <= 1e-12


def test_ac3d128_first_step(ctx, rd):
    """The 128^3 Allen-Cahn workload: first step, FP64 (1e-10, equal iterations) and mixed (1e-5)."""
    cfg = dict(wl.CONFIGS["ac3d128"])
    op = oracle_problem(cfg)
    U = wl.initial_field(cfg)
    r = pdhg.step(op, U, cfg["ht"], oracle_opts(cfg))
    p = rd.problem_from_config(cfg)
    u64, i64 = ctx.step(dev(U), cfg["ht"], p, rd.make_opts(tol=cfg["tol"], tau_u=0.9, tau_p=0.9))
    assert i64["iters"] == r.iters and max_abs(u64.cpu().numpy(), r.U) <= 1e-10
    umx, imx = ctx.step(dev(U), cfg["ht"], p, rd.make_opts(tol=cfg["tol"], tau_u=0.9, tau_p=0.9, precision="mixed"))
    assert imx["status"] == "ok" and max_abs(umx.cpu().numpy(), r.U) <= 1e-5


def test_3d_in_the_serving_mix(ctx, rd):
    """A 3-D trajectory served next to 2-D ones equals its steps alone, bitwise."""
    cfg = cfg3("allen_cahn", 32, "periodic")
    U = wl.initial_field(cfg)
    p3 = rd.problem_from_config(cfg)
    o = rd.make_opts(tol=cfg["tol"], precision="mixed")
    alone = dev(U)
    for _ in range(2):
        alone, _ = ctx.step(alone, cfg["ht"], p3, o)
    sc = rd.Context(0)
    try:
        t3 = sc.open(p3, o, dev(U))
        p2 = rd.make_problem("allen_cahn", 64, diff=(1e-4,))
        t2 = sc.open(p2, o, dev(wl.uniform_field(64, -0.1, 0.1, 3)))
        tickets = [t3.submit(cfg["ht"]), t2.submit(1e-3), t3.submit(cfg["ht"])]
        infos = {}
        for _ in range(20000):
            for tk in tickets:
                if tk not in infos:
                    i = sc.poll(tk)
                    if i is not None:
                        infos[tk] = i
            if len(infos) == len(tickets):
                break
            sc.pump()
        assert len(infos) == len(tickets)
        assert all(i["status"] == "ok" for i in infos.values())
        assert np.array_equal(t3.read().cpu().numpy(), alone.cpu().numpy())
        t3.close()
        t2.close()
    finally:
        sc.close()


def test_3d_argument_rules(ctx, rd):
    import torch
    u = torch.zeros((16, 16, 16), dtype=torch.float64, device="cuda")
    p = rd.make_problem("allen_cahn", 16, dim=3)
    with pytest.raises(rd.RDError):
        ctx.residual(u, u, 1e-3, p)
    with pytest.raises(rd.RDError):
        ctx.prox(u, 1e-3, p)
    bad = rd.make_problem("allen_cahn", 16, dim=3)
    bad.nz = 32
    ubad = torch.zeros((32, 16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(rd.RDError):     # the library refuses nz != nx
        ctx.step(ubad, 1e-3, bad, rd.make_opts())
    with pytest.raises(ValueError):     # the binding refuses a tensor of the wrong size
        ctx.step(u[:8].contiguous(), 1e-3, p, rd.make_opts())
    with pytest.raises(ValueError):
        ctx.precond_solve(torch.zeros((16, 16), dtype=torch.float64, device="cuda"), 1e-3, p)
    big = rd.make_problem("allen_cahn", 512, dim=3)
    assert rd.footprint_bytes(big, rd.make_opts()) == 0
    ch = rd.make_problem("cahn_hilliard", 16, dim=3)
    assert rd.footprint_bytes(ch, rd.make_opts()) == 0


def test_3d_kernel_timing(ctx, rd):
    cfg = cfg3("allen_cahn", 64, "periodic")
    p = rd.problem_from_config(cfg)
    u = dev(wl.initial_field(cfg))
    for prec in ("fp64", "mixed"):
        ms = ctx.profile_iteration(u, cfg["ht"], p, rd.make_opts(tol=cfg["tol"], precision=prec), reps=3)
        assert list(ms) == ["yfwd", "zsym", "yinv", "rowinv", "upd", "rowfwd"]
        assert all(0.0 < t < 100.0 for t in ms.values()), ms
