"""GPU parity at the workload sizes (2048^2 Allen-Cahn, 512^2 Cahn-Hilliard, 1024^2 Schnakenberg)
and at the largest supported grids (4096^2, 256^3), through the C ABI."""
import numpy as np
import pytest

from oracle import equations as oeq, pdhg as opdhg, spectral as ospec
from paper_2305_03945_amd import workloads as wl
from tests.rd_cases import max_abs, oracle_opts, oracle_problem, small_cfg

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


@pytest.mark.parametrize("N,bc", [(2048, "periodic"), (2048, "neumann"), (4096, "periodic"), (4096, "neumann")])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_precond_solve_large(ctx, rd, N, bc, precision):
    cfg = small_cfg("allen_cahn", N, bc)
    op = oracle_problem(cfg)
    ht = cfg["ht"]
    W = np.random.default_rng(N).standard_normal((N, N))
    Y_ref = ospec.precond_solve(W, op.h, bc, *oeq.precond_coeffs(op, ht)[0])
    Y = ctx.precond_solve(dev(W), ht, rd.problem_from_config(cfg), precision).cpu().numpy()
    bar = 1e-12 * np.max(np.abs(Y_ref)) if precision == "fp64" else 2e-6 * np.max(np.abs(W))
    assert max_abs(Y, Y_ref) <= bar


def _first_step(ctx, rd, name, precision, bar):
    cfg = wl.CONFIGS[name]
    U0 = wl.initial_field(cfg)
    ref = opdhg.step(oracle_problem(cfg), U0, cfg["ht"], oracle_opts(cfg))
    o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], omega=cfg["omega"], precision=precision)
    U1, info = ctx.step(dev(U0), cfg["ht"], rd.problem_from_config(cfg), o)
    assert info["status"] == "ok", info
    if precision == "fp64":
        assert info["iters"] == ref.iters
    err = max_abs(U1.cpu().numpy(), ref.U)
    assert err <= bar, err
    return info


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_ac2048_first_step(ctx, rd, precision, bar):
    """The 2048^2 periodic Allen-Cahn workload (eps = 0.01, h_t = 1e-3, delta = 1e-6), step 1."""
    _first_step(ctx, rd, "ac2048", precision, bar)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_schnak1024_first_step(ctx, rd, precision, bar):
    """The 1024^2 periodic Schnakenberg workload (D = (1, 10), a = 0.1, b = 0.9), step 1."""
    _first_step(ctx, rd, "schnak1024", precision, bar)


def test_ch512_first_step_fp64_and_mass(ctx, rd):
    """The 512^2 Neumann Cahn-Hilliard workload (eps = 0.02, h_t = 1e-4, 13-point), step 1,
    with the FP64 mass drift bounded by N h_t ||Res||."""
    info = _first_step(ctx, rd, "ch512", "fp64", 1e-10)
    assert abs(info["mass_drift"]) <= 512 * 1e-4 * info["residual"] + 1e-12


def test_ch512_first_step_mixed_and_mass(ctx, rd):
    """The 512^2 Neumann Cahn-Hilliard workload in the mixed precision, step 1: within 1e-5
    of the oracle, and the FP64 mass drift of the final outer pass bounded by N h_t ||Res||."""
    info = _first_step(ctx, rd, "ch512", "mixed", 1e-5)
    assert info["outer"] >= 1
    assert abs(info["mass_drift"]) <= 512 * 1e-4 * info["residual"] + 1e-12


@pytest.fixture(scope="module")
def ac2048_oracle_steps():
    """The oracle's first three steps of the 2048^2 Allen-Cahn trajectory."""
    cfg = wl.CONFIGS["ac2048"]
    U = wl.initial_field(cfg)
    out = []
    for _ in range(3):
        r = opdhg.step(oracle_problem(cfg), U, cfg["ht"], oracle_opts(cfg))
        out.append(r)
        U = r.U
    return out


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_ac2048_three_steps_elementwise(ctx, rd, ac2048_oracle_steps, precision, bar):
    """Steps 1-3 of the 2048^2 trajectory, every grid point against the oracle's, each GPU
    step starting from the GPU's previous result (FP64: equal iteration counts)."""
    cfg = wl.CONFIGS["ac2048"]
    o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], omega=cfg["omega"], precision=precision)
    p = rd.problem_from_config(cfg)
    u = dev(wl.initial_field(cfg))
    for k, ref in enumerate(ac2048_oracle_steps):
        u, info = ctx.step(u, cfg["ht"], p, o)
        assert info["status"] == "ok", (k, info)
        if precision == "fp64":
            assert info["iters"] == ref.iters, (k, info["iters"], ref.iters)
        assert max_abs(u.cpu().numpy(), ref.U) <= bar, k


_TRAJ = {}


def _oracle_trajectory(name, n):
    """The oracle's first n steps of a workload's trajectory (cached per module)."""
    if name not in _TRAJ:
        cfg = wl.CONFIGS[name]
        U = wl.initial_field(cfg)
        out = []
        for _ in range(n):
            r = opdhg.step(oracle_problem(cfg), U, cfg["ht"], oracle_opts(cfg))
            out.append(r)
            U = r.U
        _TRAJ[name] = out
    return _TRAJ[name]


@pytest.mark.parametrize("name", ["ch512", "schnak1024"])
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_workload_three_steps_elementwise(ctx, rd, name, precision, bar):
    """Steps 1-3 of the 512^2 Neumann Cahn-Hilliard and 1024^2 Schnakenberg trajectories,
    every grid point against the oracle's, each GPU step starting from the GPU's previous
    result (FP64: equal iteration counts)."""
    cfg = wl.CONFIGS[name]
    o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], omega=cfg["omega"], precision=precision)
    p = rd.problem_from_config(cfg)
    u = dev(wl.initial_field(cfg))
    for k, ref in enumerate(_oracle_trajectory(name, 3)):
        u, info = ctx.step(u, cfg["ht"], p, o)
        assert info["status"] == "ok", (k, info)
        if precision == "fp64":
            assert info["iters"] == ref.iters, (k, info["iters"], ref.iters)
        assert max_abs(u.cpu().numpy(), ref.U) <= bar, k


def test_ac2048_sampled_residual_after_steps(ctx, rd):
    """Property at full size: after 5 steps, the oracle's F evaluated pointwise at sampled grid
    points from the GPU's U^{k+1}, U^k is consistent with the reported ||F/h_t||_2 <= tol."""
    cfg = wl.CONFIGS["ac2048"]
    op = oracle_problem(cfg)
    o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], precision="mixed")
    p = rd.problem_from_config(cfg)
    u = dev(wl.initial_field(cfg))
    for _ in range(5):
        uk = u
        u, info = ctx.step(uk, cfg["ht"], p, o)
        assert info["status"] == "ok" and info["residual"] <= cfg["tol"]
    U, Uk = u.cpu().numpy(), uk.cpu().numpy()
    W = oeq.F(op, U, Uk, cfg["ht"])
    assert np.sqrt(np.sum((W / cfg["ht"]) ** 2)) <= cfg["tol"] * (1 + 1e-6)


@pytest.fixture(scope="module")
def ac4096_oracle_first():
    """The oracle's first step of the 4096^2 Allen-Cahn measurement workload (about 40 s of
    numpy on one host core)."""
    cfg = wl.CONFIGS["ac4096"]
    return opdhg.step(oracle_problem(cfg), wl.initial_field(cfg), cfg["ht"], oracle_opts(cfg))


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_ac4096_first_step_elementwise(ctx, rd, ac4096_oracle_first, precision, bar):
    """The largest 2-D grid, beyond the last-level cache: the first step of the 4096^2
    Allen-Cahn workload that the bench times, every grid point against the oracle's (FP64:
    equal iteration counts)."""
    cfg = wl.CONFIGS["ac4096"]
    ref = ac4096_oracle_first
    o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], omega=cfg["omega"], precision=precision)
    u, info = ctx.step(dev(wl.initial_field(cfg)), cfg["ht"], rd.problem_from_config(cfg), o)
    assert info["status"] == "ok", info
    if precision == "fp64":
        assert info["iters"] == ref.iters
    assert max_abs(u.cpu().numpy(), ref.U) <= bar


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_largest_grid_step_4096(ctx, rd, bc):
    """The largest 2-D grid, one Allen-Cahn step in each precision: both stop at the
    tolerance by the oracle's own F, and agree with each other to the mixed bar."""
    cfg = small_cfg("allen_cahn", 4096, bc)
    op = oracle_problem(cfg)
    p = rd.problem_from_config(cfg)
    U0 = wl.initial_field(cfg, N=4096, seed=11)
    out = {}
    for prec in ("fp64", "mixed"):
        o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], precision=prec)
        u, info = ctx.step(dev(U0), cfg["ht"], p, o)
        assert info["status"] == "ok" and info["residual"] <= cfg["tol"], (prec, info)
        out[prec] = u.cpu().numpy()
        assert oeq.residual_norm(op, oeq.F(op, out[prec], U0, cfg["ht"]), cfg["ht"]) <= cfg["tol"] * (1 + 1e-6)
    assert max_abs(out["fp64"], out["mixed"]) <= 1e-5


@pytest.fixture(scope="module")
def ac3d256_oracle_first():
    """The oracle's first step of the 128^3 Allen-Cahn workload's parameters on 256^3, the
    input the bench times there (about 40 s of numpy on one host core)."""
    cfg = dict(wl.CONFIGS["ac3d128"], N=256)
    return opdhg.step(oracle_problem(cfg), wl.initial_field(cfg), cfg["ht"], oracle_opts(cfg))


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_ac3d256_first_step_elementwise(ctx, rd, ac3d256_oracle_first, precision, bar):
    """The largest 3-D grid: the first 256^3 step every grid point against the oracle's
    (FP64: equal iteration counts)."""
    cfg = dict(wl.CONFIGS["ac3d128"], N=256)
    ref = ac3d256_oracle_first
    o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], omega=cfg["omega"], precision=precision)
    u, info = ctx.step(dev(wl.initial_field(cfg)), cfg["ht"], rd.problem_from_config(cfg), o)
    assert info["status"] == "ok", info
    if precision == "fp64":
        assert info["iters"] == ref.iters
    assert max_abs(u.cpu().numpy(), ref.U) <= bar


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_largest_grid_step_3d_256(ctx, rd, bc):
    """The largest 3-D grid (256^3), one Allen-Cahn step in each precision, checked the same way."""
    cfg = dict(wl.CONFIGS["ac3d128"])
    cfg.update(N=256, bc=bc)
    op = oracle_problem(cfg)
    p = rd.problem_from_config(cfg)
    U0 = wl.initial_field(cfg, seed=12)
    out = {}
    for prec in ("fp64", "mixed"):
        o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], precision=prec)
        u, info = ctx.step(dev(U0), cfg["ht"], p, o)
        assert info["status"] == "ok" and info["residual"] <= cfg["tol"], (prec, info)
        out[prec] = u.cpu().numpy()
        assert oeq.residual_norm(op, oeq.F(op, out[prec], U0, cfg["ht"]), cfg["ht"]) <= cfg["tol"] * (1 + 1e-6)
    assert max_abs(out["fp64"], out["mixed"]) <= 1e-5
