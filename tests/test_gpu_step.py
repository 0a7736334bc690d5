"""GPU parity of rd_step (Algorithm 1 on the device) against the oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import equations as oeq, pdhg as opdhg
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


def gpu_opts(rd, cfg, precision="fp64", tol=None, max_iter=10000, init="prev", inner_rtol=3e-2):
    return rd.make_opts(tol=cfg["tol"] if tol is None else tol, max_iter=max_iter, tau_u=cfg["tau"],
                        tau_p=cfg["tau"], omega=cfg["omega"], precision=precision, init=init,
                        inner_rtol=inner_rtol)


def compare_fp64(ctx, rd, cfg, U0, steps, tol=None, init="prev"):
    """Run `steps` steps on both sides; iteration counts must match and the states agree to 1e-10."""
    op = oracle_problem(cfg)
    oo = oracle_opts(cfg, tol=tol, init=init)
    p = rd.problem_from_config(cfg)
    o = gpu_opts(rd, cfg, tol=tol, init=init)
    Ug = dev(U0)
    U = np.array(U0)
    for k in range(steps):
        r = opdhg.step(op, U, cfg["ht"], oo)
        Ug, info = ctx.step(Ug, cfg["ht"], p, o)
        assert info["status"] == "ok", (k, info)
        assert info["iters"] == r.iters, (k, info, r.iters, r.residual)
        # The reported norm is a round-off-level quantity near the tolerance: agree loosely.
        assert info["residual"] == pytest.approx(r.residual, rel=1e-3, abs=1e-2 * (tol or cfg["tol"]))
        err = max_abs(Ug.cpu().numpy(), r.U)
        assert err <= 1e-10, (k, err)
        U = r.U
    return U


def test_ac64_ten_steps_fp64(ctx, rd):
    """The 64^2 periodic Allen-Cahn workload (eps = 0.05, h_t = 0.01, delta = 1e-10), all 10 steps."""
    cfg = wl.CONFIGS["ac64"]
    compare_fp64(ctx, rd, cfg, wl.initial_field(cfg), cfg["steps"])


@pytest.mark.parametrize("kind", ["allen_cahn", "cahn_hilliard", "schnakenberg"])
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("N", [16, 64, 128])
def test_step_fp64_matches_oracle(ctx, rd, kind, bc, N):
    cfg = small_cfg(kind, N, bc)
    tol = {"allen_cahn": 1e-8, "cahn_hilliard": 1e-5, "schnakenberg": 1e-7}[kind]
    compare_fp64(ctx, rd, cfg, wl.initial_field(cfg, N=N, seed=7), 2, tol=tol)


@pytest.mark.parametrize("kind", ["allen_cahn", "schnakenberg"])
@pytest.mark.parametrize("N", [512, 1024])
def test_step_periodic_large_columns(ctx, rd, kind, N):
    """Periodic grids whose column transforms run from registers (N >= 512): one
    step in FP64 (equal iterations, 1e-10) and in mixed precision (1e-5)."""
    cfg = small_cfg(kind, N, "periodic")
    tol = 1e-7 if kind == "allen_cahn" else 1e-5
    U0 = wl.initial_field(cfg, N=N, seed=10)
    U1 = compare_fp64(ctx, rd, cfg, U0, 1, tol=tol)
    Ug, info = ctx.step(dev(U0), cfg["ht"], rd.problem_from_config(cfg), gpu_opts(rd, cfg, "mixed", tol=tol))
    assert info["status"] == "ok" and info["residual"] <= tol
    assert max_abs(Ug.cpu().numpy(), U1) <= 1e-5


@pytest.mark.parametrize("kind,N", [("allen_cahn", 512), ("schnakenberg", 512), ("allen_cahn", 1024)])
def test_step_neumann_large(ctx, rd, kind, N):
    """Neumann (DCT-II) grids of 512^2 (two rows per row workgroup) and 1024^2 (four):
    one step in FP64 (equal iterations, 1e-10) and in mixed precision (1e-5)."""
    cfg = small_cfg(kind, N, "neumann")
    tol = 1e-7 if kind == "allen_cahn" else 1e-5
    U0 = wl.initial_field(cfg, N=N, seed=17)
    U1 = compare_fp64(ctx, rd, cfg, U0, 1, tol=tol)
    Ug, info = ctx.step(dev(U0), cfg["ht"], rd.problem_from_config(cfg), gpu_opts(rd, cfg, "mixed", tol=tol))
    assert info["status"] == "ok" and info["residual"] <= tol
    assert max_abs(Ug.cpu().numpy(), U1) <= 1e-5


@pytest.mark.parametrize("kind", ["allen_cahn", "schnakenberg"])
@pytest.mark.parametrize("N,bc", [(64, "periodic"), (256, "periodic"), (256, "neumann")])
def test_step_fp64_prox_init_matches_oracle(ctx, rd, kind, N, bc):
    """U_0 = prox(U^k): the single-workgroup step (64^2) and the batched initial pass (256^2)."""
    cfg = small_cfg(kind, N, bc)
    tol = 1e-8 if kind == "allen_cahn" else 1e-7
    compare_fp64(ctx, rd, cfg, wl.initial_field(cfg, N=N, seed=8), 2, tol=tol, init="prox")


@pytest.mark.parametrize("kind", ["allen_cahn", "schnakenberg"])
@pytest.mark.parametrize("N", [64, 256])
def test_step_mixed_prox_init_matches_oracle(ctx, rd, kind, N):
    """The mixed step from U_0 = prox(U^k) reaches the oracle's root within the mixed bar."""
    cfg = small_cfg(kind, N, "periodic")
    tol = 1e-8 if kind == "allen_cahn" else 1e-7
    op = oracle_problem(cfg)
    U = wl.initial_field(cfg, N=N, seed=8)
    r = opdhg.step(op, U, cfg["ht"], oracle_opts(cfg, tol=tol, init="prox"))
    Ug, info = ctx.step(dev(U), cfg["ht"], rd.problem_from_config(cfg),
                        gpu_opts(rd, cfg, precision="mixed", tol=tol, init="prox"))
    assert info["status"] == "ok" and info["residual"] <= tol, info
    assert max_abs(Ug.cpu().numpy(), r.U) <= 1e-5


@pytest.mark.parametrize("kind", ["allen_cahn", "cahn_hilliard", "schnakenberg"])
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("N", [32, 64, 256])
def test_step_mixed_matches_oracle(ctx, rd, kind, bc, N):
    cfg = small_cfg(kind, N, bc)
    tol = {"allen_cahn": 1e-8, "cahn_hilliard": 1e-5, "schnakenberg": 1e-7}[kind]
    op = oracle_problem(cfg)
    U = wl.initial_field(cfg, N=N, seed=9)
    p = rd.problem_from_config(cfg)
    o = gpu_opts(rd, cfg, precision="mixed", tol=tol)
    Ug = dev(U)
    for k in range(2):
        r = opdhg.step(op, U, cfg["ht"], oracle_opts(cfg, tol=tol))
        Ug, info = ctx.step(Ug, cfg["ht"], p, o)
        assert info["status"] == "ok", info
        assert info["residual"] <= tol
        assert info["outer"] >= 1
        err = max_abs(Ug.cpu().numpy(), r.U)
        assert err <= 1e-5, (k, err)
        # The mixed result is a root of the same equation to the same tolerance.
        W = oeq.F(op, Ug.cpu().numpy(), U, cfg["ht"])
        assert oeq.residual_norm(op, W, cfg["ht"]) <= tol * (1 + 1e-6)
        U = r.U
        Ug = dev(U)


def test_heat_step_exact_in_two_iterations(ctx, rd):
    """f = 0, tau = omega = 1: the root after exactly two iterations (derived from the G-prox
    dynamic; pins the transform scaling and symbol against the stencil)."""
    N = 64
    cfg = dict(kind="heat", N=N, L=1.0, bc="neumann", diff=(0.02,), ht=0.5, tol=0.0, tau=1.0, omega=1.0)
    op = oracle_problem(cfg)
    U = wl.uniform_field(N, -1, 1, 3)
    p = rd.problem_from_config(cfg)
    o = gpu_opts(rd, cfg, tol=0.0, max_iter=2)
    Ug, info = ctx.step(dev(U), 0.5, p, o)
    assert info["iters"] == 2
    ref = opdhg.step(op, U, 0.5, opdhg.Options(tol=1e-13, tau_u=1.0, tau_p=1.0)).U
    assert max_abs(Ug.cpu().numpy(), ref) <= 1e-12


def test_bitwise_determinism_and_odd_symmetry(ctx, rd):
    cfg = small_cfg("allen_cahn", 256, "periodic")
    U = wl.initial_field(cfg, N=256, seed=11)
    p = rd.problem_from_config(cfg)
    o = gpu_opts(rd, cfg, tol=1e-8)
    a, ia = ctx.step(dev(U), cfg["ht"], p, o)
    b, ib = ctx.step(dev(U), cfg["ht"], p, o)
    c, ic = ctx.step(dev(-U), cfg["ht"], p, o)
    assert ia["iters"] == ib["iters"] == ic["iters"]
    a, b, c = a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()
    assert np.array_equal(a, b)
    assert np.array_equal(c, -a)


def test_cahn_hilliard_mass_drift_reported(ctx, rd):
    cfg = small_cfg("cahn_hilliard", 128, "neumann")
    U = wl.initial_field(cfg, N=128, seed=12)
    p = rd.problem_from_config(cfg)
    o = gpu_opts(rd, cfg, tol=1e-4)
    Ug, info = ctx.step(dev(U), cfg["ht"], p, o)
    drift = float(np.sum(Ug.cpu().numpy()) - np.sum(U))
    assert abs(info["mass_drift"] - drift) <= 1e-9
    assert abs(drift) <= 128 * cfg["ht"] * info["residual"] + 1e-12


def test_noconv_and_nonfinite_and_invalid(ctx, rd):
    cfg = small_cfg("allen_cahn", 64, "periodic")
    U = wl.initial_field(cfg, N=64, seed=13)
    p = rd.problem_from_config(cfg)
    _, info = ctx.step(dev(U), cfg["ht"], p, gpu_opts(rd, cfg, tol=1e-12, max_iter=1))
    assert info["status"] == "noconv" and info["iters"] == 1
    Ubad = U.copy()
    Ubad[3, 5] = np.nan
    _, info = ctx.step(dev(Ubad), cfg["ht"], p, gpu_opts(rd, cfg))
    assert info["status"] == "nonfinite"
    _, info = ctx.step(dev(Ubad), cfg["ht"], p, gpu_opts(rd, cfg, precision="mixed"))
    assert info["status"] == "nonfinite"
    bad = rd.make_problem("allen_cahn", 48)
    with pytest.raises(rd.RDError):
        ctx.step(dev(np.zeros((48, 48))), 1e-3, bad, gpu_opts(rd, cfg))
    with pytest.raises(rd.RDError):
        ctx.step(dev(U), -1.0, p, gpu_opts(rd, cfg))


def test_zero_iterations_when_start_is_converged(ctx, rd):
    cfg = small_cfg("schnakenberg", 64, "periodic")
    a, b = cfg["a"], cfg["sb"]
    U = np.stack([np.full((64, 64), a + b), np.full((64, 64), b / (a + b) ** 2)])
    Ug, info = ctx.step(dev(U), cfg["ht"], rd.problem_from_config(cfg), gpu_opts(rd, cfg, tol=1e-9))
    assert info["iters"] == 0 and info["status"] == "ok"
    assert np.array_equal(Ug.cpu().numpy(), U)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dim", [2, 3])
def test_in_place_step_equals_out_of_place(ctx, rd, precision, dim):
    """u_n and u_np1 may alias: the in-place step gives bitwise the out-of-place result."""
    N = 64 if dim == 2 else 32
    cfg = small_cfg("allen_cahn", N, "periodic")
    cfg["dim"] = dim
    U0 = wl.uniform_field(N, -0.5, 0.5, 14, dim)
    p = rd.problem_from_config(cfg)
    o = gpu_opts(rd, cfg, precision, tol=1e-8)
    ref, i_ref = ctx.step(dev(U0), cfg["ht"], p, o)
    u = dev(U0)
    out, info = ctx.step(u, cfg["ht"], p, o, out=u)
    assert out.data_ptr() == u.data_ptr()
    assert info["iters"] == i_ref["iters"] and info["status"] == "ok"
    assert np.array_equal(u.cpu().numpy(), ref.cpu().numpy())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dim", [2, 3])
def test_step_independent_of_schedule_history(rd, precision, dim):
    """The host enqueues a step's iterations in chunks whose length it predicts from
    the previous steps on the same workspace; the device decides every inner loop,
    outer update and stop itself.  A step run after steps of very different length
    (so its first chunk is far too long or far too short) gives bitwise the result,
    iterations and outer passes of the same step in a fresh context."""
    N = 64 if dim == 2 else 16
    cfg = small_cfg("allen_cahn", N, "periodic")
    cfg["dim"] = dim
    p = rd.problem_from_config(cfg)
    o = gpu_opts(rd, cfg, precision, tol=1e-8)
    U0 = wl.uniform_field(N, -0.5, 0.5, 16, dim)
    fresh = rd.Context(0)
    try:
        ref, iref = fresh.step(dev(U0), 1e-3, p, o)
    finally:
        fresh.close()
    for history in ([1e-6, 1e-6, 1e-6], [1e-2, 3e-2, 5e-2]):   # short steps, then long ones
        c = rd.Context(0)
        try:
            for ht in history:
                c.step(dev(U0), ht, p, o)
            u, info = c.step(dev(U0), 1e-3, p, o)
            assert info["status"] == "ok" and info["iters"] == iref["iters"] and info["outer"] == iref["outer"]
            assert np.array_equal(u.cpu().numpy(), ref.cpu().numpy()), history
        finally:
            c.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_output_bound_as_iterate_buffer(rd, precision):
    """rd_step binds the output as the iterate buffer the previous step ended in (and
    skips the final copy when the step ends there; for an output that overlaps the input
    only the buffer the initial pass does not write).  Chains of in-place, ping-pong and
    fresh-output steps of varying length give bitwise the results of steps taken one by
    one in fresh contexts."""
    import torch
    N = 64
    cfg = small_cfg("allen_cahn", N, "periodic")
    p = rd.problem_from_config(cfg)
    o = gpu_opts(rd, cfg, precision, tol=1e-8)
    hts = [1e-3, 2e-3, 5e-4, 3e-3, 1e-3, 1e-3, 4e-3, 2e-3]
    ref = [dev(wl.uniform_field(N, -0.5, 0.5, 18))]
    for ht in hts:
        f = rd.Context(0)
        try:
            u, _ = f.step(ref[-1], ht, p, o)
        finally:
            f.close()
        ref.append(u)
    c = rd.Context(0)
    try:
        a = ref[0].clone()
        b = torch.empty_like(a)
        for k, ht in enumerate(hts):
            mode = k % 3
            if mode == 0:                     # in place
                c.step(a, ht, p, o, out=a)
            elif mode == 1:                   # ping-pong
                c.step(a, ht, p, o, out=b)
                a, b = b, a
            else:                             # a fresh output
                a, _ = c.step(a, ht, p, o)
            assert np.array_equal(a.cpu().numpy(), ref[k + 1].cpu().numpy()), (k, mode)
    finally:
        c.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_unaligned_output_buffer(ctx, rd, precision):
    """The result reaches an output buffer at any 8-byte offset (the device-side copy
    needs 32-byte alignment; other buffers take the host-enqueued copy): bitwise the
    aligned result, and the doubles around the output are untouched."""
    import torch
    N = 64
    cfg = small_cfg("allen_cahn", N, "periodic")
    U0 = wl.uniform_field(N, -0.5, 0.5, 15)
    p = rd.problem_from_config(cfg)
    o = gpu_opts(rd, cfg, precision, tol=1e-8)
    ref, i_ref = ctx.step(dev(U0), cfg["ht"], p, o)
    for off in (1, 2, 3, 4):
        big = torch.full((N * N + 8,), 7.0, dtype=torch.float64, device="cuda")
        out = big[off:off + N * N].view(N, N)
        _, info = ctx.step(dev(U0), cfg["ht"], p, o, out=out)
        assert info["iters"] == i_ref["iters"] and info["status"] == "ok"
        assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy()), off
        rest = torch.cat([big[:off], big[off + N * N:]]).cpu().numpy()
        assert np.all(rest == 7.0), off


def test_two_contexts_interleaved(ctx, rd):
    """Two contexts on one device, used in turn on problems that share grid sizes (so each
    holds its own cached workspaces and tables for them): every result is bitwise the
    result of the same steps on one context alone."""
    import torch
    cases = [(small_cfg("allen_cahn", 256, "periodic"), "fp64"), (small_cfg("allen_cahn", 256, "neumann"), "mixed"),
             (small_cfg("schnakenberg", 64, "periodic"), "fp64"), (small_cfg("cahn_hilliard", 64, "neumann"), "mixed")]
    runs = []
    for cfg, prec in cases:
        p, o = rd.problem_from_config(cfg), gpu_opts(rd, cfg, prec)
        u0 = dev(wl.initial_field(cfg, N=cfg["N"], seed=cfg["N"] + 7))
        runs.append((p, o, cfg["ht"], u0))
    alone = []
    for p, o, ht, u0 in runs:
        u = u0
        for _ in range(2):
            u, _ = ctx.step(u, ht, p, o)
        alone.append(u)
    other = rd.Context(0)
    try:
        states = [[u0, u0] for _, _, _, u0 in runs]
        for _ in range(2):
            for i, (p, o, ht, _) in enumerate(runs):
                states[i][0], _ = ctx.step(states[i][0], ht, p, o)
                states[i][1], _ = other.step(states[i][1], ht, p, o)
        for (a, b), ref in zip(states, alone):
            assert torch.equal(a, ref) and torch.equal(b, ref)
    finally:
        other.close()


def test_invalid_problems_rejected_before_any_device_work(ctx, rd):
    """Shapes and operator/reaction pairs the library does not take: rd_footprint_bytes
    is 0 and rd_step returns RD_E_INVALID, without touching the (one-value) buffers."""
    import ctypes
    import torch
    base = dict(kind="allen_cahn", N=64)
    cases = []
    for N in (0, 8, 48, 8192):                       # empty, below 16, not a power of two, above 4096
        cases.append(rd.make_problem("allen_cahn", N))
    p = rd.make_problem("allen_cahn", 64); p.ny = 32; cases.append(p)       # not square
    p = rd.make_problem("allen_cahn", 64); p.ly = 2.0; cases.append(p)      # unequal sides
    p = rd.make_problem("allen_cahn", 64); p.lx = p.ly = 0.0; cases.append(p)
    p = rd.make_problem("allen_cahn", 64); p.bc = 7; cases.append(p)
    p = rd.make_problem("allen_cahn", 64); p.rx = rd.RD_RX_CAHN_HILLIARD; cases.append(p)   # LAP5 + CH
    p = rd.make_problem("allen_cahn", 64); p.diff[0] = -1.0; cases.append(p)
    p = rd.make_problem("allen_cahn", 64); p.nz = -1; cases.append(p)
    p = rd.make_problem("cahn_hilliard", 64, dim=3); cases.append(p)        # no 13-point 3-D form
    p = rd.make_problem("allen_cahn", 512, dim=3); cases.append(p)          # 3-D above 256
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    ptr = ctypes.c_void_p(one.data_ptr())
    o = rd.make_opts()
    for p in cases:
        assert rd.footprint_bytes(p, o) == 0
        info = rd.Info()
        code = rd._lib.rd_step(ctx._h, ctypes.byref(p), ctypes.byref(o), ctypes.c_double(1e-3), ptr, ptr,
                               rd._stream_ptr(None), ctypes.byref(info))
        assert code == rd.RD_E_INVALID, (p.nx, p.ny, p.nz, p.op, p.rx)


def test_degenerate_steps(ctx, rd):
    """A vanishing step size (h_t = 1e-9; the plain norm's round-off floor, about
    eps |U| N / h_t, sets the tolerance) moves U by O(h_t) in a few iterations, as in the
    oracle; max_iter = 0 returns U^k unchanged with status noconv; both precisions."""
    cfg = small_cfg("allen_cahn", 64, "periodic")
    U = wl.initial_field(cfg, N=64, seed=15)
    p = rd.problem_from_config(cfg)
    op = oracle_problem(cfg)
    drive = np.abs(oeq.F(op, U, U, 1.0)).max()          # max |lambda Lap U + f(U)|
    ht, tol = 1e-9, 1e-3
    r = opdhg.step(op, U, ht, oracle_opts(cfg, tol=tol))
    assert r.iters <= 10
    for precision in ("fp64", "mixed"):
        out, info = ctx.step(dev(U), ht, p, gpu_opts(rd, cfg, precision, tol=tol))
        assert info["status"] == "ok" and info["iters"] <= 20, info
        if precision == "fp64":
            assert info["iters"] == r.iters
            assert max_abs(out.cpu().numpy(), r.U) <= 1e-10
        assert max_abs(out.cpu().numpy(), U) <= 2 * ht * drive
        out, info = ctx.step(dev(U), cfg["ht"], p, gpu_opts(rd, cfg, precision, max_iter=0))
        assert info["status"] == "noconv" and info["iters"] == 0, info
        assert np.array_equal(out.cpu().numpy(), U)
