"""GPU parity of the kernel-level entry points against the oracle (through the C ABI)."""
import numpy as np
import pytest

from oracle import equations as oeq, grid as ogrid, prox as oprox, spectral as ospec
from tests.rd_cases import max_abs, oracle_problem, small_cfg

pytestmark = pytest.mark.gpu

KINDS = ["allen_cahn", "cahn_hilliard", "schnakenberg"]
BCS = ["periodic", "neumann"]


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


def field(prob, seed, base=None):
    rng = np.random.default_rng(seed)
    if prob.ncomp == 2:
        return np.stack([1.0 + rng.uniform(-0.3, 0.3, (prob.N, prob.N)), 0.9 + rng.uniform(-0.3, 0.3, (prob.N, prob.N))])
    return rng.uniform(-0.9, 0.9, (prob.N, prob.N))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("N", [16, 64, 256, 2048])
def test_residual_matches_oracle(ctx, rd, kind, bc, N):
    cfg = small_cfg(kind, N, bc)
    op = oracle_problem(cfg)
    ht = cfg["ht"]
    U, Uk = field(op, 1), field(op, 2)
    W_ref = oeq.F(op, U, Uk, ht)
    W, res = ctx.residual(dev(U), dev(Uk), ht, rd.problem_from_config(cfg))
    W = W.cpu().numpy()
    scale = np.max(np.abs(W_ref))
    assert max_abs(W, W_ref) <= 1e-13 * scale
    assert res == pytest.approx(oeq.residual_norm(op, W_ref, ht), rel=1e-12)


@pytest.mark.parametrize("kind", KINDS + ["heat", "biharmonic"])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("N", [16, 32, 128, 512])
def test_precond_solve_fp64_matches_oracle(ctx, rd, kind, bc, N):
    base = {"heat": "allen_cahn", "biharmonic": "cahn_hilliard"}.get(kind, kind)
    cfg = small_cfg(base, N, bc)
    cfg["kind"] = kind
    op = oracle_problem(cfg)
    ht = cfg["ht"]
    rng = np.random.default_rng(N)
    shape = (op.ncomp, N, N) if op.ncomp == 2 else (N, N)
    W = rng.standard_normal(shape)
    coeffs = oeq.precond_coeffs(op, ht)
    if op.ncomp == 1:
        Y_ref = ospec.precond_solve(W, op.h, bc, *coeffs[0])
    else:
        Y_ref = np.stack([ospec.precond_solve(W[c], op.h, bc, *coeffs[c]) for c in range(2)])
    Y = ctx.precond_solve(dev(W), ht, rd.problem_from_config(cfg), "fp64").cpu().numpy()
    assert max_abs(Y, Y_ref) <= 1e-12 * np.max(np.abs(Y_ref))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("N", [16, 256, 1024])
def test_precond_solve_fp32_matches_oracle(ctx, rd, kind, bc, N):
    cfg = small_cfg(kind, N, bc)
    op = oracle_problem(cfg)
    ht = cfg["ht"]
    rng = np.random.default_rng(N + 1)
    shape = (op.ncomp, N, N) if op.ncomp == 2 else (N, N)
    W = rng.standard_normal(shape)
    coeffs = oeq.precond_coeffs(op, ht)
    if op.ncomp == 1:
        Y_ref = ospec.precond_solve(W, op.h, bc, *coeffs[0])
    else:
        Y_ref = np.stack([ospec.precond_solve(W[c], op.h, bc, *coeffs[c]) for c in range(2)])
    Y = ctx.precond_solve(dev(W), ht, rd.problem_from_config(cfg), "mixed").cpu().numpy()
    # FP32 transforms: error ~ eps32 * log2(N) relative to the field's magnitude
    assert max_abs(Y, Y_ref) <= 2e-6 * np.max(np.abs(W))


@pytest.mark.parametrize("kind", ["allen_cahn", "schnakenberg"])
@pytest.mark.parametrize("N", [64, 256])
def test_prox_matches_oracle(ctx, rd, kind, N):
    cfg = small_cfg(kind, N, "periodic")
    op = oracle_problem(cfg)
    ht = 5e-2
    c = field(op, 3)
    ref = oprox.reaction_prox(op, c, ht)
    got = ctx.prox(dev(c), ht, rd.problem_from_config(cfg)).cpu().numpy()
    assert max_abs(got, ref) <= 1e-14 * max(1.0, np.max(np.abs(ref)))
