"""Pins for F, its Jacobian and the adjoint apply (finite differences, matrix transpose)."""
import numpy as np
import pytest

from oracle import equations as eq, grid


def make(kind, bc, N=8):
    if kind == eq.SCHNAKENBERG:
        return eq.Problem(kind=kind, N=N, bc=bc, diff=(0.05, 1.0), a=0.1305, sb=0.7695, kappa=100.0)
    if kind in (eq.CAHN_HILLIARD, eq.BIHARMONIC):
        return eq.Problem(kind=kind, N=N, bc=bc, diff=(4e-4,), b=1.0)
    return eq.Problem(kind=kind, N=N, bc=bc, diff=(2.5e-3,), b=1.0)


def rand_state(prob, seed):
    rng = np.random.default_rng(seed)
    shape = (prob.ncomp, prob.N, prob.N) if prob.ncomp > 1 else (prob.N, prob.N)
    base = 0.9 if prob.ncomp > 1 else 0.0
    return base + rng.uniform(-0.5, 0.5, shape)


@pytest.mark.parametrize("kind", eq.KINDS)
@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_jacobian_matches_finite_differences(kind, bc):
    prob = make(kind, bc)
    ht = 1e-3
    U = rand_state(prob, 1)
    Uk = rand_state(prob, 2)
    d = rand_state(prob, 3) - (0.9 if prob.ncomp > 1 else 0.0)
    J = eq.jacobian(prob, U, ht)
    jd = (J @ d.reshape(-1)).reshape(U.shape)
    eps = 1e-6
    fd = (eq.F(prob, U + eps * d, Uk, ht) - eq.F(prob, U - eps * d, Uk, ht)) / (2 * eps)
    np.testing.assert_allclose(jd, fd, rtol=1e-6, atol=1e-7 * np.max(np.abs(fd)))


@pytest.mark.parametrize("kind", eq.KINDS)
@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_adjoint_is_jacobian_transpose(kind, bc):
    prob = make(kind, bc)
    ht = 1e-3
    U = rand_state(prob, 4)
    P = rand_state(prob, 5)
    J = eq.jacobian(prob, U, ht)
    ref = (J.T @ P.reshape(-1)).reshape(U.shape)
    np.testing.assert_allclose(eq.adjoint(prob, U, P, ht), ref, rtol=1e-11, atol=1e-11 * np.max(np.abs(ref)))


def test_residual_norm_system_adds_component_norms():
    prob = make(eq.SCHNAKENBERG, grid.PERIODIC)
    W = np.stack([np.full((8, 8), 3.0), np.full((8, 8), 4.0)])
    assert eq.residual_norm(prob, W, 0.5) == pytest.approx(8 * 6.0 + 8 * 8.0)
