"""Pins of the oracle's sixth-order FCH equation (Sec. 3.3)."""
import numpy as np
import pytest

from oracle import equations as eq, grid, newton, pdhg, spectral


def fch(N=16, bc=grid.PERIODIC, L=2 * np.pi, eps=0.18):
    return eq.Problem(kind=eq.FCH, N=N, L=L, bc=bc, diff=(eps * eps,))


def paper_initial(prob):
    """u0(x, y) = 2 exp(sin x + sin y - 2) + 2.2 exp(-sin x - sin y - 2) - 1 (Sec. 3.3)."""
    x = np.arange(prob.N) * prob.h
    X, Y = np.meshgrid(x, x)
    return 2 * np.exp(np.sin(X) + np.sin(Y) - 2) + 2.2 * np.exp(-np.sin(X) - np.sin(Y) - 2) - 1


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_fch_preconditioner_inverts_the_cubic_stencil_operator(bc):
    """G = (I - alpha Lap + beta Lap^2 - gamma Lap^3)^2 applied with the sparse 5-point
    matrix undoes the transform solve (the cubic symbol matches the stencil)."""
    prob = fch(N=12, bc=bc, L=1.0)
    a, b, g = eq.precond_coeffs(prob, 1e-3)[0]
    assert a == 0.0 and b > 0.0 and g > 0.0
    Lm = grid.lap5_matrix(12, prob.h, bc)
    A = np.eye(144) - a * Lm.toarray() + b * (Lm @ Lm).toarray() - g * (Lm @ Lm @ Lm).toarray()
    w = np.random.default_rng(3).standard_normal((12, 12))
    y = spectral.precond_solve(w, prob.h, bc, a, b, g)
    np.testing.assert_allclose((A @ (A @ y.ravel())).reshape(12, 12), w, rtol=0, atol=1e-9 * np.abs(w).max())


def test_fch_preconditioner_is_the_papers():
    """beta mu^2 + gamma mu^3 = h_t eps^2 mu (eps^2 mu + 2 - eps^2) mu: the symbol of
    -h_t eps^2 Lap (eps^2 Lap - (2 - eps^2)) Lap with Lap -> -mu."""
    prob = fch()
    ht, e2 = 1e-3, 0.18 ** 2
    a, b, g = eq.precond_coeffs(prob, ht)[0]
    for mu in (0.5, 3.0, 40.0):
        assert b * mu ** 2 + g * mu ** 3 == pytest.approx(ht * e2 * mu * (e2 * mu + 2 - e2) * mu, rel=1e-14)


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_fch_constant_state_needs_no_iteration(bc):
    prob = fch(bc=bc)
    U = np.full((16, 16), 0.3)
    r = pdhg.step(prob, U, 1e-3, pdhg.Options(tol=1e-12, tau_u=0.58, tau_p=0.58))
    assert r.iters == 0 and np.array_equal(r.U, U)


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_fch_step_reaches_newton_root_and_conserves_mass(bc):
    prob = fch(N=12, bc=bc)
    U0 = paper_initial(prob)
    ht = 1e-3
    r = pdhg.step(prob, U0, ht, pdhg.Options(tol=1e-9, tau_u=0.58, tau_p=0.58))
    assert r.status == pdhg.OK
    root = newton.root(prob, U0, ht)
    assert np.max(np.abs(r.U - root.U)) <= 1e-8
    # sum F = sum(U - U^k): mass moves by at most N h_t ||Res||
    assert abs(r.U.sum() - U0.sum()) <= prob.N * ht * 1e-9 + 1e-12


def test_fch_paper_example_first_steps():
    """Sec. 3.3: [0, 2 pi]^2, eps = 0.18, N = 128 (h = pi / 64), h_t = 1e-3,
    tau = 0.58, delta = 0.5e-5: the steps converge (the paper reports no count)."""
    prob = fch(N=128)
    U = paper_initial(prob)
    for _ in range(2):
        r = pdhg.step(prob, U, 1e-3, pdhg.Options(tol=0.5e-5, tau_u=0.58, tau_p=0.58, max_iter=3000))
        assert r.status == pdhg.OK and r.iters < 3000
        U = r.U
