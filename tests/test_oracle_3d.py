"""Pins of the oracle's 3-D grids (7-point Laplacian): the method is posed on a
domain in R^d (Sec. 2); the operators, the preconditioner and Algorithm 1 carry
over with the 7-point stencil and 3-D transforms."""
import numpy as np
import pytest

from oracle import equations as eq, grid, newton, pdhg, prox, spectral


def prob3(kind=eq.ALLEN_CAHN, N=8, bc=grid.PERIODIC, **kw):
    base = dict(diff=(2.5e-3,), b=1.0)
    if kind == eq.SCHNAKENBERG:
        base = dict(diff=(1.0, 10.0), a=0.1, sb=0.9, kappa=1.0)
    base.update(kw)
    return eq.Problem(kind=kind, N=N, L=1.0, bc=bc, dim=3, **base)


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_lap7_eigenmodes(bc):
    N, h = 8, 1.0 / 8
    s = spectral.laplacian_eigenvalues_1d(N, h, bc)
    j = np.arange(N)
    for kx, ky, kz in [(1, 0, 0), (2, 3, 1), (3, 3, 5), (0, 0, 0)]:
        if bc == grid.PERIODIC:
            m = [np.cos(2 * np.pi * k * j / N) for k in (kz, ky, kx)]
        else:
            m = [np.cos(np.pi * k * (2 * j + 1) / (2 * N)) for k in (kz, ky, kx)]
        e = m[0][:, None, None] * m[1][None, :, None] * m[2][None, None, :]
        np.testing.assert_allclose(grid.lap7(e, h, bc), -(s[kx] + s[ky] + s[kz]) * e, atol=1e-10 * (1 + s.max()))


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_lap7_stencil_matches_matrix_and_reduces_to_lap5(bc):
    N, h = 6, 0.2
    u = np.random.default_rng(1).standard_normal((N, N, N))
    M = grid.lap7_matrix(N, h, bc)
    np.testing.assert_allclose(grid.lap7(u, h, bc), (M @ u.ravel()).reshape(N, N, N), rtol=1e-12, atol=1e-10)
    # a field constant along z: the 3-D Laplacian is the 2-D one of every slice
    v = np.random.default_rng(2).standard_normal((N, N))
    w = np.broadcast_to(v, (N, N, N)).copy()
    for z in range(N):
        np.testing.assert_allclose(grid.lap7(w, h, bc)[z], grid.lap5(v, h, bc), rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_precond_3d_inverts_the_stencil_operator(bc):
    N, h, alpha = 6, 1.0 / 6, 0.01
    M = grid.lap7_matrix(N, h, bc).toarray()
    A = np.eye(N ** 3) - alpha * M
    w = np.random.default_rng(3).standard_normal((N, N, N))
    y = spectral.precond_solve(w, h, bc, alpha, 0.0)
    np.testing.assert_allclose((A @ (A @ y.ravel())).reshape(N, N, N), w, atol=1e-10 * np.abs(w).max())


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_heat_3d_exact_in_two_iterations(bc):
    p = prob3(eq.HEAT, bc=bc)
    U = np.random.default_rng(4).uniform(-1, 1, p.shape)
    r = pdhg.step(p, U, 1e-2, pdhg.Options(tol=0.0, max_iter=2, tau_u=1.0, tau_p=1.0))
    M = grid.lap7_matrix(p.N, p.h, bc).toarray()
    exact = np.linalg.solve(np.eye(p.N ** 3) - 1e-2 * p.lam * M, U.ravel()).reshape(p.shape)
    assert np.max(np.abs(r.U - exact)) <= 1e-12


@pytest.mark.parametrize("kind", [eq.ALLEN_CAHN, eq.SCHNAKENBERG])
@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_3d_step_reaches_newton_root(kind, bc):
    p = prob3(kind, N=6, bc=bc)
    rng = np.random.default_rng(5)
    if kind == eq.SCHNAKENBERG:
        U = np.stack([1.0 + 0.05 * rng.uniform(-1, 1, p.shape), 0.9 + 0.05 * rng.uniform(-1, 1, p.shape)])
    else:
        U = rng.uniform(-0.9, 0.9, p.shape)
    r = pdhg.step(p, U, 1e-3, pdhg.Options(tol=1e-10))
    assert r.status == pdhg.OK
    root = newton.root(p, U, 1e-3)
    assert np.max(np.abs(r.U - root.U)) <= 1e-10


def test_3d_constant_states():
    p = prob3(eq.ALLEN_CAHN, N=6)
    U = np.full(p.shape, 0.37)
    r = pdhg.step(p, U, 1e-2, pdhg.Options(tol=1e-12))
    np.testing.assert_allclose(r.U, prox.ac_cubic_root(U, 1e-2, 1.0), rtol=0, atol=1e-12)
    s = prob3(eq.SCHNAKENBERG, N=6)
    V = np.stack([np.ones(s.shape), np.full(s.shape, 0.9)])
    assert pdhg.step(s, V, 1e-3, pdhg.Options(tol=1e-10)).iters == 0


def test_3d_z_invariant_step_equals_2d_step():
    """A 3-D state constant along z steps like its 2-D slice (same iterations)."""
    p2 = eq.Problem(kind=eq.ALLEN_CAHN, N=8, bc=grid.PERIODIC, diff=(2.5e-3,), b=1.0)
    p3 = prob3(eq.ALLEN_CAHN, N=8)
    v = np.random.default_rng(6).uniform(-0.9, 0.9, (8, 8))
    r2 = pdhg.step(p2, v, 1e-2, pdhg.Options(tol=1e-10))
    r3 = pdhg.step(p3, np.broadcast_to(v, (8, 8, 8)).copy(), 1e-2, pdhg.Options(tol=1e-10 * np.sqrt(8)))
    assert r2.iters == r3.iters
    for z in range(8):
        assert np.max(np.abs(r3.U[z] - r2.U)) <= 1e-12
