"""Pins for the oracle's transforms and preconditioner solve (textbook sums, dense solves)."""
import json
import os

import numpy as np
import pytest

from oracle import grid, spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


@pytest.mark.parametrize("N", [4, 8, 16])
def test_forward_transforms_match_naive_sums(N):
    rng = np.random.default_rng(N)
    w = rng.standard_normal((N, N))
    F = spectral.naive_dft_matrix(N)
    np.testing.assert_allclose(spectral.forward_transform(w, grid.PERIODIC), F @ w @ F.T, atol=1e-11)
    C = spectral.naive_dct2_matrix(N)
    np.testing.assert_allclose(spectral.forward_transform(w, grid.NEUMANN), C @ w @ C.T, atol=1e-11)
    np.testing.assert_allclose(C @ C.T, np.eye(N), atol=1e-13)


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_round_trip(bc):
    rng = np.random.default_rng(3)
    w = rng.standard_normal((16, 16))
    np.testing.assert_allclose(spectral.inverse_transform(spectral.forward_transform(w, bc), bc), w, atol=1e-13)


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
@pytest.mark.parametrize("alpha,beta", [(0.3, 0.0), (0.0, 0.002), (0.05, 0.001)])
@pytest.mark.parametrize("N", [8, 16])
def test_precond_solve_matches_dense_matrix(bc, alpha, beta, N):
    h = 1.0 / N
    rng = np.random.default_rng(11)
    w = rng.standard_normal((N, N))
    G = spectral.precond_matrix(N, h, bc, alpha, beta)
    y_dense = np.linalg.solve(G, w.reshape(-1)).reshape(N, N)
    y = spectral.precond_solve(w, h, bc, alpha, beta)
    # The dense solve loses about cond(G) * eps; G's condition number reaches ~1e8 here.
    cond = np.max(spectral.precond_symbol(N, h, bc, alpha, beta))
    np.testing.assert_allclose(y, y_dense, rtol=0, atol=100 * cond * 2.2e-16 * np.max(np.abs(y_dense)))


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_precond_solve_inverts_stencil_operator(bc):
    """G (G^-1 w) = w with G applied as two applications of (I - a Lap + b Lap Lap) by stencils."""
    N, h = 32, 1.0 / 32
    a, b = 0.01, 1e-6
    rng = np.random.default_rng(5)
    w = rng.standard_normal((N, N))
    y = spectral.precond_solve(w, h, bc, a, b)
    A = lambda v: v - a * grid.lap5(v, h, bc) + b * grid.lap13(v, h, bc)
    np.testing.assert_allclose(A(A(y)), w, atol=1e-10)


def test_heat_condition_number_formula():
    """Sec. 2.1: kappa(I - h_t lambda Lap^P) = 1 + 4 lambda N^2 h_t (1-D, unit length, even N)."""
    with open(GOLDEN) as f:
        cases = json.load(f)["heat_condition_number"]["cases"]
    for c in cases:
        N, lam, ht = c["N"], c["lambda"], c["ht"]
        T = np.diag(-2.0 * np.ones(N)) + np.diag(np.ones(N - 1), 1) + np.diag(np.ones(N - 1), -1)
        T[0, -1] = T[-1, 0] = 1.0
        A = np.eye(N) - ht * lam * T * N * N
        ev = np.linalg.eigvalsh(A)
        assert abs(ev.max() / ev.min() - (1.0 + 4.0 * lam * N * N * ht)) < 1e-9 * ev.max()
        s = spectral.laplacian_eigenvalues_1d(N, 1.0 / N, grid.PERIODIC)
        np.testing.assert_allclose(np.sort(1.0 + ht * lam * s), np.sort(ev), rtol=1e-12)
