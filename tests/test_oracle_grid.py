"""Pins for the oracle's discrete operators (closed forms, the paper's printed blocks)."""
import json
import os

import numpy as np
import pytest

from oracle import grid, spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def fourier_mode(N, k, l):
    j = np.arange(N)
    phase = 2.0 * np.pi * (np.outer(j * l, np.ones(N)) + np.outer(np.ones(N), j * k)) / N
    return np.cos(phase), np.sin(phase)


def cosine_mode(N, k, l):
    j = np.arange(N)
    cx = np.cos(np.pi * k * (2 * j + 1) / (2 * N))
    cy = np.cos(np.pi * l * (2 * j + 1) / (2 * N))
    return np.outer(cy, cx)


@pytest.mark.parametrize("N", [8, 16])
def test_lap5_periodic_fourier_modes(N):
    h = 1.0 / N
    for k, l in [(0, 0), (1, 0), (0, 3), (2, 5), (N // 2, N // 2), (N - 1, 1)]:
        mu = 4.0 / h ** 2 * (np.sin(np.pi * k / N) ** 2 + np.sin(np.pi * l / N) ** 2)
        for m in fourier_mode(N, k, l):
            np.testing.assert_allclose(grid.lap5(m, h, grid.PERIODIC), -mu * m, atol=1e-9 * max(mu, 1))


@pytest.mark.parametrize("N", [8, 16])
def test_lap5_neumann_cosine_modes(N):
    h = 0.7 / N
    for k, l in [(0, 0), (1, 0), (0, 3), (2, 5), (N - 1, N - 1)]:
        mu = 4.0 / h ** 2 * (np.sin(np.pi * k / (2 * N)) ** 2 + np.sin(np.pi * l / (2 * N)) ** 2)
        m = cosine_mode(N, k, l)
        np.testing.assert_allclose(grid.lap5(m, h, grid.NEUMANN), -mu * m, atol=1e-9 * max(mu, 1))


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_eigen_table_matches_modes(bc):
    N, h = 16, 1.0 / 16
    s = spectral.laplacian_eigenvalues_1d(N, h, bc)
    for k in range(N):
        m = fourier_mode(N, k, 0)[0] if bc == grid.PERIODIC else cosine_mode(N, k, 0)
        np.testing.assert_allclose(grid.lap5(m, h, bc), -s[k] * m, atol=1e-9 * max(s[k], 1))


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
@pytest.mark.parametrize("N", [8, 16, 32])
def test_lap13_equals_lap5_squared(bc, N):
    rng = np.random.default_rng(N)
    u = rng.standard_normal((N, N))
    h = 1.0 / N
    a = grid.lap13(u, h, bc)
    b = grid.lap5(grid.lap5(u, h, bc), h, bc)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.max(np.abs(b)))


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_lap13_on_modes_gives_mu_squared(bc):
    N, h = 16, 1.0 / 16
    s = spectral.laplacian_eigenvalues_1d(N, h, bc)
    for k, l in [(1, 2), (3, 0), (7, 7)]:
        m = fourier_mode(N, k, l)[0] if bc == grid.PERIODIC else cosine_mode(N, k, l)
        mu = s[k] + s[l]
        np.testing.assert_allclose(grid.lap13(m, h, bc), mu * mu * m, atol=1e-9 * mu * mu)


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_stencil_matches_block_matrix(bc):
    N = 12
    h = 1.0 / N
    rng = np.random.default_rng(7)
    u = rng.standard_normal((N, N))
    M = grid.lap5_matrix(N, h, bc)
    np.testing.assert_allclose(grid.lap5(u, h, bc), grid.apply_matrix(M, u), rtol=1e-13, atol=1e-10)


def test_neumann_matrix_blocks_are_the_papers():
    g = golden()["neumann_blocks_N5"]
    N = 5
    M = grid.lap5_matrix(N, 1.0, grid.NEUMANN).toarray()
    blk = lambda i, j: M[i * N:(i + 1) * N, j * N:(j + 1) * N]
    np.testing.assert_array_equal(blk(0, 0), np.array(g["L1"]))
    np.testing.assert_array_equal(blk(N - 1, N - 1), np.array(g["L1"]))
    for i in range(1, N - 1):
        np.testing.assert_array_equal(blk(i, i), np.array(g["L2"]))
    for i in range(N - 1):
        np.testing.assert_array_equal(blk(i, i + 1), np.eye(N))
        np.testing.assert_array_equal(blk(i + 1, i), np.eye(N))
    np.testing.assert_array_equal(blk(0, N - 1), np.zeros((N, N)))


def test_periodic_matrix_blocks_are_the_papers():
    g = golden()["periodic_block_N5"]
    N = 5
    M = grid.lap5_matrix(N, 1.0, grid.PERIODIC).toarray()
    blk = lambda i, j: M[i * N:(i + 1) * N, j * N:(j + 1) * N]
    for i in range(N):
        np.testing.assert_array_equal(blk(i, i), np.array(g["L"]))
        np.testing.assert_array_equal(blk(i, (i + 1) % N), np.eye(N))
        np.testing.assert_array_equal(blk((i + 1) % N, i), np.eye(N))


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_laplacian_columns_sum_to_zero(bc):
    M = grid.lap5_matrix(8, 0.1, bc).toarray()
    np.testing.assert_allclose(M.sum(axis=0), 0.0, atol=1e-9)
