"""Laplacian eigenvalues and the preconditioner solve ``Y = G^-1 W`` (FP64, test only).

The preconditioner of Sec. 2.1 ("Choosing the matrix G") is ``G = A A^T`` for the
linear part ``A`` of ``F``.  For every equation handled here ``A`` is a polynomial
in the 5-point Laplacian, so

    G = (I - alpha Lap + beta Lap Lap)^2,

with (alpha, beta) = (lambda h_t, 0) for Allen-Cahn / heat / each Schnakenberg
component (``D_i h_t``), and (0, lambda h_t) for Cahn-Hilliard / biharmonic.
For the sixth-order FCH equation (Sec. 3.3) a cubic term enters,
``G = (I - alpha Lap + beta Lap^2 - gamma Lap^3)^2`` with symbol
``(1 + alpha mu + beta mu^2 + gamma mu^3)^2``.
``G`` is diagonalised by the 2-D DFT for periodic grids (Sec. 2.1, "Application of
FFT") and by the 2-D DCT-II for Neumann grids (Remark 1).  With ``mu`` the
eigenvalue of ``-Lap`` the symbol is ``g = (1 + alpha mu + beta mu^2)^2``.

The transforms are library primitives (numpy / scipy pocketfft); tests pin them
against dense matrix solves and naive transform sums.
"""
import numpy as np
import scipy.fft as sfft

from . import grid


def laplacian_eigenvalues_1d(N, h, bc):
    """Eigenvalues ``s_k`` of the 1-D negative second difference, k = 0..N-1.

    Periodic (Fourier mode exp(2 pi i k j / N)): ``s_k = (4/h^2) sin^2(pi k / N)``;
    this is the formula behind the heat-equation example of Sec. 2.1.
    Neumann (DCT-II mode cos(pi k (2j+1) / (2N))): ``s_k = (4/h^2) sin^2(pi k / (2N))``.
    """
    k = np.arange(N, dtype=np.float64)
    if bc == grid.PERIODIC:
        return 4.0 / h ** 2 * np.sin(np.pi * k / N) ** 2
    if bc == grid.NEUMANN:
        return 4.0 / h ** 2 * np.sin(np.pi * k / (2 * N)) ** 2
    raise ValueError(bc)


def laplacian_symbol(N, h, bc, dim=2):
    """Eigenvalues of ``-Lap``: mu[ky, kx] = s_ky + s_kx (2-D), or
    mu[kz, ky, kx] = s_kz + s_ky + s_kx for the 7-point Laplacian (3-D)."""
    s = laplacian_eigenvalues_1d(N, h, bc)
    if dim == 3:
        return s[:, None, None] + s[None, :, None] + s[None, None, :]
    return s[:, None] + s[None, :]


def precond_symbol(N, h, bc, alpha, beta, gamma=0.0, dim=2):
    """Eigenvalues of ``G = (I - alpha Lap + beta Lap^2 - gamma Lap^3)^2`` on the grid."""
    mu = laplacian_symbol(N, h, bc, dim)
    return (1.0 + alpha * mu + beta * mu * mu + gamma * mu * mu * mu) ** 2


def forward_transform(w, bc):
    """DFT (periodic) or orthonormal DCT-II (Neumann) over every axis of the field."""
    if bc == grid.PERIODIC:
        return np.fft.fftn(w)
    if bc == grid.NEUMANN:
        return sfft.dctn(w, type=2, norm="ortho")
    raise ValueError(bc)


def inverse_transform(what, bc):
    """Inverse of ``forward_transform`` (real part for the periodic case)."""
    if bc == grid.PERIODIC:
        return np.real(np.fft.ifftn(what))
    if bc == grid.NEUMANN:
        return sfft.idctn(what, type=2, norm="ortho")
    raise ValueError(bc)


def precond_solve(w, h, bc, alpha, beta, gamma=0.0):
    """``Y = G^-1 W``: transform, divide by the symbol, transform back.

    This is the step "Solve G Y_n = W_n via 2D FFT (DCT)" of Algorithm 1.
    """
    N = w.shape[0]
    g = precond_symbol(N, h, bc, alpha, beta, gamma, dim=np.ndim(w))
    return inverse_transform(forward_transform(w, bc) / g, bc)


def precond_matrix(N, h, bc, alpha, beta, gamma=0.0):
    """Dense ``G`` assembled from the sparse Laplacian matrix (for pins on small grids)."""
    Lm = grid.lap5_matrix(N, h, bc).toarray()
    A = np.eye(N * N) - alpha * Lm + beta * (Lm @ Lm) - gamma * (Lm @ Lm @ Lm)
    return A @ A


def naive_dft_matrix(N):
    """F[k, j] = exp(-2 pi i k j / N), summed directly from the definition."""
    j = np.arange(N)
    return np.exp(-2j * np.pi * np.outer(j, j) / N)


def naive_dct2_matrix(N):
    """Orthonormal DCT-II matrix C[k, j] = c_k cos(pi k (2j+1) / (2N)),
    c_0 = sqrt(1/N), c_k = sqrt(2/N) otherwise."""
    j = np.arange(N)
    C = np.cos(np.pi * np.outer(j, 2 * j + 1) / (2 * N))
    C[0, :] *= np.sqrt(1.0 / N)
    C[1:, :] *= np.sqrt(2.0 / N)
    return C
