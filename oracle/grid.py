"""Discrete Laplacians on an N x N (or N x N x N) grid, FP64 (test infrastructure only).

Fields are numpy arrays of shape (N, N) indexed ``[y, x]`` (x fastest), or
(N, N, N) indexed ``[z, y, x]`` for the 7-point Laplacian of 3-D grids (the
paper poses the method on a domain in R^d; its examples are 2-D).  Every
operator here is symmetric under x <-> y, so the paper's garbled vectorisation
index (Sec. 2.1, just before eq. 11) does not change any result.

Grid spacing ``h = L / N`` for both boundary conditions.  For periodic grids this
is the paper's ``h_x = L / N_x`` (Sec. 2.1).  For Neumann grids it is the
cell-centred reading of Remark 1: the ghost value ``U_{-1} = U_0`` sits half a cell
outside the first point, which puts N points on a side of length ``N h``.

Two independent constructions are provided so that each can pin the other:

* stencil functions (``lap5``, ``lap13``) acting on padded arrays, and
* sparse matrices (``lap5_matrix``) assembled from the block forms the paper
  prints: the block-circulant ``Lap^P`` of Sec. 2.1 and the ``L_1 / L_2`` block
  matrix ``Lap^N`` of Remark 1 (eq. 24).
"""
import numpy as np
import scipy.sparse as sp

PERIODIC = "periodic"
NEUMANN = "neumann"


def spacing(N, L):
    """Grid spacing h = L / N (Sec. 2.1; cell-centred reading of Remark 1)."""
    return float(L) / int(N)


def _pad(u, width, bc):
    """Extend a field by ``width`` ghost cells on every side.

    Periodic: wrap around.  Neumann: half-sample mirror, ``U_{-1-m} = U_m`` and
    ``U_{N+m} = U_{N-1-m}``; for m = 0 this is the ghost rule ``U_{-1} = U_0`` of
    Remark 1.
    """
    if bc == PERIODIC:
        return np.pad(u, width, mode="wrap")
    if bc == NEUMANN:
        return np.pad(u, width, mode="symmetric")
    raise ValueError(bc)


def lap5(u, h, bc):
    """Five-point Laplacian (central differences), Sec. 2.1 and Remark 1.

    (Lap u)[y, x] = (u[y, x-1] + u[y, x+1] + u[y-1, x] + u[y+1, x] - 4 u[y, x]) / h^2
    with ghost values from ``_pad``.
    """
    e = _pad(np.asarray(u, dtype=np.float64), 1, bc)
    c = e[1:-1, 1:-1]
    return (e[1:-1, :-2] + e[1:-1, 2:] + e[:-2, 1:-1] + e[2:, 1:-1] - 4.0 * c) / (h * h)


def lap13(u, h, bc):
    """Thirteen-point biharmonic stencil, the ``Lap Lap`` of eq. (29).

    Coefficients over h^4: centre 20; the four axis neighbours -8; the four
    diagonal neighbours 2; the four axis points at distance two 1.  With the
    half-sample mirror ghosts this equals ``lap5(lap5(u))`` exactly for both
    boundary conditions (a test checks this).
    """
    e = _pad(np.asarray(u, dtype=np.float64), 2, bc)
    n = u.shape[0]

    def at(dy, dx):
        return e[2 + dy:2 + dy + n, 2 + dx:2 + dx + n]

    axis1 = at(0, -1) + at(0, 1) + at(-1, 0) + at(1, 0)
    diag = at(-1, -1) + at(-1, 1) + at(1, -1) + at(1, 1)
    axis2 = at(0, -2) + at(0, 2) + at(-2, 0) + at(2, 0)
    h4 = h ** 4
    return (20.0 * at(0, 0) - 8.0 * axis1 + 2.0 * diag + axis2) / h4


def lap7(u, h, bc):
    """Seven-point Laplacian of a 3-D field: the 1-D second difference along each of
    the three axes, with the same ghost rules as ``lap5``."""
    e = _pad(np.asarray(u, dtype=np.float64), 1, bc)
    c = e[1:-1, 1:-1, 1:-1]
    return (e[1:-1, 1:-1, :-2] + e[1:-1, 1:-1, 2:] + e[1:-1, :-2, 1:-1] + e[1:-1, 2:, 1:-1]
            + e[:-2, 1:-1, 1:-1] + e[2:, 1:-1, 1:-1] - 6.0 * c) / (h * h)


def lap(u, h, bc):
    """The Laplacian of a 2-D (5-point) or 3-D (7-point) field."""
    return lap5(u, h, bc) if np.ndim(u) == 2 else lap7(u, h, bc)


def _second_difference_1d(N, bc):
    """The N x N tridiagonal 1-D second difference (without 1/h^2).

    Periodic: circulant with -2 on the diagonal and 1 on both wrapped
    off-diagonals.  Neumann: -1 in the two corner diagonal entries (the ghost
    ``U_{-1} = U_0`` folds into the diagonal), -2 elsewhere.
    """
    main = -2.0 * np.ones(N)
    off = np.ones(N - 1)
    T = sp.diags([off, main, off], [-1, 0, 1], format="lil")
    if bc == PERIODIC:
        T[0, N - 1] = 1.0
        T[N - 1, 0] = 1.0
    elif bc == NEUMANN:
        T[0, 0] = -1.0
        T[N - 1, N - 1] = -1.0
    else:
        raise ValueError(bc)
    return T.tocsr()


def lap5_matrix(N, h, bc):
    """Sparse N^2 x N^2 Laplacian assembled from the paper's block forms.

    Periodic: the block-circulant ``Lap^P`` of Sec. 2.1, diagonal blocks ``L``
    (tridiagonal circulant with -4 on the diagonal) and identity off-diagonal
    blocks, wrapped.  Neumann: ``Lap^N`` of Remark 1 (eq. 24), diagonal blocks
    ``L_1`` (first and last) and ``L_2`` with identity couplings.

    Both are ``kron(I, T) + kron(T, I)`` for the 1-D second difference ``T``;
    the Neumann corner entries reproduce the -2/-3 and -3/-4 diagonals of
    ``L_1`` / ``L_2``.  Row index = y * N + x.
    """
    T = _second_difference_1d(N, bc)
    I = sp.identity(N, format="csr")
    return ((sp.kron(I, T) + sp.kron(T, I)) / (h * h)).tocsr()


def lap7_matrix(N, h, bc):
    """Sparse N^3 x N^3 seven-point Laplacian, kron(I, I, T) + kron(I, T, I) + kron(T, I, I);
    row index = (z * N + y) * N + x."""
    T = _second_difference_1d(N, bc)
    I = sp.identity(N, format="csr")
    return ((sp.kron(I, sp.kron(I, T)) + sp.kron(I, sp.kron(T, I)) + sp.kron(T, sp.kron(I, I))) / (h * h)).tocsr()


def apply_matrix(M, u):
    """Apply an N^2 x N^2 matrix to an (N, N) field."""
    n = u.shape[0]
    return (M @ u.reshape(-1)).reshape(n, n)
