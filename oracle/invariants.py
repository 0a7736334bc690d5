"""Invariants of the exact step that pin the oracle (FP64, test only).

* Allen-Cahn discrete energy, the grid version of eq. (27):
      E_h(U) = h^2 sum [ lambda/2 |grad_h U|^2 + b W(U) ],  W(u) = (u^2 - 1)^2 / 4,
  with |grad_h U|^2 from forward differences across every cell face of the grid
  (wrapped faces for periodic grids, interior faces only for Neumann grids, which
  is the face sum whose gradient is -Lap^N).
* Mass sum(U): conserved by the Cahn-Hilliard step, whose right-hand side is a
  Laplacian (eq. 28) and the discrete Laplacian's columns sum to zero.
"""
import numpy as np

from . import grid


def double_well(u):
    """W(u) = (u^2 - 1)^2 / 4 (eq. 26)."""
    return 0.25 * (u * u - 1.0) ** 2


def grad_sq_sum(U, bc):
    """Sum over cell faces of the squared forward difference (no 1/h^2)."""
    if bc == grid.PERIODIC:
        dx = np.roll(U, -1, axis=1) - U
        dy = np.roll(U, -1, axis=0) - U
        return float(np.sum(dx * dx) + np.sum(dy * dy))
    dx = U[:, 1:] - U[:, :-1]
    dy = U[1:, :] - U[:-1, :]
    return float(np.sum(dx * dx) + np.sum(dy * dy))


def energy(U, lam, b, h, bc):
    """E_h(U) for Allen-Cahn / Cahn-Hilliard (eq. 27 with a = lambda)."""
    return h * h * (0.5 * lam * grad_sq_sum(U, bc) / (h * h) + b * float(np.sum(double_well(U))))


def mass(U):
    return float(np.sum(U))
