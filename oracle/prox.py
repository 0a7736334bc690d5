"""Pointwise implicit reaction step (FP64, test only).

The exact-prox PDHG of Sec. 2.1 (eq. 16) and the introduction (eq. 8) needs
``(Id + tau_u grad F^T P)^-1``, which the paper replaces by a linearisation.  What
remains pointwise-solvable is the reaction part alone: with diffusion dropped,
one backward-Euler step of the reaction ODE at every grid point,

    Allen-Cahn:    u - c - h_t b (u - u^3) = 0
                   (the proximal map argmin_u 1/2 (u - c)^2 + h_t b W(u)),
    Schnakenberg:  u - c_u - h_t kappa (a - u + u^2 v) = 0,
                   v - c_v - h_t kappa (b - u^2 v) = 0.

Sec. 2.1 ("Initial guess") allows a better starting point ``U_0`` than ``U^k``;
this map is the reaction-only predictor ``U_0 = prox(U^k)``.  It does not apply
to Cahn-Hilliard, whose reaction sits under a Laplacian, and is the identity for
the linear heat / biharmonic steps.

Allen-Cahn root: ``h_t b u^3 + (1 - h_t b) u - c`` is strictly increasing when
``h_t b < 1``, so the real root is unique; it is found by bisection on a
bracket that provably contains it, then polished with two Newton steps.
"""
import numpy as np

from . import equations as eq


def ac_cubic_root(c, ht, b):
    """Unique real root of h_t b u^3 + (1 - h_t b) u - c = 0, elementwise."""
    c = np.asarray(c, dtype=np.float64)
    alpha = ht * b
    beta = 1.0 - ht * b
    if not (beta > 0.0):
        raise ValueError("the Allen-Cahn prox needs h_t b < 1 for a unique root")

    def g(u):
        return alpha * u ** 3 + beta * u - c

    # g(R) >= beta R - |c| > 0 and g(-R) < 0 for R = |c| / beta + 1.
    R = np.abs(c) / beta + 1.0
    lo, hi = -R, R.copy()
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        pos = g(mid) > 0.0
        hi = np.where(pos, mid, hi)
        lo = np.where(pos, lo, mid)
    u = 0.5 * (lo + hi)
    for _ in range(2):
        u = u - g(u) / (3.0 * alpha * u ** 2 + beta)
    return u


def schnakenberg_point_solve(cu, cv, ht, a, b, kappa, iters=60):
    """Per-point root of the Schnakenberg reaction step.

    Eliminating v = (c_v + h_t kappa b) / (1 + h_t kappa u^2) leaves one scalar
    equation in u, solved by Newton from u = c_u with a fixed, generous count.
    """
    cu = np.asarray(cu, dtype=np.float64)
    cv = np.asarray(cv, dtype=np.float64)
    gam = ht * kappa
    B = cv + gam * b

    def phi(u):
        return u - cu - gam * (a - u + u * u * B / (1.0 + gam * u * u))

    def dphi(u):
        return 1.0 + gam - gam * B * 2.0 * u / (1.0 + gam * u * u) ** 2

    u = cu.copy()
    for _ in range(iters):
        u = u - phi(u) / dphi(u)
    v = B / (1.0 + gam * u * u)
    return u, v


def reaction_prox(prob, c, ht):
    """The pointwise predictor for the given problem (identity where none applies)."""
    k = prob.kind
    if k == eq.ALLEN_CAHN:
        return ac_cubic_root(c, ht, prob.b)
    if k == eq.SCHNAKENBERG:
        u, v = schnakenberg_point_solve(c[0], c[1], ht, prob.a, prob.sb, prob.kappa)
        return np.stack([u, v])
    return np.array(c, dtype=np.float64, copy=True)
