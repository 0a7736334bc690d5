"""The nonlinear step equation ``F(U) = 0`` and its Jacobian (FP64, test only).

One implicit (backward Euler) step ``U^k -> U^{k+1}`` of a reaction-diffusion
equation is the root of ``F(U) = 0`` (Sec. 2.1, eq. 12).  The equations:

* ``allen_cahn``:  u_t = lambda Lap u + f(u),  f(u) = b (u - u^3)
  (Sec. 3.1, eq. 25 with a = lambda, W'(u) = u^3 - u).
  F(U) = U - U^k - h_t (lambda Lap U + f(U))                        (eq. 12)
* ``heat``: the same with f = 0 (Sec. 2.1, heat-equation example).
* ``cahn_hilliard``: u_t = -lambda Lap Lap u + Lap g(u),  g(u) = b (u^3 - u)
  (Sec. 3.2, eq. 28).
  F(U) = U - U^k + lambda h_t Lap Lap U - h_t Lap g(U)
  This is eq. (29) with the sign of the biharmonic term taken from the PDE
  (eq. 28); eq. (29) as printed has ``I - lambda h_t Lap Lap``, which would be
  anti-diffusive.
* ``biharmonic``: the same with g = 0.
* ``schnakenberg`` (Sec. 3.4.1, eqs. 35-36), U = (u, v):
  F_u = U - U^k - h_t (D1 Lap U + kappa (a - U + U^2 V))
  F_v = V - V^k - h_t (D2 Lap V + kappa (b - U^2 V))
* ``fch`` (Sec. 3.3, the sixth-order functionalized Cahn-Hilliard equation),
  u_t = Lap (eps^2 Lap - W2(u) + eps^2) (eps^2 Lap u - W1(u)), W = (u^2 - 1)^2 / 4,
  F(U) = U - U^k - h_t Lap (eps^2 Lap - diag W2(U) + eps^2 I)(eps^2 Lap U - W1(U)),
  with ``diff[0] = eps^2`` and W1, W2, W3 the first three derivatives of W.  The
  paper states W2(u) = 3u^2; with its W, W1(u) = u^3 - u and W2(u) = 3u^2 - 1
  (which is the value 2 at u = +-1 that the paper's preconditioner uses); this
  reading is taken.

``adjoint(U, P~)`` is ``grad F(U)^T P~``, the vector the U-update of the G-prox
PDHG dynamic subtracts (eqs. 23, 32 and the Schnakenberg update of Sec. 3.4.1).
All Laplacians are symmetric, so ``Lap^T = Lap``.
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import grid

ALLEN_CAHN = "allen_cahn"
CAHN_HILLIARD = "cahn_hilliard"
SCHNAKENBERG = "schnakenberg"
HEAT = "heat"
BIHARMONIC = "biharmonic"
FCH = "fch"
KINDS = (ALLEN_CAHN, CAHN_HILLIARD, SCHNAKENBERG, HEAT, BIHARMONIC, FCH)


@dataclass
class Problem:
    """One implicit step's equation.

    kind   : one of KINDS
    N, L   : points per side and side length of the square domain
    bc     : grid.PERIODIC or grid.NEUMANN
    diff   : lambda (scalar equations) or (D1, D2) (Schnakenberg)
    b      : reaction coefficient for Allen-Cahn / Cahn-Hilliard
    a, sb, kappa : Schnakenberg a, b, kappa
    """
    kind: str
    N: int
    L: float = 1.0
    bc: str = grid.PERIODIC
    diff: tuple = (1.0,)
    b: float = 1.0
    a: float = 0.0
    sb: float = 0.0
    kappa: float = 1.0
    dim: int = 2
    extra: dict = field(default_factory=dict)

    @property
    def h(self):
        return grid.spacing(self.N, self.L)

    @property
    def shape(self):
        """Shape of one component's field."""
        return (self.N,) * self.dim

    @property
    def ncomp(self):
        return 2 if self.kind == SCHNAKENBERG else 1

    @property
    def lam(self):
        return float(self.diff[0])


def reaction_ac(u, b):
    """Allen-Cahn reaction f(u) = -b W'(u) = b (u - u^3), W = (u^2 - 1)^2 / 4 (eq. 26)."""
    return b * (u - u * u * u)


def reaction_ac_prime(u, b):
    """f'(u) = b (1 - 3 u^2)."""
    return b * (1.0 - 3.0 * u * u)


def chem_potential_ch(u, b):
    """Cahn-Hilliard bulk term g(u) = b W'(u) = b (u^3 - u)."""
    return b * (u * u * u - u)


def chem_potential_ch_prime(u, b):
    """g'(u) = b (3 u^2 - 1)."""
    return b * (3.0 * u * u - 1.0)


def fch_w1(u):
    """W1(u) = W'(u) = u^3 - u."""
    return u * u * u - u


def fch_w2(u):
    """W2(u) = 3 u^2 - 1."""
    return 3.0 * u * u - 1.0


def fch_w3(u):
    """W3(u) = 6 u."""
    return 6.0 * u


def _check_dim(prob):
    if prob.dim == 3 and prob.kind not in (ALLEN_CAHN, HEAT, SCHNAKENBERG):
        raise ValueError("3-D grids: 7-point Laplacian equations only (Allen-Cahn, heat, Schnakenberg)")


def F(prob, U, Uk, ht):
    """The step residual F(U); shape prob.shape, or (2,) + prob.shape for Schnakenberg.
    On 3-D grids the 5-point Laplacian is replaced by the 7-point one."""
    _check_dim(prob)
    h, bc, k = prob.h, prob.bc, prob.kind
    if k == ALLEN_CAHN:
        return U - Uk - ht * (prob.lam * grid.lap(U, h, bc) + reaction_ac(U, prob.b))
    if k == HEAT:
        return U - Uk - ht * prob.lam * grid.lap(U, h, bc)
    if k == CAHN_HILLIARD:
        return (U - Uk + prob.lam * ht * grid.lap13(U, h, bc)
                - ht * grid.lap5(chem_potential_ch(U, prob.b), h, bc))
    if k == BIHARMONIC:
        return U - Uk + prob.lam * ht * grid.lap13(U, h, bc)
    if k == FCH:
        e2 = prob.lam
        mu = e2 * grid.lap5(U, h, bc) - fch_w1(U)
        nu = e2 * grid.lap5(mu, h, bc) - fch_w2(U) * mu + e2 * mu
        return U - Uk - ht * grid.lap5(nu, h, bc)
    if k == SCHNAKENBERG:
        u, v = U[0], U[1]
        d1, d2 = prob.diff
        u2v = u * u * v
        fu = u - Uk[0] - ht * (d1 * grid.lap(u, h, bc) + prob.kappa * (prob.a - u + u2v))
        fv = v - Uk[1] - ht * (d2 * grid.lap(v, h, bc) + prob.kappa * (prob.sb - u2v))
        return np.stack([fu, fv])
    raise ValueError(k)


def adjoint(prob, U, Pt, ht):
    """grad F(U)^T P~, with the reaction derivative at the given (old) U."""
    _check_dim(prob)
    h, bc, k = prob.h, prob.bc, prob.kind
    if k == ALLEN_CAHN:
        return Pt - prob.lam * ht * grid.lap(Pt, h, bc) - ht * reaction_ac_prime(U, prob.b) * Pt
    if k == HEAT:
        return Pt - prob.lam * ht * grid.lap(Pt, h, bc)
    if k == CAHN_HILLIARD:
        return (Pt + prob.lam * ht * grid.lap13(Pt, h, bc)
                - ht * chem_potential_ch_prime(U, prob.b) * grid.lap5(Pt, h, bc))
    if k == BIHARMONIC:
        return Pt + prob.lam * ht * grid.lap13(Pt, h, bc)
    if k == FCH:
        # grad F^T = I - h_t [(eps^2 Lap - D)(eps^2 Lap - D + eps^2) - diag(W3(U) B)] Lap,
        # D = diag W2(U), B = eps^2 Lap U - W1(U)
        e2 = prob.lam
        D = fch_w2(U)
        B = e2 * grid.lap5(U, h, bc) - fch_w1(U)
        q = grid.lap5(Pt, h, bc)
        a = e2 * grid.lap5(q, h, bc) - D * q + e2 * q
        return Pt - ht * (e2 * grid.lap5(a, h, bc) - D * a) + ht * fch_w3(U) * B * q
    if k == SCHNAKENBERG:
        u, v = U[0], U[1]
        p, q = Pt[0], Pt[1]
        d1, d2 = prob.diff
        kap = prob.kappa
        gu = p - ht * (d1 * grid.lap(p, h, bc) + kap * (-p + 2.0 * u * v * (p - q)))
        gv = q - ht * (d2 * grid.lap(q, h, bc) + kap * u * u * (p - q))
        return np.stack([gu, gv])
    raise ValueError(k)


def precond_coeffs(prob, ht):
    """Per-component (alpha, beta, gamma) of G = (I - alpha Lap + beta Lap^2 - gamma Lap^3)^2.

    Allen-Cahn / heat: G = (I - lambda h_t Lap)^2 (Sec. 2.1).
    Cahn-Hilliard / biharmonic: G = (I + lambda h_t Lap Lap)^2 (Sec. 3.2, sign as in F).
    Schnakenberg: G_u = (I - h_t D1 Lap)^2, G_v = (I - h_t D2 Lap)^2 (Sec. 3.4.1).
    FCH: G = (I - h_t eps^2 Lap (eps^2 Lap - (2 - eps^2) I) Lap)^2 (Sec. 3.3: W2 replaced
    by its value 2 at the wells), i.e. beta = h_t eps^2 (2 - eps^2), gamma = h_t eps^4.
    """
    k = prob.kind
    if k in (ALLEN_CAHN, HEAT):
        return [(prob.lam * ht, 0.0, 0.0)]
    if k in (CAHN_HILLIARD, BIHARMONIC):
        return [(0.0, prob.lam * ht, 0.0)]
    if k == FCH:
        e2 = prob.lam
        return [(0.0, ht * e2 * (2.0 - e2), ht * e2 * e2)]
    if k == SCHNAKENBERG:
        return [(prob.diff[0] * ht, 0.0, 0.0), (prob.diff[1] * ht, 0.0, 0.0)]
    raise ValueError(k)


def residual_norm(prob, W, ht):
    """The stopping quantity of Sec. 2.1: ||Res(U)||_2 with Res = F(U) / h_t.

    Plain (unweighted) Euclidean norm over grid points.  For the two-component
    system the norms of the components are added (Sec. 3.4.1).
    """
    if prob.ncomp == 1:
        return float(np.sqrt(np.sum((W / ht) ** 2)))
    return float(sum(np.sqrt(np.sum((W[c] / ht) ** 2)) for c in range(prob.ncomp)))


def jacobian(prob, U, ht):
    """Sparse Jacobian of F at U, assembled from the sparse Laplacian matrix."""
    _check_dim(prob)
    N, h, bc, k = prob.N, prob.h, prob.bc, prob.kind
    Lm = grid.lap5_matrix(N, h, bc) if prob.dim == 2 else grid.lap7_matrix(N, h, bc)
    I = sp.identity(N ** prob.dim, format="csr")
    if k == ALLEN_CAHN:
        return (I - ht * prob.lam * Lm - ht * sp.diags(reaction_ac_prime(U, prob.b).ravel())).tocsr()
    if k == HEAT:
        return (I - ht * prob.lam * Lm).tocsr()
    if k == CAHN_HILLIARD:
        return (I + prob.lam * ht * (Lm @ Lm)
                - ht * (Lm @ sp.diags(chem_potential_ch_prime(U, prob.b).ravel()))).tocsr()
    if k == BIHARMONIC:
        return (I + prob.lam * ht * (Lm @ Lm)).tocsr()
    if k == FCH:
        e2 = prob.lam
        u = U.ravel()
        D = sp.diags(fch_w2(u))
        B = e2 * (Lm @ u) - fch_w1(u)
        A = e2 * Lm - D + e2 * I
        return (I - ht * (Lm @ (A @ (e2 * Lm - D) - sp.diags(fch_w3(u) * B)))).tocsr()
    if k == SCHNAKENBERG:
        u, v = U[0].ravel(), U[1].ravel()
        d1, d2 = prob.diff
        kap = prob.kappa
        juu = I - ht * (d1 * Lm + kap * (-I + sp.diags(2.0 * u * v)))
        juv = -ht * kap * sp.diags(u * u)
        jvu = ht * kap * sp.diags(2.0 * u * v)
        jvv = I - ht * (d2 * Lm - kap * sp.diags(u * u))
        return sp.bmat([[juu, juv], [jvu, jvv]], format="csr")
    raise ValueError(k)
