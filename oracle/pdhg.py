"""Algorithm 1: one implicit step by the G-prox linearized PDHG dynamic (FP64, test only).

For ``F`` from ``equations`` the iteration is (Sec. 2.1, eqs. 21-23; Sec. 3.2,
eqs. 30-32; Sec. 3.4.1 for the system):

    P_{n+1} = P_n + tau_p G^-1 F(U_n)
    P~      = P_{n+1} + omega (P_{n+1} - P_n)
    U_{n+1} = U_n - tau_u grad F(U_n)^T P~

started from U_0 = U^k (or the reaction predictor, Sec. 2.1 "Initial guess")
and P_0 = 0, and stopped as soon as ||Res(U_n)||_2 <= delta with
Res = F(U_n) / h_t (Sec. 2.1, "Stopping criterion").  The test is made before
every iteration, so a step whose start already satisfies it takes 0 iterations.

Readings of the paper taken here:
* omega = 1 is used throughout the experiments (Sec. 3); the proof of Theorem 1
  (Appendix A) also corresponds to omega = 1 in this notation.
* "while ||Res|| >= delta" (Algorithm 1) and "terminate iff ||Res|| <= delta"
  (Sec. 2.1) differ only at equality; the stop is taken at <= delta.
* ``precond=False`` replaces G by the identity (the plain linearized PDHG of
  eq. 17); it exists for the Theorem 1 rate check.
* A guard not in the paper: the step is declared non-finite when the residual is
  NaN/Inf or has grown beyond 1e8 times its initial value.
"""
from dataclasses import dataclass, field

import numpy as np

from . import equations as eq
from . import prox, spectral

OK = "ok"
NOCONV = "noconv"
NONFINITE = "nonfinite"
DIVERGENCE_FACTOR = 1e8


@dataclass
class Options:
    tol: float = 1e-10
    max_iter: int = 10000
    tau_u: float = 0.9
    tau_p: float = 0.9
    omega: float = 1.0
    init: str = "prev"          # "prev": U_0 = U^k;  "prox": U_0 = reaction_prox(U^k)
    precond: bool = True


@dataclass
class StepResult:
    U: np.ndarray
    iters: int
    residual: float
    status: str
    history: list = field(default_factory=list)


def precond_apply(prob, W, ht, precond=True):
    """Y = G^-1 W, component by component ("Solve G Y_n = W_n", Algorithm 1)."""
    if not precond:
        return np.array(W, copy=True)
    coeffs = eq.precond_coeffs(prob, ht)
    if prob.ncomp == 1:
        return spectral.precond_solve(W, prob.h, prob.bc, *coeffs[0])
    return np.stack([spectral.precond_solve(W[c], prob.h, prob.bc, *coeffs[c])
                     for c in range(prob.ncomp)])


def initial_guess(prob, Uk, ht, init):
    if init == "prev":
        return np.array(Uk, dtype=np.float64, copy=True)
    if init == "prox":
        return prox.reaction_prox(prob, Uk, ht)
    raise ValueError(init)


def step(prob, Uk, ht, opts=None, keep_history=False, U0=None):
    """One time step U^k -> U^{k+1} (the body of the time loop of Algorithm 1).

    ``U0`` overrides the initial guess (used to check that the root is a fixed
    point of the iteration, Sec. 2.1).
    """
    opts = opts or Options()
    Uk = np.asarray(Uk, dtype=np.float64)
    if U0 is None:
        U = initial_guess(prob, Uk, ht, opts.init)
    else:
        U = np.array(U0, dtype=np.float64, copy=True)
    P = np.zeros_like(U)
    history = []
    n = 0
    res0 = None
    while True:
        W = eq.F(prob, U, Uk, ht)
        res = eq.residual_norm(prob, W, ht)
        if keep_history:
            history.append(res)
        if res0 is None:
            res0 = res
        if not np.isfinite(res) or res > DIVERGENCE_FACTOR * res0:
            status = NONFINITE
            break
        if res <= opts.tol:
            status = OK
            break
        if n >= opts.max_iter:
            status = NOCONV
            break
        Y = precond_apply(prob, W, ht, opts.precond)
        P_next = P + opts.tau_p * Y
        P_tilde = P_next + opts.omega * (P_next - P)
        U = U - opts.tau_u * eq.adjoint(prob, U, P_tilde, ht)
        P = P_next
        n += 1
    return StepResult(U=U, iters=n, residual=res, status=status, history=history)


def run(prob, U0, ht, steps, opts=None):
    """The time loop of Algorithm 1: returns the list of per-step results."""
    out = []
    U = np.asarray(U0, dtype=np.float64)
    for _ in range(steps):
        r = step(prob, U, ht, opts)
        out.append(r)
        U = r.U
    return out
