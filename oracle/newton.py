"""The plain definition of a step's result: the root of F(U) = 0 (FP64, test only).

The paper defines ``U^{k+1}`` as the solution of the implicit scheme (Sec. 2.1,
eq. 11) and notes that Newton's method is the usual way to get it (Sec. 1).
This module computes that root directly: damped Newton from ``U^k`` with a
sparse direct solve of the Jacobian system and Armijo backtracking on ||F||_2,
iterated until ||F||_2 stops decreasing (round-off level).  It is independent of
the PDHG iteration and of the FFT/DCT preconditioner.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from . import equations as eq


@dataclass
class NewtonResult:
    U: np.ndarray
    iters: int
    fnorm: float


def _norm(W):
    return float(np.sqrt(np.sum(W * W)))


def root(prob, Uk, ht, U0=None, max_iter=100):
    Uk = np.asarray(Uk, dtype=np.float64)
    U = np.array(Uk if U0 is None else U0, dtype=np.float64, copy=True)
    Fu = eq.F(prob, U, Uk, ht)
    fn = _norm(Fu)
    it = 0
    while it < max_iter and fn > 0.0:
        J = eq.jacobian(prob, U, ht)
        d = spla.spsolve(J.tocsc(), -Fu.reshape(-1)).reshape(U.shape)
        t = 1.0
        while True:
            Un = U + t * d
            Fn = eq.F(prob, Un, Uk, ht)
            fnn = _norm(Fn)
            if fnn <= (1.0 - 1e-4 * t) * fn or t < 1e-8:
                break
            t *= 0.5
        it += 1
        if not fnn < fn:
            # No decrease along the Newton direction: round-off floor reached.
            break
        U, Fu, fn = Un, Fn, fnn
    return NewtonResult(U=U, iters=it, fnorm=fn)
