"""Closed forms from the convergence analysis (FP64, test only).

Theorem 1 and its proof (Appendix A): for affine ``F(U) = A U - b`` with ``A``
symmetric, the linearized PDHG map (omega = 1 in the notation of eq. 19) is
``X_{n+1} - X_* = M (X_n - X_*)`` with

    M ~ diag over eigenvalues lambda_k of  D_k = [[1 - 2 t_k, -tau_u lambda_k],
                                                   [tau_p lambda_k, 1        ]],
    t_k = tau_u tau_p lambda_k^2,

whose spectral radius is phi(t_k) with

    phi(t) = sqrt(1 - t)            for 0 < t <= 1,
    phi(t) = t - 1 + sqrt(t^2 - t)  for t > 1.

The iteration converges iff every t_k < 4/3 (phi(4/3) = 1).  Corollary 1 carries
this over to the G-prox dynamic with lambda_k the eigenvalues of A^T G^-1 A.

Remark 2 gives the optimal eta_* (the value of tau_u tau_p lambda_max^2 that
minimises the rate) and the optimal rate gamma_* in closed form as functions of
the condition number kappa; eta_* is also the root of eq. (equation eta) of
Appendix A, sqrt(1 - eta/kappa^2) = eta - 1 + sqrt(eta^2 - eta) on [1, 4/3).
"""
import numpy as np
from scipy.optimize import brentq


def phi(t):
    """Spectral radius of D_k as a function of t = tau_u tau_p lambda_k^2 (Appendix A)."""
    t = np.asarray(t, dtype=np.float64)
    small = np.sqrt(np.clip(1.0 - t, 0.0, None))
    large = t - 1.0 + np.sqrt(np.clip(t * t - t, 0.0, None))
    return np.where(t <= 1.0, small, large)


def iteration_block(lam, tau_u, tau_p):
    """The 2x2 block D_k of the proof of Theorem 1 for one eigenvalue lambda."""
    return np.array([[1.0 - 2.0 * tau_u * tau_p * lam * lam, -tau_u * lam],
                     [tau_p * lam, 1.0]])


def spectral_radius(eigs, tau_u, tau_p):
    """rho(M) = max_k phi(tau_u tau_p lambda_k^2)."""
    eigs = np.asarray(eigs, dtype=np.float64)
    return float(np.max(phi(tau_u * tau_p * eigs * eigs)))


def _remark2_denominator(kappa):
    k = float(kappa)
    return ((0.75 * k * k + 1.5 - 0.25 / (k * k))
            + (k - 1.0) / (2.0 * k) * np.sqrt((k - 1.0) * (3.0 * k + 1.0))
            * np.sqrt(0.75 * k * k + 1.5 + 2.0 * k - 0.25 / (k * k)))


def eta_star_closed(kappa):
    """eta_*(kappa) as printed in Remark 2."""
    return 2.0 * kappa * kappa / _remark2_denominator(kappa)


def gamma_star_closed(kappa):
    """gamma_*(kappa) as printed in Remark 2."""
    return float(np.sqrt(1.0 - 2.0 / _remark2_denominator(kappa)))


def eta_star_root(kappa):
    """eta_* as the root of sqrt(1 - eta/kappa^2) = eta - 1 + sqrt(eta^2 - eta) on [1, 4/3)."""
    k2 = float(kappa) ** 2

    def g(eta):
        return np.sqrt(1.0 - eta / k2) - (eta - 1.0 + np.sqrt(eta * eta - eta))

    if g(1.0) <= 0.0:
        return 1.0
    return brentq(g, 1.0, 4.0 / 3.0, xtol=1e-15, rtol=1e-15)


def gamma_from_eta(eta, kappa):
    return float(np.sqrt(1.0 - eta / float(kappa) ** 2))
