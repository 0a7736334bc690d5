"""Pins for the oracle's Algorithm 1: closed forms, brute force, invariants, paper numbers."""
import json
import os

import numpy as np
import pytest

from oracle import equations as eq, grid, invariants, newton, pdhg, prox, spectral, theory

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def golden(key):
    with open(GOLDEN) as f:
        return json.load(f)[key]


def problem(kind, bc, N=16, **kw):
    if kind == eq.SCHNAKENBERG:
        d = dict(diff=(1.0, 10.0), a=0.1, sb=0.9, kappa=1.0)
    elif kind in (eq.CAHN_HILLIARD, eq.BIHARMONIC):
        d = dict(diff=(4e-4,), b=1.0)
    else:
        d = dict(diff=(2.5e-3,), b=1.0)
    d.update(kw)
    return eq.Problem(kind=kind, N=N, bc=bc, **d)


def rand_field(prob, seed, lo=-0.9, hi=0.9):
    rng = np.random.default_rng(seed)
    if prob.ncomp == 2:
        return np.stack([1.0 + rng.uniform(-0.01, 0.01, (prob.N, prob.N)),
                         0.9 + rng.uniform(-0.01, 0.01, (prob.N, prob.N))])
    return rng.uniform(lo, hi, (prob.N, prob.N))


# ---------------------------------------------------------------- structure
@pytest.mark.parametrize("kind", [eq.HEAT, eq.BIHARMONIC])
@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_linear_step_exact_in_two_iterations(kind, bc):
    """f = 0, G = A^2, tau_u = tau_p = omega = 1: U_1 = 2 U* - U_0 and U_2 = U* (derived from
    the G-prox dynamic, Sec. 2.1, with the 2x2 blocks of Appendix A at t = 1)."""
    prob = problem(kind, bc, N=16, diff=(0.02,) if kind == eq.HEAT else (1e-5,))
    ht = 0.5
    Uk = rand_field(prob, 1)
    ustar = newton.root(prob, Uk, ht).U
    o1 = pdhg.Options(tol=0.0, max_iter=1, tau_u=1.0, tau_p=1.0, omega=1.0)
    r1 = pdhg.step(prob, Uk, ht, o1)
    np.testing.assert_allclose(r1.U, 2 * ustar - Uk, atol=1e-12)
    o2 = pdhg.Options(tol=0.0, max_iter=2, tau_u=1.0, tau_p=1.0, omega=1.0)
    r2 = pdhg.step(prob, Uk, ht, o2)
    np.testing.assert_allclose(r2.U, ustar, atol=1e-12)
    assert r2.residual < 1e-9


@pytest.mark.parametrize("kind", [eq.ALLEN_CAHN, eq.CAHN_HILLIARD, eq.SCHNAKENBERG])
def test_root_is_fixed_point(kind):
    """(U*, 0) is an equilibrium of the dynamic (Sec. 2.1)."""
    prob = problem(kind, grid.PERIODIC, N=16)
    ht = 1e-3 if kind != eq.CAHN_HILLIARD else 1e-4
    Uk = rand_field(prob, 2, -0.3, 0.3)
    ustar = newton.root(prob, Uk, ht).U
    r0 = pdhg.step(prob, Uk, ht, pdhg.Options(tol=1e-6), U0=ustar)
    assert r0.iters == 0
    r = pdhg.step(prob, Uk, ht, pdhg.Options(tol=0.0, max_iter=5), U0=ustar)
    np.testing.assert_allclose(r.U, ustar, atol=1e-12)


@pytest.mark.parametrize("kind", [eq.ALLEN_CAHN, eq.CAHN_HILLIARD, eq.SCHNAKENBERG])
@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_pdhg_reaches_newton_root(kind, bc):
    prob = problem(kind, bc, N=16)
    ht = {eq.ALLEN_CAHN: 1e-2, eq.CAHN_HILLIARD: 1e-4, eq.SCHNAKENBERG: 1e-3}[kind]
    Uk = rand_field(prob, 3)
    nr = newton.root(prob, Uk, ht)
    assert nr.fnorm < 1e-12
    tau = 0.7 if kind == eq.CAHN_HILLIARD else 0.9
    r = pdhg.step(prob, Uk, ht, pdhg.Options(tol=1e-8, tau_u=tau, tau_p=tau))
    assert r.status == pdhg.OK
    if kind == eq.ALLEN_CAHN:
        # J is an M-matrix with ||J^-1||_inf <= 1 / (1 - h_t b); ||F||_inf <= h_t ||Res||_2.
        bound = ht * r.residual / (1.0 - ht * prob.b)
    else:
        bound = 50 * ht * r.residual
    assert np.max(np.abs(r.U - nr.U)) <= bound + 1e-14


def test_newton_root_residual_is_roundoff():
    prob = problem(eq.ALLEN_CAHN, grid.PERIODIC, N=32)
    Uk = rand_field(prob, 4)
    nr = newton.root(prob, Uk, 1e-2)
    assert nr.fnorm < 1e-13


# ---------------------------------------------------------------- rates (Theorem 1, Corollary 1)
def _envelope_rate(hist, a, b, w=10):
    """Decay rate of the envelope of an oscillating sequence between the largest
    samples near iterations a and b."""
    h = np.asarray(hist)
    j1 = a - w + int(np.argmax(h[a - w:a + w]))
    j2 = b - w + int(np.argmax(h[b - w:b + w]))
    return (h[j2] / h[j1]) ** (1.0 / (j2 - j1))


def _heat_mode(N, k, l):
    j = np.arange(N)
    return np.outer(np.cos(2 * np.pi * l * j / N), np.cos(2 * np.pi * k * j / N))


@pytest.mark.parametrize("tau,modes", [(0.6, [(1, 0)]), (0.6, [(3, 2)]), (0.75, [(5, 4)]), (0.8, [(8, 8)]),
                                       (0.8, [(7, 6)]), (0.6, [(1, 0), (6, 7)]),
                                       (0.8, [(1, 1), (8, 8)])])
def test_theorem1_rate_unpreconditioned(tau, modes):
    """G = I on the heat step: started on eigenmodes of A = I - lambda h_t Lap, the residual
    decays at max over the present modes of phi(tau_u tau_p lambda_k^2) (Appendix A)."""
    N = 16
    prob = problem(eq.HEAT, grid.PERIODIC, N=N, diff=(1.0,))
    h = prob.h
    ht = 0.05 * h * h
    s = spectral.laplacian_eigenvalues_1d(N, h, grid.PERIODIC)
    Uk = sum(_heat_mode(N, k, l) for k, l in modes)
    lam_k = np.array([1.0 + ht * (s[k] + s[l]) for k, l in modes])
    rho = theory.spectral_radius(lam_k, tau, tau)
    r = pdhg.step(prob, Uk, ht, pdhg.Options(tol=0.0, max_iter=70, tau_u=tau, tau_p=tau, precond=False),
                  keep_history=True)
    # Measure late enough for the slowest present mode to dominate, and early
    # enough to stay far above the round-off floor.
    b = int(min(55, np.log(1e-9) / np.log(rho)))
    a = max(b - 25, 8)
    assert _envelope_rate(r.history, a, b, w=min(8, (b - a) // 3)) == pytest.approx(rho, rel=0.015)


def test_theorem1_divergence_above_four_thirds():
    N = 16
    prob = problem(eq.HEAT, grid.PERIODIC, N=N, diff=(1.0,))
    h = prob.h
    ht = 0.05 * h * h
    lam_max = 1.0 + ht * 8.0 / h ** 2
    tau = np.sqrt(1.2 / lam_max ** 2 * (4.0 / 3.0))  # t_max = 1.6 > 4/3
    Uk = rand_field(prob, 6)
    r = pdhg.step(prob, Uk, ht, pdhg.Options(tol=0.0, max_iter=60, tau_u=tau, tau_p=tau, precond=False),
                  keep_history=True)
    assert r.history[-1] > 10 * r.history[0]


@pytest.mark.parametrize("tau", [0.8, 1.1])
def test_corollary1_rate_with_exact_preconditioner(tau):
    """G = A^2 commutes with A, so A^T G^-1 A = I and the rate is phi(tau_u tau_p)."""
    prob = problem(eq.HEAT, grid.NEUMANN, N=16, diff=(0.05,))
    Uk = rand_field(prob, 7)
    r = pdhg.step(prob, Uk, 0.3, pdhg.Options(tol=0.0, max_iter=40, tau_u=tau, tau_p=tau), keep_history=True)
    expected = float(theory.phi(tau * tau))
    got = (r.history[32] / r.history[12]) ** (1.0 / 20)
    assert got == pytest.approx(expected, rel=0.05)


def test_phi_matches_block_eigenvalues_and_threshold():
    for lam in [0.3, 1.0, 1.7]:
        for tu, tp in [(0.5, 0.9), (0.9, 0.9), (1.0, 1.2)]:
            ev = np.linalg.eigvals(theory.iteration_block(lam, tu, tp))
            assert np.max(np.abs(ev)) == pytest.approx(float(theory.phi(tu * tp * lam * lam)), rel=1e-7, abs=1e-7)
    t43 = golden("theorem1_threshold")["value"]
    assert float(theory.phi(t43)) == pytest.approx(1.0, abs=1e-12)
    assert float(theory.phi(t43 - 1e-3)) < 1.0 < float(theory.phi(t43 + 1e-3))


@pytest.mark.parametrize("kappa", [1.0, 1.5, 3.0, 10.0, 100.0])
def test_remark2_closed_forms(kappa):
    e_closed = theory.eta_star_closed(kappa)
    e_root = theory.eta_star_root(kappa)
    assert e_closed == pytest.approx(e_root, rel=1e-9, abs=1e-12)
    assert 1.0 <= e_closed < 4.0 / 3.0
    assert theory.gamma_star_closed(kappa) == pytest.approx(theory.gamma_from_eta(e_root, kappa), abs=1e-9)
    # The optimum equalises the slowest and fastest modes of Theorem 1.
    assert float(theory.phi(e_root / kappa ** 2)) == pytest.approx(float(theory.phi(e_root)), abs=1e-9)


def test_remark2_limits():
    assert theory.eta_star_closed(1.0) == pytest.approx(1.0)
    assert theory.gamma_star_closed(1.0) == pytest.approx(0.0, abs=1e-12)
    k = 1e3
    assert theory.gamma_star_closed(k) == pytest.approx(np.sqrt(1 - 4 / (3 * k * k)), rel=1e-9)


# ---------------------------------------------------------------- closed-form steps
@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_heat_step_on_eigenmode(bc):
    N = 16
    prob = problem(eq.HEAT, bc, N=N, diff=(0.01,))
    h, ht = prob.h, 0.1
    j = np.arange(N)
    if bc == grid.PERIODIC:
        k, l = 3, 5
        mode = np.outer(np.cos(2 * np.pi * l * j / N), np.cos(2 * np.pi * k * j / N))
        mu = 4 / h ** 2 * (np.sin(np.pi * k / N) ** 2 + np.sin(np.pi * l / N) ** 2)
    else:
        k, l = 2, 7
        mode = np.outer(np.cos(np.pi * l * (2 * j + 1) / (2 * N)), np.cos(np.pi * k * (2 * j + 1) / (2 * N)))
        mu = 4 / h ** 2 * (np.sin(np.pi * k / (2 * N)) ** 2 + np.sin(np.pi * l / (2 * N)) ** 2)
    r = pdhg.step(prob, mode, ht, pdhg.Options(tol=1e-12))
    np.testing.assert_allclose(r.U, mode / (1.0 + 0.01 * ht * mu), atol=1e-12)


def test_allen_cahn_constant_state_is_cubic_root():
    N, ht, b = 16, 0.05, 1.0
    prob = problem(eq.ALLEN_CAHN, grid.PERIODIC, N=N, b=b)
    for c in [-0.7, 0.2, 0.95]:
        r = pdhg.step(prob, np.full((N, N), c), ht, pdhg.Options(tol=1e-12))
        roots = np.roots([ht * b, 0.0, 1.0 - ht * b, -c])
        real = roots[np.abs(roots.imag) < 1e-12].real
        assert len(real) == 1
        np.testing.assert_allclose(r.U, real[0], atol=1e-13)
        np.testing.assert_allclose(prox.ac_cubic_root(c, ht, b), real[0], atol=1e-14)


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_cahn_hilliard_constant_state_unchanged(bc):
    prob = problem(eq.CAHN_HILLIARD, bc, N=16)
    r = pdhg.step(prob, np.full((16, 16), 0.3), 1e-4, pdhg.Options(tol=1e-8, tau_u=0.7, tau_p=0.7))
    np.testing.assert_allclose(r.U, 0.3, atol=1e-14)


def test_schnakenberg_steady_state_needs_no_iteration():
    prob = problem(eq.SCHNAKENBERG, grid.PERIODIC, N=16)
    a, b = prob.a, prob.sb
    U = np.stack([np.full((16, 16), a + b), np.full((16, 16), b / (a + b) ** 2)])
    r = pdhg.step(prob, U, 1e-3, pdhg.Options(tol=1e-9))
    assert r.iters == 0


def test_prox_schnakenberg_solves_pointwise_system():
    rng = np.random.default_rng(8)
    cu = 1.0 + rng.uniform(-0.2, 0.2, 50)
    cv = 0.9 + rng.uniform(-0.2, 0.2, 50)
    ht, a, b, kap = 1e-2, 0.1, 0.9, 1.0
    u, v = prox.schnakenberg_point_solve(cu, cv, ht, a, b, kap)
    np.testing.assert_allclose(u - cu - ht * kap * (a - u + u * u * v), 0.0, atol=1e-14)
    np.testing.assert_allclose(v - cv - ht * kap * (b - u * u * v), 0.0, atol=1e-14)


def test_prox_predictor_does_not_change_the_root():
    prob = problem(eq.ALLEN_CAHN, grid.PERIODIC, N=16)
    Uk = rand_field(prob, 9)
    a = pdhg.step(prob, Uk, 1e-2, pdhg.Options(tol=1e-11, init="prev"))
    b = pdhg.step(prob, Uk, 1e-2, pdhg.Options(tol=1e-11, init="prox"))
    np.testing.assert_allclose(a.U, b.U, atol=1e-12)


# ---------------------------------------------------------------- invariants
def test_allen_cahn_maximum_principle_and_energy_decay():
    N = 32
    prob = problem(eq.ALLEN_CAHN, grid.PERIODIC, N=N)
    ht, lam, b = 1e-2, prob.lam, prob.b
    U = rand_field(prob, 10, -1.0, 1.0)
    for _ in range(3):
        r = pdhg.step(prob, U, ht, pdhg.Options(tol=1e-11))
        assert np.max(np.abs(r.U)) <= 1.0 + 1e-12
        dU = r.U - U
        e0 = invariants.energy(U, lam, b, prob.h, prob.bc)
        e1 = invariants.energy(r.U, lam, b, prob.h, prob.bc)
        assert e1 <= e0 - prob.h ** 2 * (1.0 / ht - b / 2.0) * np.sum(dU * dU) * (1 - 1e-9) + 1e-12
        U = r.U


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_cahn_hilliard_mass_conservation(bc):
    N = 32
    prob = problem(eq.CAHN_HILLIARD, bc, N=N)
    ht = 1e-4
    U = rand_field(prob, 11, -0.05, 0.05)
    for _ in range(2):
        r = pdhg.step(prob, U, ht, pdhg.Options(tol=1e-4, tau_u=0.7, tau_p=0.7))
        drift = abs(invariants.mass(r.U) - invariants.mass(U))
        assert drift <= N * ht * r.residual + 1e-12
        U = r.U


@pytest.mark.parametrize("kind", [eq.ALLEN_CAHN, eq.CAHN_HILLIARD])
@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_odd_symmetry_bitwise(kind, bc):
    prob = problem(kind, bc, N=16)
    ht = 1e-2 if kind == eq.ALLEN_CAHN else 1e-4
    U = rand_field(prob, 12, -0.5, 0.5)
    o = pdhg.Options(tol=1e-6, tau_u=0.7, tau_p=0.7)
    a = pdhg.step(prob, U, ht, o)
    b = pdhg.step(prob, -U, ht, o)
    assert a.iters == b.iters
    assert np.array_equal(b.U, -a.U)


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_transpose_equivariance(bc):
    prob = problem(eq.ALLEN_CAHN, bc, N=16)
    U = rand_field(prob, 13)
    o = pdhg.Options(tol=1e-11)
    a = pdhg.step(prob, U, 1e-2, o)
    b = pdhg.step(prob, U.T.copy(), 1e-2, o)
    np.testing.assert_allclose(b.U, a.U.T, atol=1e-13)


# ---------------------------------------------------------------- numbers printed in the paper
def test_paper_schnakenberg_iteration_count():
    g = golden("schnakenberg_iterations")
    N = 128
    a, b = 0.1305, 0.7695
    prob = eq.Problem(kind=eq.SCHNAKENBERG, N=N, L=1.0, bc=grid.NEUMANN, diff=(0.05, 1.0), a=a, sb=b, kappa=100.0)
    x = (np.arange(N) + 0.5) * prob.h
    X, Y = np.meshgrid(x, x)
    U = np.stack([a + b + 1e-3 * np.exp(-100 * ((X - 1 / 3) ** 2 + (Y - 1 / 2) ** 2)),
                  np.full((N, N), b / (a + b) ** 2)])
    lo, hi = g["accept_range"]
    for _ in range(g["steps_checked"]):
        r = pdhg.step(prob, U, 1.0 / 5000, pdhg.Options(tol=1e-7, tau_u=0.9, tau_p=0.9))
        assert r.status == pdhg.OK and lo <= r.iters <= hi
        U = r.U


def test_paper_allen_cahn_circle_iteration_count():
    g = golden("allen_cahn_circle_iterations")
    N, L, eps = 100, 0.5, 0.01
    prob = eq.Problem(kind=eq.ALLEN_CAHN, N=N, L=L, bc=grid.PERIODIC, diff=(eps,), b=1.0 / eps)
    x = -0.25 + np.arange(N) * prob.h
    X, Y = np.meshgrid(x, x)
    U = np.where(X ** 2 + Y ** 2 < 0.2 ** 2, 1.0, -1.0)
    for _ in range(g["steps_checked"]):
        r = pdhg.step(prob, U, 1e-3, pdhg.Options(tol=1e-7, tau_u=0.5, tau_p=0.5))
        assert r.status == pdhg.OK and r.iters < g["max_iters"]
        U = r.U


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_biharmonic_step_on_eigenmode(bc):
    """f = 0 Cahn-Hilliard-type step: U^{k+1} = mode / (1 + lambda h_t mu^2).  This fixes the
    sign of the biharmonic term (read from eq. 28, since eq. 29 prints the opposite sign)."""
    N = 16
    lam, ht = 1e-5, 0.01
    prob = problem(eq.BIHARMONIC, bc, N=N, diff=(lam,))
    s = spectral.laplacian_eigenvalues_1d(N, prob.h, bc)
    j = np.arange(N)
    k, l = 3, 2
    if bc == grid.PERIODIC:
        mode = np.outer(np.cos(2 * np.pi * l * j / N), np.cos(2 * np.pi * k * j / N))
    else:
        mode = np.outer(np.cos(np.pi * l * (2 * j + 1) / (2 * N)), np.cos(np.pi * k * (2 * j + 1) / (2 * N)))
    mu = s[k] + s[l]
    r = pdhg.step(prob, mode, ht, pdhg.Options(tol=1e-12, tau_u=0.9, tau_p=0.9))
    np.testing.assert_allclose(r.U, mode / (1.0 + lam * ht * mu * mu), atol=1e-12)
