"""Pins of the reaction terms' signs and of the FCH operator, from the PDEs themselves.

Round-off-level self-consistency (finite-difference Jacobians, PDHG root = Newton
root, mass conservation) holds for an operator whose reaction sign is flipped
consistently, so these pins come from outside the oracle:

* Linear amplification.  About a constant state ``c`` the step of a small
  eigenmode ``e`` of the discrete Laplacian (``Lap e = -mu e``) is fixed by the
  linearised PDE: ``U^{k+1} = c' + eta e + O(delta^2)`` with
  ``eta = delta / (1 - h_t sigma(mu))`` and ``sigma`` the PDE's growth rate of
  that mode (backward Euler).  The rates, derived by hand from the equations:

  - Allen-Cahn (Sec. 3.1, eq. 25), u_t = lambda Lap u + b (u - u^3):
    ``sigma = -lambda mu + b (1 - 3 c'^2)`` about the new constant c'.
  - Cahn-Hilliard (Sec. 3.2, the CH equation), u_t = -a Lap Lap u + b Lap W'(u):
    ``sigma = -lambda mu^2 - mu b (3 c^2 - 1)``; for ``c = 0`` long waves grow
    (spinodal decomposition), which is what fixes the sign of the reaction.
  - FCH (Sec. 3.3, the sixth-order equation),
    u_t = Lap (eps^2 Lap - W''(u) + eps^2)(eps^2 Lap u - W'(u)):
    ``sigma = -mu [(eps^2 mu + W''(c))(eps^2 mu + W''(c) - eps^2) + W'''(c) W'(c)]``.
  - Schnakenberg (Sec. 3.4.1) about its steady state: the 2 x 2 linearisation
    of the kinetics plus ``-D_i mu`` on the diagonal.

* Energy decay.  Cahn-Hilliard is the H^-1 gradient flow of the energy of
  eq. (27) (Sec. 3.2); the FCH equation is the H^-1 flow of
  ``E(u) = int 1/2 (eps^2 Lap u - W'(u))^2 - eps^2 (eps^2/2 |grad u|^2 + W(u))``
  (its variational derivative is ``(eps^2 Lap - W'' + eps^2)(eps^2 Lap u - W')``).
  The discrete energies decay along the oracle's steps.

Each linear-mode pin is also run on a copy of the oracle's equation module with
the sign planted wrong (in memory, on the CPU) and must then fail.
"""
import os
import types

import numpy as np
import pytest

import oracle
from oracle import equations as eq, grid, invariants, newton

EQ_SOURCE = os.path.join(os.path.dirname(oracle.__file__), "equations.py")


def mode(N, bc, k, l):
    """Eigenmode of the discrete Laplacian: cos(2 pi (k x + l y) / N) on periodic grids,
    cos(pi k (x + 1/2) / N) cos(pi l (y + 1/2) / N) on Neumann grids (x, y grid indices)."""
    j = np.arange(N, dtype=np.float64)
    if bc == grid.PERIODIC:
        return np.cos(2 * np.pi * (k * j[None, :] + l * j[:, None]) / N)
    return np.cos(np.pi * k * (j[None, :] + 0.5) / N) * np.cos(np.pi * l * (j[:, None] + 0.5) / N)


def mode_mu(N, h, bc, k, l):
    """-Lap e = mu e: mu = s_k + s_l, s_k = (4/h^2) sin^2(pi k / N) (periodic) or
    (4/h^2) sin^2(pi k / (2N)) (Neumann)."""
    d = N if bc == grid.PERIODIC else 2 * N
    s = lambda m: 4.0 / h ** 2 * np.sin(np.pi * m / d) ** 2
    return s(k) + s(l)


def project(U, e):
    return float(np.sum(U * e) / np.sum(e * e))


def step_root(prob, Uk, ht):
    r = newton.root(prob, Uk, ht)
    return r.U


def mutated_equations(replacements):
    """A copy of the oracle's equation module with source replacements applied (each must
    match), for planting a wrong sign in memory."""
    src = open(EQ_SOURCE).read()
    for old, new in replacements:
        assert src.count(old) >= 1, old
        src = src.replace(old, new)
    mod = types.ModuleType("oracle._mutated_equations")
    mod.__package__ = "oracle"
    mod.__file__ = EQ_SOURCE
    exec(compile(src, EQ_SOURCE, "exec"), mod.__dict__)
    return mod


# ---------------------------------------------------------------- closed-form gains
def ch_gain(lam, b, c, mu, ht):
    sigma = -lam * mu * mu - mu * b * (3 * c * c - 1)
    return 1.0 / (1.0 - ht * sigma)


def fch_gain(e2, c, mu, ht):
    w1, w2, w3 = c ** 3 - c, 3 * c * c - 1, 6 * c
    sigma = -mu * ((e2 * mu + w2) * (e2 * mu + w2 - e2) + w3 * w1)
    return 1.0 / (1.0 - ht * sigma)


def ac_new_constant(c, b, ht):
    """The real root of h_t b u^3 + (1 - h_t b) u - c = 0 (unique for h_t b < 1)."""
    r = np.roots([ht * b, 0.0, 1.0 - ht * b, -c])
    return float(np.real(r[np.argmin(np.abs(np.imag(r)))]))


def ac_gain(lam, b, c_new, mu, ht):
    sigma = -lam * mu + b * (1 - 3 * c_new * c_new)
    return 1.0 / (1.0 - ht * sigma)


# ---------------------------------------------------------------- measured gains
def measured_gain(prob, c, k, l, ht, delta, c_new=None):
    e = mode(prob.N, prob.bc, k, l)
    U = step_root(prob, c + delta * e, ht)
    base = c if c_new is None else c_new
    return project(U - base, e) / delta, U


CH_CASES = [  # (bc, c, k, l): long waves about c = 0 grow, short ones decay
    (grid.PERIODIC, 0.0, 1, 0), (grid.PERIODIC, 0.0, 2, 1), (grid.PERIODIC, 0.0, 5, 3),
    (grid.PERIODIC, 0.4, 1, 1), (grid.NEUMANN, 0.0, 1, 0), (grid.NEUMANN, -0.3, 3, 2), (grid.NEUMANN, 0.8, 6, 1),
]


def ch_problem(bc, N=16):
    """C3's parameters (lambda = eps^2 = 4e-4, b = 1) on the unit square."""
    return eq.Problem(kind=eq.CAHN_HILLIARD, N=N, bc=bc, diff=(4e-4,), b=1.0)


def ch_gain_error(bc, c, k, l, ht=1e-3, delta=1e-5, N=16):
    prob = ch_problem(bc, N)
    mu = mode_mu(prob.N, prob.h, bc, k, l)
    got, U = measured_gain(prob, c, k, l, ht, delta)
    want = ch_gain(prob.lam, prob.b, c, mu, ht)
    return abs(got - want) / abs(want), got, want, U


@pytest.mark.parametrize("bc,c,k,l", CH_CASES)
def test_cahn_hilliard_eigenmode_gain(bc, c, k, l):
    err, got, want, U = ch_gain_error(bc, c, k, l)
    assert err <= 1e-7, (got, want)
    # the mean is the conserved mass
    assert abs(U.mean() - c) <= 1e-14


def test_cahn_hilliard_spinodal_modes_grow():
    """About c = 0 the longest wave grows and the shortest decays (the gains bracket 1): on
    a 32^2 grid the shortest wave's mu = 8192 lies beyond the spinodal band mu < b / lambda."""
    _, g_long, _, _ = ch_gain_error(grid.PERIODIC, 0.0, 1, 0, N=32)
    _, g_short, _, _ = ch_gain_error(grid.PERIODIC, 0.0, 16, 16, N=32)
    assert g_long > 1.0 > g_short


def test_cahn_hilliard_flipped_reaction_fails_the_pin(monkeypatch):
    """An oracle with g -> -g (anti-diffusive spinodal term) fails the gain pin."""
    monkeypatch.setattr(newton, "eq", mutated_equations([
        ("return b * (u * u * u - u)", "return -b * (u * u * u - u)"),
        ("return b * (3.0 * u * u - 1.0)", "return -b * (3.0 * u * u - 1.0)"),
    ]))
    errs = [ch_gain_error(bc, c, k, l)[0] for bc, c, k, l in CH_CASES]
    assert max(errs) > 1e-3


FCH_CASES = [(grid.PERIODIC, 0.0, 1, 0), (grid.PERIODIC, 0.3, 2, 1), (grid.PERIODIC, -0.95, 3, 0),
             (grid.PERIODIC, 0.5, 6, 5), (grid.NEUMANN, 0.3, 1, 1), (grid.NEUMANN, 1.0, 4, 2),
             (grid.NEUMANN, -0.6, 9, 7)]


def fch_problem(bc, N=32):
    """The paper's FCH example (eps = 0.18 on [0, 2 pi]^2) on a 32^2 grid."""
    return eq.Problem(kind=eq.FCH, N=N, L=2 * np.pi, bc=bc, diff=(0.18 ** 2,))


def fch_gain_error(bc, c, k, l, ht=1e-2, delta=1e-5):
    prob = fch_problem(bc)
    mu = mode_mu(prob.N, prob.h, bc, k, l)
    got, U = measured_gain(prob, c, k, l, ht, delta)
    want = fch_gain(prob.lam, c, mu, ht)
    return abs(got - want) / abs(want), got, want, U


@pytest.mark.parametrize("bc,c,k,l", FCH_CASES)
def test_fch_eigenmode_gain(bc, c, k, l):
    err, got, want, U = fch_gain_error(bc, c, k, l)
    assert err <= 1e-8, (got, want)
    assert abs(U.mean() - c) <= 1e-13


FCH_FLIPS = {
    "+eps^2 -> -eps^2": [("nu = e2 * grid.lap5(mu, h, bc) - fch_w2(U) * mu + e2 * mu",
                          "nu = e2 * grid.lap5(mu, h, bc) - fch_w2(U) * mu - e2 * mu"),
                         ("A = e2 * Lm - D + e2 * I", "A = e2 * Lm - D - e2 * I")],
    "-W'' -> +W''": [("nu = e2 * grid.lap5(mu, h, bc) - fch_w2(U) * mu + e2 * mu",
                      "nu = e2 * grid.lap5(mu, h, bc) + fch_w2(U) * mu + e2 * mu"),
                     ("A = e2 * Lm - D + e2 * I", "A = e2 * Lm + D + e2 * I"),
                     ("return (I - ht * (Lm @ (A @ (e2 * Lm - D) - sp.diags(fch_w3(u) * B)))).tocsr()",
                      "return (I - ht * (Lm @ (A @ (e2 * Lm - D) + sp.diags(fch_w3(u) * B)))).tocsr()")],
    "-h_t Lap -> +h_t Lap": [("return U - Uk - ht * grid.lap5(nu, h, bc)", "return U - Uk + ht * grid.lap5(nu, h, bc)"),
                             ("return (I - ht * (Lm @ (A @ (e2 * Lm - D)", "return (I + ht * (Lm @ (A @ (e2 * Lm - D)")],
}


@pytest.mark.parametrize("flip", sorted(FCH_FLIPS))
def test_fch_planted_operator_errors_fail_the_pin(monkeypatch, flip):
    monkeypatch.setattr(newton, "eq", mutated_equations(FCH_FLIPS[flip]))
    errs = [fch_gain_error(bc, c, k, l)[0] for bc, c, k, l in FCH_CASES]
    assert max(errs) > 1e-2


@pytest.mark.parametrize("bc,c,k,l", [(grid.PERIODIC, 0.2, 1, 0), (grid.PERIODIC, -0.5, 3, 2),
                                      (grid.NEUMANN, 0.7, 2, 2)])
def test_allen_cahn_eigenmode_gain(bc, c, k, l):
    prob = eq.Problem(kind=eq.ALLEN_CAHN, N=16, bc=bc, diff=(2.5e-3,), b=1.0)
    ht, delta = 1e-2, 1e-5
    c_new = ac_new_constant(c, prob.b, ht)
    mu = mode_mu(prob.N, prob.h, bc, k, l)
    got, U = measured_gain(prob, c, k, l, ht, delta, c_new=c_new)
    want = ac_gain(prob.lam, prob.b, c_new, mu, ht)
    assert abs(got - want) <= 1e-7 * abs(want), (got, want)


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_schnakenberg_eigenmode_response(bc):
    """About the steady state (u*, v*) = (a + b, b / (a + b)^2) a pair of small mode
    amplitudes (du, dv) is mapped by the inverse of the linearised backward-Euler matrix
    [[1 + h_t (D1 mu + kappa (1 - 2 u* v*)), -h_t kappa u*^2],
     [2 h_t kappa u* v*, 1 + h_t (D2 mu + kappa u*^2)]]."""
    a, sb, kap, d1, d2 = 0.1, 0.9, 1.0, 1.0, 10.0
    prob = eq.Problem(kind=eq.SCHNAKENBERG, N=16, bc=bc, diff=(d1, d2), a=a, sb=sb, kappa=kap)
    us, vs = a + sb, sb / (a + sb) ** 2
    ht, delta = 1e-2, 1e-5
    k, l = 1, 1
    e = mode(16, bc, k, l)
    mu = mode_mu(16, prob.h, bc, k, l)
    du, dv = delta, -0.6 * delta
    U = step_root(prob, np.stack([us + du * e, vs + dv * e]), ht)
    got = np.array([project(U[0] - us, e), project(U[1] - vs, e)])
    M = np.array([[1 + ht * (d1 * mu + kap * (1 - 2 * us * vs)), -ht * kap * us * us],
                  [2 * ht * kap * us * vs, 1 + ht * (d2 * mu + kap * us * us)]])
    want = np.linalg.solve(M, [du, dv])
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-6 * delta)


# ---------------------------------------------------------------- energy decay
def fch_energy(U, e2, h, bc):
    """h^2 [ sum 1/2 mu^2 - eps^2 (eps^2/2 |grad_h U|^2 + W(U)) ], mu = eps^2 Lap U - W'(U),
    |grad_h U|^2 from forward differences across the grid's cell faces."""
    mu = e2 * grid.lap5(U, h, bc) - (U ** 3 - U)
    grad = invariants.grad_sq_sum(U, bc) / (h * h)
    return h * h * (0.5 * float(np.sum(mu * mu)) - e2 * (0.5 * e2 * grad + float(np.sum(invariants.double_well(U)))))


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_cahn_hilliard_energy_decays(bc):
    """Backward Euler for the H^-1 flow decays the energy of eq. (27) (a = lambda, b):
    C3's parameters (lambda = 4e-4, b = 1, h_t = 1e-4 <= 8 lambda / b^2) on a 32^2 grid,
    noise about 0, ten steps; the mass is unchanged."""
    prob = eq.Problem(kind=eq.CAHN_HILLIARD, N=32, bc=bc, diff=(4e-4,), b=1.0)
    U = np.random.default_rng(7).uniform(-0.05, 0.05, (32, 32))
    ht = 1e-4
    E = [invariants.energy(U, prob.lam, prob.b, prob.h, bc)]
    m0 = U.sum()
    for _ in range(10):
        U = step_root(prob, U, ht)
        E.append(invariants.energy(U, prob.lam, prob.b, prob.h, bc))
        assert abs(U.sum() - m0) <= 1e-11
    assert all(E[i + 1] < E[i] for i in range(10)), E


@pytest.mark.parametrize("bc", [grid.PERIODIC, grid.NEUMANN])
def test_fch_energy_decays(bc):
    """The FCH energy decays along steps of the paper's example (eps = 0.18 on [0, 2 pi]^2,
    h_t = 1e-3, the initial state of Sec. 3.3) on a 32^2 grid."""
    prob = fch_problem(bc, N=32)
    x = np.arange(32) * prob.h
    X, Y = np.meshgrid(x, x)
    U = 2 * np.exp(np.sin(X) + np.sin(Y) - 2) + 2.2 * np.exp(-np.sin(X) - np.sin(Y) - 2) - 1
    E = [fch_energy(U, prob.lam, prob.h, bc)]
    for _ in range(8):
        U = step_root(prob, U, 1e-3)
        E.append(fch_energy(U, prob.lam, prob.h, bc))
    assert all(E[i + 1] < E[i] for i in range(8)), E
