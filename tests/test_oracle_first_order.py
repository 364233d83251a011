"""Pins of the oracle's first-order convex-splitting scheme (the Eyre splitting
of Section 1: convex part of the energy at the new time level, concave part
-|grad phi|^2 at the old one) against what the mathematics fixes:

* the step written in phi alone (definition.solve_step_fo_phi, a different
  formulation from the three-field system N(u) = S the multigrid solves);
* an exact 3x3 solve of the linearised point equations;
* the linear amplification factor of a small Fourier mode (closed form);
* unconditional energy stability, F_h(phi^{k+1}) <= F_h(phi^k), at time steps
  far beyond any explicit limit;
* first order in time on smooth data (rate 1 of Cauchy differences);
* mass conservation and constant states as exact fixed points.
"""
import math

import numpy as np
import pytest

from oracle import cfas
from oracle import definition as D
from paper_1611_06288_amd import inputs


def plane_wave(n, r, s, t):
    i = np.arange(n)
    k, j, ii = np.meshgrid(i, i, i, indexing="ij")
    return np.cos(2 * np.pi * (r * ii + s * j + t * k) / n)


@pytest.mark.parametrize("n,tau,cycle", [(8, 0.5, "V"), (12, 0.3, "F"), (8, 5.0, "F")])
def test_multigrid_step_matches_phi_form(n, tau, cycle):
    L, eps = n * math.pi / 4, 0.25
    h = L / n
    phk = inputs.polycrystal_phi0(n, L, 1, seed=31 + n, radius_cells=3)
    want = D.solve_step_fo_phi(phk, h, eps, tau)
    s = cfas.Solver(n, L, eps, tau, tol=1e-12, cycle=cycle, scheme=1)
    mu0, om0 = cfas.initial_guess(phk, h, eps)
    phi, mu, om, info = s.step(phk, phk, mu0, om0)
    assert info.status == 0
    got = np.stack([phi, mu, om])
    assert np.max(np.abs(got - want)) <= 1e-10 * max(1.0, np.max(np.abs(want)))
    # the residual of the three-field system at the phi-form solution is zero
    f = cfas.source_fo(phk, h)
    _, m = cfas.residual_fo(want, f, h, eps, tau)
    assert m < 1e-9


def test_source_ignores_the_older_level():
    n, h = 6, 0.7
    g = inputs.rng(32)
    phk = g.uniform(-1, 1, (n, n, n))
    f = cfas.source_fo(phk, h)
    assert np.array_equal(f[0], phk)
    assert np.max(np.abs(f[1] - 2.0 * D.lap(phk, h))) < 1e-12
    assert np.all(f[2] == 0.0)


def test_local_solve_is_exact():
    g = inputs.rng(33)
    h, eps, tau = 0.6, 0.15, 0.4
    for picard in (False, True):
        for _ in range(10):
            phin, f1, f2, f3, smu, som, sphi = g.uniform(-1, 1, 7)
            phi, mu, om = cfas.local_solve_fo(h, eps, tau, picard, phin, f1, f2, f3, smu, som, sphi)
            c = (phin ** 2 if picard else 3 * phin ** 2) + (1.0 - eps)
            extra = 0.0 if picard else phin ** 3 - 3 * phin ** 2 * phin
            A = np.array([[1.0, 6 * tau / h ** 2, 0.0], [-c, 1.0, 6 / h ** 2], [6 / h ** 2, 0.0, 1.0]])
            b = np.array([f1 + tau * smu / h ** 2, f2 + som / h ** 2 + extra, f3 + sphi / h ** 2])
            x = np.linalg.solve(A, b)
            assert np.max(np.abs(np.array([phi, mu, om]) - x)) <= 1e-12 * max(1.0, np.max(np.abs(x)))


@pytest.mark.parametrize("n,mode,tau", [(8, (1, 2, 0), 0.5), (12, (1, 1, 1), 0.2), (16, (2, 0, 1), 3.0)])
def test_small_mode_follows_the_amplification_factor(n, mode, tau):
    """About phi = 0 the cubic is O(a^3): each step multiplies the mode by the
    closed-form factor to ~1e-12 relative."""
    L, eps, amp = n * math.pi / 4, 0.25, 1e-7
    h = L / n
    base = plane_wave(n, *mode)
    lam = (4 / h ** 2) * sum(math.sin(math.pi * q / n) ** 2 for q in mode)
    G = D.fo_linear_factor(lam, eps, tau)
    phis, infos, _ = cfas.simulate(amp * base, L, eps, tau, 4, tol=1e-18, scheme=1)
    for k in range(1, 5):
        coef = float(np.sum(phis[k] * base) / np.sum(base * base))
        assert abs(coef - amp * G ** k) <= 1e-10 * amp
        assert np.max(np.abs(phis[k] - coef * base)) <= 1e-10 * amp


@pytest.mark.parametrize("tau", [1.0, 20.0])
def test_energy_decreases_for_any_time_step(tau):
    """Convex splitting makes F_h non-increasing step by step, whatever tau."""
    n = 12
    L, eps = n * math.pi / 4, 0.25
    h = L / n
    phi0 = inputs.polycrystal_phi0(n, L, 2, seed=34, radius_cells=3)
    phis, infos, _ = cfas.simulate(phi0, L, eps, tau, 6, tol=1e-11, cycle="F", scheme=1,
                                   max_cycles=2000)
    E = [D.energy(p, h, eps) for p in phis]
    assert all(b <= a + 1e-10 * abs(a) for a, b in zip(E, E[1:])), E
    assert E[-1] < E[0]
    m0 = D.mass(phis[0], h)
    assert all(abs(D.mass(p, h) - m0) <= h ** 3 * n ** 3 * 1e-11 for p in phis)


def test_first_order_in_time():
    """Cauchy differences of the solution at T over tau, tau/2, tau/4 on a
    smooth mode halve with tau (rate 1 within 0.1)."""
    n, L, eps, T = 16, 32.0, 0.025, 1.0
    h = L / n
    phi0 = inputs.smooth_mode_phi0(n, L, noise=0.0)
    sol = {}
    for m in (8, 16, 32):
        phis, _, _ = cfas.simulate(phi0, L, eps, T / m, m, tol=1e-13, scheme=1)
        sol[m] = phis[-1]
    e1 = np.max(np.abs(sol[8] - sol[16]))
    e2 = np.max(np.abs(sol[16] - sol[32]))
    rate = math.log2(e1 / e2)
    assert abs(rate - 1.0) < 0.1, (e1, e2, rate)


def test_constant_state_is_a_fixed_point():
    n, L, eps, tau = 8, 8 * math.pi / 4, 0.25, 0.5
    h = L / n
    phi0 = np.full((n, n, n), 0.3)
    mu, om = cfas.initial_guess(phi0, h, eps)
    s = cfas.Solver(n, L, eps, tau, tol=1e-13, scheme=1)
    phi, mu2, om2, info = s.step(phi0, phi0, mu, om)
    assert info.cycles == 0 and np.array_equal(phi, phi0)


def test_first_order_refuses_variable_mobility():
    with pytest.raises(cfas.OracleError):
        cfas.Solver(8, 6.0, 0.25, 0.5, mobility=(1.0, 0.0, -1.0, 0.05), scheme=1)


@pytest.mark.parametrize("n", [3, 4])
def test_coarsest_newton_is_quadratic(n):
    """Newton with the exact Jacobian: a handful of iterations to 1e-14 (a
    wrong Jacobian still converges, but linearly)."""
    L, eps, tau = n * 2.0, 0.25, 0.5
    h = L / n
    g = inputs.rng(35 + n)
    u0 = np.stack([0.3 + 0.2 * g.uniform(-1, 1, (n, n, n)), g.uniform(-1, 1, (n, n, n)),
                   g.uniform(-1, 1, (n, n, n))])
    f = cfas.apply_N_fo(u0, h, eps, tau)
    start = np.stack([np.full((n, n, n), 0.3), np.zeros((n, n, n)), np.zeros((n, n, n))])
    u, it = cfas.coarse_solve_fo(start, f, h, eps, tau)
    assert 1 <= it <= 7, it
    assert np.max(np.abs(u - u0)) < 1e-11
