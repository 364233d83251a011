"""Pins of the oracle's variable-mobility form (Section 5, first equation in
flux form, phi - tau d(M(A phi*) D mu) = ...) against what the mathematics
fixes: an independently assembled matrix (definition.py builds
d diag(M) D from the face operators of Section 2; the C oracle sums face
fluxes), symmetry and semi-definiteness of that operator, the reduction of a
constant mobility c to M = 1 with time step c tau, an exact 3x3 solve, the
dense Newton step, and conservation of mass and decay of the modified energy.
"""
import math

import numpy as np
import pytest

from oracle import cfas
from oracle import definition as D
from paper_1611_06288_amd import inputs

MOB = (1.0, 0.0, -1.0, 0.05)      # M(v) = max(0.05, 1 - v^2)
MOB_LIN = (0.8, 0.9, 0.0, 0.1)    # M(v) = max(0.1, 0.8 + 0.9 v)


def rand_fields(n, seed, mean=0.2):
    g = inputs.rng(seed)
    phk = mean + 0.2 * g.uniform(-1, 1, (n, n, n))
    phkm1 = phk + 0.05 * g.uniform(-1, 1, (n, n, n))
    u = np.stack([phk + 0.03 * g.uniform(-1, 1, (n, n, n)), g.uniform(-1, 1, (n, n, n)),
                  g.uniform(-1, 1, (n, n, n))])
    return phkm1, phk, u


@pytest.mark.parametrize("mob", [MOB, MOB_LIN])
def test_flux_operator_matches_assembled_matrix(mob):
    n, h, eps, tau = 6, 0.8, 0.2, 0.3
    phkm1, phk, u = rand_fields(n, 11)
    phs = 1.5 * phk - 0.5 * phkm1
    got = cfas.apply_N_m(u, phk, phs, h, eps, tau, mob)
    want = D.apply_N_mob(u, phk, phs, h, eps, tau, mob)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_mobility_operator_structure():
    n, h = 4, 0.5
    _, phk, _ = rand_fields(n, 12)
    Lm = D.mobility_matrix(n, h, phk, MOB).toarray()
    assert np.max(np.abs(Lm - Lm.T)) < 1e-12                  # symmetric
    assert np.max(np.abs(Lm.sum(axis=1))) < 1e-11             # constants in the kernel
    ev = np.linalg.eigvalsh(Lm)
    assert ev.max() < 1e-10 and ev.min() < -1.0               # negative semi-definite
    # M = 1 is the plain 7-point Laplacian
    L1 = D.mobility_matrix(n, h, phk, (1.0, 0.0, 0.0, 0.0)).toarray()
    assert np.max(np.abs(L1 - D.lap_matrix(n, h).toarray())) < 1e-12


def test_local_solve_is_exact():
    g = inputs.rng(13)
    h, eps, tau = 0.6, 0.15, 0.4
    for _ in range(20):
        phin, phk, f1, f2, f3, smu, som, sphi = g.uniform(-1, 1, 8)
        msum = g.uniform(0.5, 6.0)
        phi, mu, om = cfas.local_solve_m(h, eps, tau, False, phin, phk, f1, f2, f3, msum, smu, som,
                                         sphi)
        # the linearised point equations, written out
        c = D.g_cubic_dphi(phin, phk) + 0.5 * (1.0 - eps)
        A = np.array([[1.0, tau * msum / h ** 2, 0.0], [-c, 1.0, 6.0 / h ** 2],
                      [3.0 / h ** 2, 0.0, 1.0]])
        b = np.array([f1 + tau * smu / h ** 2,
                      f2 + som / h ** 2 + D.g_cubic(phin, phk) - D.g_cubic_dphi(phin, phk) * phin,
                      f3 + sphi / (2 * h ** 2)])
        x = np.linalg.solve(A, b)
        assert np.max(np.abs(np.array([phi, mu, om]) - x)) <= 1e-12 * max(1.0, np.max(np.abs(x)))


def test_constant_mobility_is_a_rescaled_time_step():
    """M = c turns tau d(M D mu) into (c tau) Delta_h mu: the step equals the
    M = 1 step with time step c tau (closed form)."""
    n, L, eps, tau, c = 8, 6.0, 0.2, 0.3, 0.7
    h = L / n
    phkm1, phk, _ = rand_fields(n, 14)
    a = D.solve_step_dense_mob(phkm1, phk, h, eps, tau, (c, 0.0, 0.0, 0.0))
    b = D.solve_step_dense(phkm1, phk, h, eps, c * tau)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    # and the multigrid oracle agrees with both
    s = cfas.Solver(n, L, eps, tau, tol=1e-13, mobility=(c, 0.0, 0.0, 0.0))
    mu0, om0 = cfas.initial_guess(phk, h, eps)
    phi, mu, om, info = s.step(phkm1, phk, mu0, om0)
    assert info.status == 0
    assert np.max(np.abs(phi - b[0])) < 1e-11


@pytest.mark.parametrize("mob", [MOB, MOB_LIN])
def test_multigrid_step_matches_dense_newton(mob):
    n, L, eps, tau = 8, 8.0, 0.25, 0.5
    h = L / n
    phkm1, phk, _ = rand_fields(n, 15, mean=0.28)
    want = D.solve_step_dense_mob(phkm1, phk, h, eps, tau, mob)
    s = cfas.Solver(n, L, eps, tau, tol=1e-12, mobility=mob)
    mu0, om0 = cfas.initial_guess(phk, h, eps)
    phi, mu, om, info = s.step(phkm1, phk, mu0, om0)
    assert info.status == 0
    got = np.stack([phi, mu, om])
    assert np.max(np.abs(got - want)) <= 1e-10 * max(1.0, np.max(np.abs(want)))


def test_mass_conserved_and_modified_energy_decays():
    n = 16
    p = inputs.polycrystal_params(n)
    phi0 = inputs.polycrystal_phi0(n, p.L, 2, seed=21, radius_cells=4)
    phis, infos, _ = cfas.simulate(phi0, p.L, p.eps, p.dt, 6, tol=1e-12, mobility=MOB)
    h = p.L / n
    m0 = np.sum(phis[0])
    for k in range(1, len(phis)):
        assert abs(np.sum(phis[k]) - m0) <= 1e-11 * abs(m0)
    E = [cfas.energy(phis[k], h, p.eps, phis[k - 1])[1] for k in range(1, len(phis))]
    assert all(E[k + 1] <= E[k] + 1e-9 * abs(E[k]) for k in range(len(E) - 1)), E
    # the mobility actually varies on this data
    phs = 1.5 * phis[-1] - 0.5 * phis[-2]
    M = D.mobility(phs, MOB)
    assert M.max() - M.min() > 0.1


@pytest.mark.parametrize("mob", [MOB, MOB_LIN])
def test_flux_operator_with_the_floor_reached(mob):
    """phi* spread so that a good share of the faces sit on the floor mmin of
    M: the flux operator still equals the independently assembled matrix."""
    n, h, eps, tau = 6, 0.8, 0.2, 0.3
    phkm1, phk, u = rand_fields(n, 16)
    phs = inputs.rng(17).uniform(-1.3, 1.3, (n, n, n))
    A = [D.face_average_matrix(n, ax) @ phs.ravel() for ax in range(3)]
    floor = sum(int(np.sum(D.mobility(a, mob) == mob[3])) for a in A)
    assert floor > 10, floor
    got = cfas.apply_N_m(u, phk, phs, h, eps, tau, mob)
    want = D.apply_N_mob(u, phk, phs, h, eps, tau, mob)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("n", [3, 4])
def test_coarsest_newton_is_quadratic(n):
    """Newton with the exact Jacobian of the flux form: a handful of iterations
    to 1e-14 (a wrong Jacobian still converges, but linearly)."""
    L, eps, tau = n * 2.0, 0.25, 0.5
    h = L / n
    g = inputs.rng(18 + n)
    phk = 0.285 + 0.1 * g.uniform(-1, 1, (n, n, n))
    phs = 0.2 + g.uniform(-1, 1, (n, n, n))
    u0 = np.stack([phk + 0.2 * g.uniform(-1, 1, (n, n, n)), g.uniform(-1, 1, (n, n, n)),
                   g.uniform(-1, 1, (n, n, n))])
    f = cfas.apply_N_m(u0, phk, phs, h, eps, tau, MOB)
    start = np.stack([phk, np.zeros_like(phk), np.zeros_like(phk)])
    u, it = cfas.coarse_solve_m(start, f, phk, phs, h, eps, tau, MOB)
    assert 1 <= it <= 7, it
    assert np.max(np.abs(u - u0)) < 1e-11
