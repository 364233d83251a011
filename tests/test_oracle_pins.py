"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it rests on.  None of them compares the oracle
with itself: they use brute-force Fourier modes, identities, closed forms,
fixed points, printed tables and an independently written direct solver.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import cfas
from oracle import definition as D
from paper_1611_06288_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mode(n, r, s, t):
    idx = np.arange(n)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    return np.exp(2j * np.pi * (r * i + s * j + t * k) / n)


# ---------------------------------------------------------------- P1 -----
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_laplacian_symbol_bruteforce(n):
    """Section 4.1: d_x D_x acts on exp(2 pi i r x/L) as u_r^2 with
    u_r = 2 i sin(pi r h/L)/h; Delta_h is the sum over axes.  Checked on every
    mode of tiny grids, for Delta_h, Delta_h^2 and Delta_h^3, on both oracles."""
    L = 1.7 * n
    h = L / n
    for r in range(n):
        for s in range(n):
            for t in range(n):
                m = _mode(n, r, s, t)
                ur2 = [(2j * math.sin(math.pi * q * h / L) / h) ** 2 for q in (r, s, t)]
                lam = sum(ur2).real
                for fn in (lambda v: cfas.laplacian(v, h), lambda v: D.lap(v, h)):
                    re, im = m.real.copy(), m.imag.copy()
                    for p in (1, 2, 3):
                        re, im = fn(re), fn(im)
                        got = re + 1j * im
                        assert np.max(np.abs(got - lam ** p * m)) <= 1e-12 * max(1.0, abs(lam) ** p)


def test_symbol_bounds():
    """Section 4.1: (2/pi)|v_r| <= |u_r| <= |v_r| for -R <= r <= R, m = 2R+1."""
    for m in (5, 9, 17, 33):
        R = (m - 1) // 2
        L = 2.3
        h = L / m
        for r in range(-R, R + 1):
            ur = abs(2 * math.sin(math.pi * r * h / L) / h)
            vr = abs(2 * math.pi * r / L)
            assert 2 / math.pi * vr <= ur + 1e-14 and ur <= vr + 1e-14


def test_lap_symbol_helper_matches_fft():
    n, L = 6, 4.0
    v = inputs.random_field(n, 3)
    ref = np.real(np.fft.ifftn(np.fft.fftn(v) * D.lap_symbol(n, L)))
    assert np.max(np.abs(ref - cfas.laplacian(v, L / n))) < 1e-13


# ---------------------------------------------------------------- P2 -----
def test_summation_by_parts_and_energy_faces():
    """Lemma lemma1: (f, Delta g) = -(grad f, grad g), (f, Delta^2 g) = (Delta f, Delta g),
    (f, Delta^3 g) = -(grad Delta f, grad Delta g).  The gradient norm is the
    face sum of Section 2, so F_h can be rebuilt without faces: a wrong face sum
    in the energy fails here."""
    n, L, eps = 7, 5.0, 0.3
    h = L / n
    f = inputs.random_field(n, 11)
    g = inputs.random_field(n, 12)
    ip = lambda a, b: h ** 3 * float(np.sum(a * b))

    def gip(a, b):
        tot = 0.0
        for ax in range(3):
            tot += float(np.sum((np.roll(a, -1, ax) - a) * (np.roll(b, -1, ax) - b))) / h ** 2
        return h ** 3 * tot

    Lf, Lg = cfas.laplacian(f, h), cfas.laplacian(g, h)
    assert abs(ip(f, Lg) + gip(f, g)) < 1e-11 * abs(gip(f, g))
    assert abs(ip(f, cfas.laplacian(Lg, h)) - ip(Lf, Lg)) < 1e-11 * abs(ip(Lf, Lg))
    L3g = cfas.laplacian(cfas.laplacian(Lg, h), h)
    assert abs(ip(f, L3g) + gip(Lf, Lg)) < 1e-11 * abs(gip(Lf, Lg))
    # energy without face sums: -|grad phi|^2 = (phi, Delta phi)
    phi = 0.3 + 0.2 * f
    F_sbp = (0.25 * h ** 3 * np.sum(phi ** 4) + 0.5 * (1 - eps) * ip(phi, phi)
             + ip(phi, cfas.laplacian(phi, h)) + 0.5 * ip(cfas.laplacian(phi, h), cfas.laplacian(phi, h)))
    Fc, Ft, mass = cfas.energy(phi, h, eps, phi_prev=phi)
    assert abs(Fc - F_sbp) < 1e-12 * abs(F_sbp)
    assert Ft == pytest.approx(Fc, rel=1e-15, abs=1e-15)
    assert mass == pytest.approx(h ** 3 * np.sum(phi), rel=1e-14)
    assert D.energy(phi, h, eps) == pytest.approx(F_sbp, rel=1e-12)
    # modified energy term: 1/2 |grad(phi - prev)|^2 = -1/2 (w, Delta w)
    prev = phi + 0.1 * g
    w = phi - prev
    _, Ft2, _ = cfas.energy(phi, h, eps, phi_prev=prev)
    assert Ft2 - Fc == pytest.approx(-0.5 * ip(w, cfas.laplacian(w, h)), rel=1e-11)


# ---------------------------------------------------------------- P3 -----
@pytest.mark.parametrize("picard", [False, True])
def test_local_solve_matches_linear_algebra(picard):
    """Section 5 smoothing scheme: the pointwise 3x3 system, built here from the
    equations N(u) = f with neighbours fixed, solved by numpy."""
    g = inputs.rng(5)
    for _ in range(200):
        h = g.uniform(0.2, 3.0)
        tau = g.uniform(1e-3, 2.0)
        eps = g.uniform(0.0, 0.5)
        phin, phk, f1, f2, f3 = g.uniform(-1, 1, 5)
        smu, som, sphi = g.uniform(-5, 5, 3)
        if picard:
            q = 0.25 * (phin ** 2 + phk ** 2)
            c, extra = q + 0.5 * (1 - eps), q * phk
        else:
            gp = 0.25 * (3 * phin ** 2 + 2 * phin * phk + phk ** 2)
            gv = 0.25 * (phin + phk) * (phin ** 2 + phk ** 2)
            c, extra = gp + 0.5 * (1 - eps), gv - gp * phin
        # phi - tau (smu - 6 mu)/h^2 = f1
        # mu - c phi - (som - 6 om)/h^2 = f2 + extra
        # om - (sphi - 6 phi)/(2 h^2) = f3
        A = np.array([[1.0, 6 * tau / h ** 2, 0.0],
                      [-c, 1.0, 6 / h ** 2],
                      [3 / h ** 2, 0.0, 1.0]])
        b = np.array([f1 + tau * smu / h ** 2, f2 + extra + som / h ** 2, f3 + sphi / (2 * h ** 2)])
        ref = np.linalg.solve(A, b)
        got = cfas.local_solve(h, eps, tau, picard, phin, phk, f1, f2, f3, smu, som, sphi)
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))


def test_half_sweep_zeroes_linear_residuals_on_its_colour():
    """After a half-sweep, the two linear equations (N1, N3) hold exactly at
    every updated point, and at the other colour nothing moved."""
    n, L, eps, tau = 8, 9.0, 0.2, 0.3
    h = L / n
    g = inputs.rng(9)
    phk = 0.3 + 0.1 * g.uniform(-1, 1, (n, n, n))
    u = np.stack([phk + 0.05 * g.uniform(-1, 1, (n, n, n)), g.uniform(-1, 1, (n, n, n)),
                  g.uniform(-1, 1, (n, n, n))])
    f = D.source(phk, phk, h, eps)
    idx = np.arange(n)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    for colour in (0, 1):
        u2 = cfas.smooth_half(u, f, phk, h, eps, tau, colour)
        mask = ((i + j + k) % 2) == colour
        r = f - D.apply_N(u2, phk, h, eps, tau)
        assert np.max(np.abs(r[0][mask])) < 1e-12
        assert np.max(np.abs(r[2][mask])) < 1e-12
        assert np.array_equal(u2[:, ~mask], u[:, ~mask])
        # Newton on the cubic: iterating the point solve drives N2 to zero too
        u3 = u2
        for _ in range(30):
            u3 = cfas.smooth_half(u3, f, phk, h, eps, tau, colour)
        r3 = f - D.apply_N(u3, phk, h, eps, tau)
        assert np.max(np.abs(r3[:, mask])) < 1e-11


# ---------------------------------------------------------------- P4 -----
@pytest.mark.parametrize("n", [6, 8, 12])
def test_constant_state_is_exact_fixed_point(n):
    """Scheme (1.10): a constant phi is a steady state; with the consistent
    guess mu = c^3 + (1-eps)c, omega = 0 the step needs zero cycles."""
    L, eps, tau, c = 1.3 * n, 0.25, 0.5, 0.285
    phi = np.full((n, n, n), c)
    s = cfas.Solver(n, L, eps, tau, tol=1e-13)
    mu, om = cfas.initial_guess(phi, L / n, eps)
    assert np.allclose(mu, c ** 3 + (1 - eps) * c, rtol=1e-15)
    out, mu2, om2, info = s.step(phi, phi, mu, om)
    assert info.status == 0 and info.cycles == 0
    assert np.array_equal(out, phi)


@pytest.mark.parametrize("n", [6, 7, 8])
def test_initial_guess_is_the_gradient_of_the_discrete_energy(n):
    """The first-step guess mu = phi^3 + (1-eps) phi + 2 Delta_h phi +
    Delta_h^2 phi is the discrete chemical potential of (equation-PFC): the
    gradient of F_h (PFC energy-discrete-1) in the h^3-weighted inner
    product.  So along any direction v the central difference of F_h must
    equal h^3 sum(mu v).  F_h is a quartic polynomial in phi, so the
    five-point difference used here is exact up to rounding.  The last
    direction is the constant one (d/dc F_h(phi + c) = h^3 sum(mu))."""
    L, eps = 1.3 * n, 0.25
    h = L / n
    g = inputs.rng(100 + n)
    phi = 0.2 + 0.3 * g.uniform(-1.0, 1.0, size=(n, n, n))
    mu, om = cfas.initial_guess(phi, h, eps)

    def slope(v, d=1e-3):
        def F(t):
            return D.energy(phi + t * v, h, eps)
        return (8.0 * (F(d) - F(-d)) - (F(2 * d) - F(-2 * d))) / (12.0 * d)

    dirs = [g.standard_normal((n, n, n)) for _ in range(3)] + [np.ones_like(phi)]
    for trial, v in enumerate(dirs):
        v = v / np.linalg.norm(v)
        fd = slope(v)
        got = h ** 3 * float(np.sum(mu * v))
        assert abs(fd - got) <= 1e-9 * max(1.0, abs(got)), (trial, fd, got)


@pytest.mark.parametrize("mode", [(1, 0, 0), (1, 2, 0), (2, 1, 3)])
def test_initial_guess_omega_and_mu_on_a_fourier_mode(mode):
    """On phi = a cos(2 pi (r i + s j + t k)/n) the guess must give
    omega = lambda phi and mu = phi^3 + (1 - eps) phi + (2 lambda + lambda^2) phi
    with the brute-force symbol lambda = -(4/h^2) sum sin^2(pi r/n) of
    Section 4.1 (a sign or factor slip on either Laplacian term changes the
    lambda polynomial)."""
    n, L, eps, a = 8, 10.4, 0.3, 0.4
    h = L / n
    phi = np.ascontiguousarray(a * _mode(n, *mode).real)
    lam = -(4.0 / h ** 2) * sum(math.sin(math.pi * r / n) ** 2 for r in mode)
    mu, om = cfas.initial_guess(phi, h, eps)
    assert np.max(np.abs(om - lam * phi)) < 1e-12 * max(1.0, abs(lam))
    want = phi ** 3 + (1.0 - eps) * phi + (2.0 * lam + lam * lam) * phi
    assert np.max(np.abs(mu - want)) < 1e-12 * max(1.0, lam * lam)


def test_transfers_preserve_constants_and_linear_fields():
    """Restriction (8-child mean) and cell-centred trilinear interpolation:
    constants are preserved; a field linear in x is reproduced exactly away
    from the periodic seam (both operators are second-order accurate)."""
    nc = 8
    hc = 1.0
    c = np.full((nc, nc, nc), 2.5)
    assert np.allclose(cfas.prolong_add(c, np.zeros((16, 16, 16))), 2.5, rtol=0, atol=1e-15)
    assert np.allclose(cfas.restrict(np.full((16, 16, 16), -1.25)), -1.25, rtol=0, atol=1e-15)
    xc = (np.arange(nc) + 0.5) * hc
    ec = np.broadcast_to(3.0 * xc + 1.0, (nc, nc, nc)).copy()
    fine = cfas.prolong_add(ec, np.zeros((2 * nc,) * 3))
    xf = (np.arange(2 * nc) + 0.5) * hc / 2
    interior = slice(1, 2 * nc - 1)
    assert np.allclose(fine[:, :, interior], (3.0 * xf + 1.0)[interior], atol=1e-13)
    lin_f = np.broadcast_to(2.0 * xf - 0.5, (2 * nc,) * 3).copy()
    assert np.allclose(cfas.restrict(lin_f), 2.0 * xc - 0.5, atol=1e-13)
    # sums: restriction of a sum-zero field has zero sum; P keeps the mean
    g = inputs.random_field(nc, 4)
    g -= g.mean()
    assert abs(cfas.prolong_add(g, np.zeros((2 * nc,) * 3)).sum()) < 1e-11


# ---------------------------------------------------------------- P5 -----
def _mode_recurrence(lam, eps, tau, a0, steps):
    """Linearised scheme (1.10) about phi = 0 on one Fourier mode (eigenvalue
    lam of Delta_h), derived by substituting the mode into the three equations:
    a' - a = tau lam [ (1-eps)/2 (a'+a) + 3 lam a - lam a_prev + lam^2 (a'+a)/2 ]."""
    beta = 0.5 * (1 - eps) + 0.5 * lam ** 2
    a_prev, a = a0, a0
    out = [a0]
    for _ in range(steps):
        a_next = (a * (1 + tau * lam * beta + 3 * tau * lam ** 2) - tau * lam ** 2 * a_prev) / (1 - tau * lam * beta)
        a_prev, a = a, a_next
        out.append(a)
    return out


@pytest.mark.parametrize("n,mode,tau", [(8, (1, 2, 0), 0.5), (12, (1, 1, 1), 0.2), (16, (2, 0, 1), 0.05)])
def test_single_linear_mode_follows_recurrence(n, mode, tau):
    """Small-amplitude single mode, mean zero: the cubic term is O(a^3), so
    each step must follow the linear recurrence to ~1e-12 relative."""
    L, eps, amp = n * math.pi / 4, 0.25, 1e-7
    h = L / n
    r, s, t = mode
    base = np.real(_mode(n, r, s, t))
    phi0 = amp * base
    lam = -(4 / h ** 2) * sum(math.sin(math.pi * q / n) ** 2 for q in mode)
    ref = _mode_recurrence(lam, eps, tau, amp, 5)
    phis, infos, _ = cfas.simulate(phi0, L, eps, tau, 5, tol=1e-19)
    for kstep in range(1, 6):
        coef = float(np.sum(phis[kstep] * base) / np.sum(base * base))
        assert abs(coef - ref[kstep]) <= 1e-10 * abs(amp)
        assert np.max(np.abs(phis[kstep] - coef * base)) <= 1e-10 * amp
    # the definition solver too
    dphis, _ = D.simulate_dense(phi0, h, eps, tau, 2, solver="nk")
    coef = float(np.sum(dphis[2] * base) / np.sum(base * base))
    assert abs(coef - ref[2]) <= 1e-10 * amp


# ---------------------------------------------------------------- P7 -----
def test_mass_identity_any_iterate():
    """Summing N1 over the periodic grid kills Delta_h mu, so for ANY iterate
    sum(phi) - sum(phi^k) = -sum(r1), and for the converged step the mass
    drift is bounded by the tolerance."""
    n, L, eps, tau = 16, 16 * math.pi / 4, 0.25, 0.5
    h = L / n
    phi0 = inputs.polycrystal_phi0(n, L, 1, seed=21, radius_cells=4)
    mu, om = cfas.initial_guess(phi0, h, eps)
    f = cfas.source(phi0, phi0, h, eps)
    u = np.stack([phi0, mu, om])
    s = cfas.Solver(n, L, eps, tau)
    for _ in range(3):
        u, _ = s.cycle(u, f, phi0)
        r, _ = cfas.residual(u, f, phi0, h, eps, tau)
        drift = np.sum(u[0]) - np.sum(phi0)
        assert abs(drift + np.sum(r[0])) < 1e-12 * np.sum(np.abs(phi0))
    phis, infos, _ = cfas.simulate(phi0, L, eps, tau, 3, tol=1e-10)
    for a, b in zip(phis[:-1], phis[1:]):
        assert abs(D.mass(b, h) - D.mass(a, h)) <= h ** 3 * n ** 3 * 1e-10


# ---------------------------------------------------------------- P8 -----
def _energy_identity_defect(phis, mus, h, eps, tau):
    """F~(a,b) - F~(b,c) + tau|grad mu|^2 + 1/2|grad(a - 2b + c)|^2 per step
    (test of the first equation of (1.10) with mu, see prop:hu09)."""
    out = []
    for k in range(1, len(phis)):
        a = phis[k]
        b = phis[k - 1]
        c = phis[k - 2] if k >= 2 else phis[0]
        Fa = D.modified_energy(a, b, h, eps)
        Fb = D.modified_energy(b, c, h, eps)
        rhs = -tau * D.grad_norm2(mus[k - 1], h) - 0.5 * D.grad_norm2(a - 2 * b + c, h)
        out.append((Fa - Fb - rhs, Fa, Fb))
    return out


def test_energy_identity_and_decay_fas():
    n, eps, tau = 16, 0.25, 0.5
    L = n * math.pi / 4
    h = L / n
    phi0 = inputs.polycrystal_phi0(n, L, 2, seed=8, radius_cells=4)
    mus = []
    phis, infos, _ = cfas.simulate(phi0, L, eps, tau, 4, tol=1e-12,
                                   callback=lambda k, p, mu, om, i: mus.append(mu.copy()))
    for defect, Fa, Fb in _energy_identity_defect(phis, mus, h, eps, tau):
        assert abs(defect) < 1e-8 * max(1.0, abs(Fa))
        assert Fa <= Fb + 1e-10               # monotone modified energy
    # the oracle's own energy routine agrees with the definition
    F0, Ft, _ = cfas.energy(phis[2], h, eps, phis[1])
    assert Ft == pytest.approx(D.modified_energy(phis[2], phis[1], h, eps), rel=1e-12)
    # Proposition prop:hu09 bound
    bound = D.modified_energy(phis[1], phis[0], h, eps)
    for p in phis[1:]:
        assert D.energy(p, h, eps) <= bound + 1e-10


def test_energy_identity_definition_solver():
    n, eps, tau = 6, 0.25, 0.5
    L = 1.5 * math.pi
    h = L / n
    phi0 = 0.285 + 0.1 * inputs.random_field(n, 31)
    phis, mus = D.simulate_dense(phi0, h, eps, tau, 4)
    for defect, Fa, Fb in _energy_identity_defect(phis, mus, h, eps, tau):
        assert abs(defect) < 1e-12 * max(1.0, abs(Fa))


# ---------------------------------------------------------------- P9 -----
@pytest.mark.parametrize("n,solver", [(6, "dense"), (8, "dense"), (12, "nk"), (16, "nk")])
def test_fas_converges_to_the_unique_step_solution(n, solver):
    """Proposition prop:hu09: the step has one solution; the FAS mirror reaches
    the directly solved one to within the residual tolerance's reach."""
    L, eps, tau, tol = n * math.pi / 4, 0.25, 0.5, 1e-12
    h = L / n
    phk = inputs.polycrystal_phi0(n, L, 1, seed=40 + n, radius_cells=3)
    phkm1 = phk + 0.01 * inputs.random_field(n, 41)
    ref = (D.solve_step_dense if solver == "dense" else D.solve_step_nk)(phkm1, phk, h, eps, tau)
    s = cfas.Solver(n, L, eps, tau, tol=tol, max_cycles=400)
    mu, om = cfas.initial_guess(phk, h, eps)
    out, mu2, om2, info = s.step(phkm1, phk, mu, om)
    assert info.status == 0
    assert np.max(np.abs(out - ref[0])) <= 10 * tol * (1 + tau * 6 / h ** 2) ** 2
    assert np.max(np.abs(mu2 - ref[1])) <= 1e-9
    assert np.max(np.abs(om2 - ref[2])) <= 1e-9


def test_coarse_solve_reaches_exact_solution():
    n, L, eps, tau = 4, 4 * 16.0, 0.25, 0.5
    h = L / n
    g = inputs.rng(77)
    phk = 0.285 + 0.1 * g.uniform(-1, 1, (n, n, n))
    u0 = np.stack([phk, g.uniform(-1, 1, (n, n, n)), g.uniform(-1, 1, (n, n, n))])
    f = D.apply_N(u0, phk, h, eps, tau) + 0.01 * g.uniform(-1, 1, (3, n, n, n))
    u, it = cfas.coarse_solve(np.stack([phk, u0[1], u0[2]]), f, phk, h, eps, tau)
    assert 1 <= it < 30
    r = f - D.apply_N(u, phk, h, eps, tau)
    assert np.max(np.abs(r)) < 1e-13


def test_step_cycles_V_and_F_agree_on_result():
    n, eps, tau = 16, 0.25, 0.5
    L = n * math.pi / 4
    phi0 = inputs.polycrystal_phi0(n, L, 2, seed=3, radius_cells=4)
    pv, iv, _ = cfas.simulate(phi0, L, eps, tau, 2, tol=1e-11, cycle="V")
    pf, if_, _ = cfas.simulate(phi0, L, eps, tau, 2, tol=1e-11, cycle="F")
    pp, ip_, _ = cfas.simulate(phi0, L, eps, tau, 2, tol=1e-11, lin="picard")
    assert np.max(np.abs(pv[-1] - pf[-1])) < 1e-9
    assert np.max(np.abs(pv[-1] - pp[-1])) < 1e-9
    assert sum(i.cycles for i in if_) <= sum(i.cycles for i in iv)


# --------------------------------------------------------------- P10 -----
@pytest.mark.parametrize("n", [16, 32])
def test_multigrid_complexity_table2(n):
    """Table tab:complexity (Section 6.1): cycles to 1e-8 at the 10th step,
    tau = 1e-3, eps = 0.025, Omega = [0,3.2]^3, init1.  The paper's restriction,
    interpolation and start guess are not stated, so counts are matched within
    +-1 for V(2,2) and +-2 for V(1,1)."""
    ref = json.load(open(os.path.join(GOLDEN, "table2_complexity.json")))
    for nu in ((1, 1), (2, 2)):
        phis, infos, _ = cfas.simulate(inputs.paper_init1(n), 3.2, 0.025, 1e-3, 10, tol=1e-8,
                                       nu1=nu[0], nu2=nu[1])
        want = ref["cycles"][f"{nu[0]},{nu[1]}"][str(n)]
        slack = 1 if nu == (2, 2) else 2
        assert abs(infos[9].cycles - want) <= slack, (nu, infos[9].cycles, want)


# ---------------------------------------------------------------- P6 -----
def test_second_order_in_space_and_time():
    """Theorem thm:convergence: error O(tau^2 + h^2).  Smooth data, refinement
    path tau = 0.02 h, Cauchy differences compared on the coarse grid through
    the 8-child cell average (itself O(h^2)).  The paper's Table tab:cov
    reports rates 2.0099 and 2.0096; the observed rate must be within 0.1."""
    rates = json.load(open(os.path.join(GOLDEN, "table1_cauchy.json")))["rates"]
    L, eps, T = 32.0, 0.025, 0.64
    sol = {}
    for n in (8, 16, 32):
        h = L / n
        tau = 0.02 * h
        steps = int(round(T / tau))
        phis, _, _ = cfas.simulate(inputs.smooth_mode_phi0(n, L, noise=0.0), L, eps, tau, steps, tol=1e-10)
        sol[n] = phis[-1]
    e1 = math.sqrt((L / 8) ** 3 * np.sum((cfas.restrict(sol[16]) - sol[8]) ** 2))
    e2 = math.sqrt((L / 16) ** 3 * np.sum((cfas.restrict(sol[32]) - sol[16]) ** 2))
    rate = math.log2(e1 / e2)
    assert abs(rate - rates["32-64"]) < 0.1, rate


def test_time_order_linear_mode_analytic():
    """Second order in time alone: the linear-mode recurrence of the scheme
    against the exact semi-discrete decay exp(sigma_h t),
    sigma_h = lam((1 + lam)^2 - eps), from (equation-PFC) linearised at 0."""
    n, L, eps = 8, 8.0, 0.025
    h = L / n
    lam = -(4 / h ** 2) * math.sin(math.pi / n) ** 2
    sigma = lam * ((1 + lam) ** 2 - eps)
    T = 2.0
    errs = []
    for steps in (40, 80, 160):
        tau = T / steps
        a = _mode_recurrence(lam, eps, tau, 1.0, steps)[-1]
        errs.append(abs(a - math.exp(sigma * T)))
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2


# --------------------------------------------------------------- P11 -----
def test_adjoint_dense_matches_finite_differences():
    """Implicit-function adjoint of the exactly solved rollout against central
    differences of the same exact rollout (4^3, 3 steps)."""
    n, eps, tau, steps = 4, 0.2, 0.3, 3
    L = 4.0
    h = L / n
    phi0 = 0.2 + 0.05 * inputs.random_field(n, 5)
    target = 0.2 + 0.05 * inputs.random_field(n, 6)
    loss, gphi, geps = D.rollout_loss_grad_dense(phi0, target, h, eps, tau, steps)
    v = inputs.unit_direction(phi0.shape, 7)
    d = 1e-6

    def L_of(p, e):
        phis, _ = D.simulate_dense(p, h, e, tau, steps)
        return float(np.sum((phis[-1] - target) ** 2))

    fd = (L_of(phi0 + d * v, eps) - L_of(phi0 - d * v, eps)) / (2 * d)
    assert fd == pytest.approx(float(np.sum(gphi * v)), rel=1e-6)
    fde = (L_of(phi0, eps + d) - L_of(phi0, eps - d)) / (2 * d)
    assert fde == pytest.approx(geps, rel=1e-6)
