"""Definition oracle (numpy/scipy, FP64).  Test infrastructure only.

Solves the discrete system of one step of scheme (1.10) directly, with no
multigrid, plus the discrete energy and the Fourier symbols of Section 4.
Written from the paper (arXiv:1611.06288):

* Section 2: cell-centred periodic grid, ``Delta_h`` (7-point), face
  differences ``D_x, D_y, D_z``, norms, discrete energy ``F_h``
  (PFC energy-discrete-1), summation-by-parts identities (Lemma lemma1).
* Section 3, scheme (1.10) in the three-unknown form of Section 5 with M = 1:
  operator N (scheme-PFC-o1..o3) and source S (scheme-PFC-s1..s3).
* Section 4.1: eigenvalues of the difference operators on Fourier modes,
  ``D_x <-> 2 i sin(pi r h / L) / h`` and ``d_x D_x <-> (2 i sin(pi r h/L)/h)^2``.
* Proposition prop:hu09: the step solution is unique, so "the" result of a
  step is well defined and any solver converging to it is comparable.
* The adjoint of one step follows from the implicit-function theorem applied
  to ``G(u; phi^k, phi^{k-1}, eps) = N(u) - S = 0``.
* Section 5 with a variable mobility: the first equation in flux form,
  ``phi - tau d_x(M(A_x phi*) D_x mu) - ... ``, assembled here as the sparse
  matrix ``d_x diag(M_face) D_x + ...`` from the face operators of Section 2
  (``mobility_matrix``); M(v) = max(mmin, m0 + m1 v + m2 v^2) and
  phi* = 3/2 phi^kappa - 1/2 phi^{kappa-1} (the paper leaves M open).

Solvers:
* ``solve_step_dense`` -- Newton with the dense 3n^3 Jacobian (n <= 8).
* ``solve_step_nk``    -- Newton on phi alone after eliminating omega and mu
  (exact, the eliminated equations are linear), inner GMRES preconditioned
  by the constant-coefficient FFT symbol (n <= 32).

Parity status: every function here is pinned by the tests in
``tests/test_oracle_*.py`` (symbols by brute force, SBP identities, closed
forms, fixed points, energy identity, mass identity, order of accuracy).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ------------------------------------------------------------ operators ---

def lap(v: np.ndarray, h: float) -> np.ndarray:
    """Delta_h on the last three axes, periodic."""
    s = (np.roll(v, 1, -1) + np.roll(v, -1, -1) + np.roll(v, 1, -2) + np.roll(v, -1, -2)
         + np.roll(v, 1, -3) + np.roll(v, -1, -3))
    return (s - 6.0 * v) / (h * h)


def lap_matrix(n: int, h: float) -> sp.csr_matrix:
    """Delta_h as a sparse n^3 x n^3 matrix acting on C-ordered [k][j][i] arrays."""
    idx = np.arange(n ** 3).reshape(n, n, n)
    rows, cols, vals = [], [], []
    for axis in range(3):
        for shift in (1, -1):
            nb = np.roll(idx, shift, axis)
            rows.append(idx.ravel())
            cols.append(nb.ravel())
            vals.append(np.full(n ** 3, 1.0 / h ** 2))
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(np.full(n ** 3, -6.0 / h ** 2))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n ** 3, n ** 3))


def lap_symbol(n: int, L: float) -> np.ndarray:
    """Eigenvalues of Delta_h on the modes exp(2 pi i (r x + s y + t z)/L),
    indexed [t][s][r] like numpy's fftn: -(4/h^2) sum sin^2(pi r h / L)."""
    h = L / n
    r = np.arange(n)
    s1 = np.sin(np.pi * r / n) ** 2
    return -(4.0 / h ** 2) * (s1[:, None, None] + s1[None, :, None] + s1[None, None, :])


def face_difference_matrix(n: int, h: float, axis: int) -> sp.csr_matrix:
    """D along `axis` (Section 2): face (i + 1/2) value (v_{i+1} - v_i)/h; the
    face i + 1/2 is stored at cell index i."""
    idx = np.arange(n ** 3).reshape(n, n, n)
    nb = np.roll(idx, -1, axis)     # cell i + 1 along the axis
    P = n ** 3
    rows = np.concatenate([idx.ravel(), idx.ravel()])
    cols = np.concatenate([nb.ravel(), idx.ravel()])
    vals = np.concatenate([np.full(P, 1.0 / h), np.full(P, -1.0 / h)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(P, P))


def face_average_matrix(n: int, axis: int) -> sp.csr_matrix:
    """A along `axis` (Section 2): face (i + 1/2) value (v_{i+1} + v_i)/2."""
    idx = np.arange(n ** 3).reshape(n, n, n)
    nb = np.roll(idx, -1, axis)
    P = n ** 3
    rows = np.concatenate([idx.ravel(), idx.ravel()])
    cols = np.concatenate([nb.ravel(), idx.ravel()])
    return sp.csr_matrix((np.full(2 * P, 0.5), (rows, cols)), shape=(P, P))


def mobility(v, mob):
    m0, m1, m2, mmin = mob
    return np.maximum(mmin, m0 + m1 * v + m2 * v * v)


def mobility_matrix(n: int, h: float, phs: np.ndarray, mob) -> sp.csr_matrix:
    """sum over axes of d (diag(M(A phs)) D), with d = -D^T (the cell
    difference of face values, Section 2), as a sparse n^3 x n^3 matrix."""
    Lm = sp.csr_matrix((n ** 3, n ** 3))
    for axis in range(3):
        D = face_difference_matrix(n, h, axis)
        Mf = mobility(face_average_matrix(n, axis) @ phs.ravel(), mob)
        Lm = Lm + (-D.T) @ sp.diags(Mf) @ D
    return Lm.tocsr()


def apply_N_mob(u, phk, phs, h, eps, tau, mob):
    phi, mu, om = u
    n = phk.shape[0]
    Lm = mobility_matrix(n, h, phs, mob)
    return np.stack([
        phi - tau * (Lm @ mu.ravel()).reshape(phi.shape),
        mu - g_cubic(phi, phk) - 0.5 * (1.0 - eps) * phi - lap(om, h),
        om - 0.5 * lap(phi, h),
    ])


def solve_step_dense_mob(phkm1, phk, h, eps, tau, mob, guess=None, tol=1e-14, maxit=50):
    """Newton with the dense Jacobian on N(u) = S with variable mobility
    (n <= 8); phi* = 3/2 phk - 1/2 phkm1.  Returns u (3,n,n,n)."""
    n = phk.shape[0]
    P = n ** 3
    phs = 1.5 * phk - 0.5 * phkm1
    S = source(phk, phkm1, h, eps)
    L = lap_matrix(n, h).toarray()
    Lm = mobility_matrix(n, h, phs, mob).toarray()
    I, Z = np.eye(P), np.zeros((P, P))
    u = np.stack([phk.copy(), chemical_potential(phk, h, eps), lap(phk, h)]) if guess is None \
        else np.array(guess, dtype=np.float64)
    for _ in range(maxit):
        r = (S - apply_N_mob(u, phk, phs, h, eps, tau, mob)).ravel()
        D = np.diag((g_cubic_dphi(u[0], phk) + 0.5 * (1.0 - eps)).ravel())
        J = np.block([[I, -tau * Lm, Z], [-D, I, -L], [-0.5 * L, Z, I]])
        du = np.linalg.solve(J, r)
        u = u + du.reshape(3, n, n, n)
        if np.max(np.abs(du)) <= tol * max(1.0, np.max(np.abs(u))):
            break
    return u


def g_cubic(phi, a):
    """Second-order convex treatment of phi^3: 1/4 (phi + a)(phi^2 + a^2)."""
    return 0.25 * (phi + a) * (phi * phi + a * a)


def g_cubic_dphi(phi, a):
    return 0.25 * (3.0 * phi * phi + 2.0 * phi * a + a * a)


def g_cubic_da(phi, a):
    return 0.25 * (phi * phi + 2.0 * phi * a + 3.0 * a * a)


def apply_N(u, phk, h, eps, tau):
    phi, mu, om = u
    return np.stack([
        phi - tau * lap(mu, h),
        mu - g_cubic(phi, phk) - 0.5 * (1.0 - eps) * phi - lap(om, h),
        om - 0.5 * lap(phi, h),
    ])


def source(phk, phkm1, h, eps):
    lk = lap(phk, h)
    return np.stack([phk, 0.5 * (1.0 - eps) * phk + 3.0 * lk - lap(phkm1, h), 0.5 * lk])


def chemical_potential(phi, h, eps):
    """Discrete mu of (equation-PFC): phi^3 + (1-eps) phi + 2 Delta phi + Delta^2 phi."""
    l1 = lap(phi, h)
    return phi ** 3 + (1.0 - eps) * phi + 2.0 * l1 + lap(l1, h)


# --------------------------------------------------------------- energy ---

def grad_norm2(v, h):
    """|grad_h v|_2^2 = h^3 * sum over x, y, z faces of (D v)^2."""
    tot = 0.0
    for axis in range(3):
        d = (np.roll(v, -1, axis) - v) / h
        tot += float(np.sum(d * d))
    return h ** 3 * tot


def energy(phi, h, eps):
    """F_h (PFC energy-discrete-1)."""
    h3 = h ** 3
    return (0.25 * h3 * float(np.sum(phi ** 4)) + 0.5 * (1.0 - eps) * h3 * float(np.sum(phi ** 2))
            - grad_norm2(phi, h) + 0.5 * h3 * float(np.sum(lap(phi, h) ** 2)))


def modified_energy(phi, phi_prev, h, eps):
    """F_h(phi) + 1/2 |grad_h(phi - phi_prev)|^2, the quantity bounded in
    Proposition prop:hu09."""
    return energy(phi, h, eps) + 0.5 * grad_norm2(phi - phi_prev, h)


def mass(phi, h):
    return h ** 3 * float(np.sum(phi))


# ------------------------------------------------ direct step solutions ---

def step_jacobian_dense(u, phk, h, eps, tau):
    """Dense Jacobian dN/du, blocks ordered (phi, mu, omega)."""
    n = phk.shape[0]
    P = n ** 3
    Lm = lap_matrix(n, h).toarray()
    I = np.eye(P)
    D = np.diag((g_cubic_dphi(u[0], phk) + 0.5 * (1.0 - eps)).ravel())
    Z = np.zeros((P, P))
    return np.block([[I, -tau * Lm, Z], [-D, I, -Lm], [-0.5 * Lm, Z, I]])


def solve_step_dense(phkm1, phk, h, eps, tau, guess=None, tol=1e-14, maxit=50):
    """Newton with the dense Jacobian on N(u) = S (n <= 8).  Returns u (3,n,n,n)."""
    n = phk.shape[0]
    S = source(phk, phkm1, h, eps)
    u = np.stack([phk.copy(), chemical_potential(phk, h, eps), lap(phk, h)]) if guess is None \
        else np.array(guess, dtype=np.float64)
    for _ in range(maxit):
        r = (S - apply_N(u, phk, h, eps, tau)).ravel()
        J = step_jacobian_dense(u, phk, h, eps, tau)
        du = np.linalg.solve(J, r)
        u = u + du.reshape(3, n, n, n)
        if np.max(np.abs(du)) <= tol * max(1.0, np.max(np.abs(u))):
            break
    return u


def solve_step_fo_phi(phk, h, eps, tau, tol=1e-14, maxit=50):
    """The first-order convex-splitting step written in phi alone (Section 1:
    convex part of the energy at the new level, concave part at the old one):
    phi - tau Lap(phi^3 + (1-eps) phi + Lap^2 phi) = phk + 2 tau Lap^2 phk,
    by Newton with dense matrices (n <= 12).  Returns (phi, mu, omega) with
    omega = Lap phi and mu = phi^3 + (1-eps) phi + 2 Lap phk + Lap omega."""
    n = phk.shape[0]
    P = n ** 3
    Lm = lap_matrix(n, h).toarray()
    L3 = Lm @ Lm @ Lm
    b = phk.ravel() + 2.0 * tau * (Lm @ (Lm @ phk.ravel()))
    x = phk.ravel().copy()
    for _ in range(maxit):
        G = x - tau * (Lm @ (x ** 3 + (1.0 - eps) * x)) - tau * (L3 @ x) - b
        J = np.eye(P) - tau * Lm * (3.0 * x ** 2 + (1.0 - eps))[None, :] - tau * L3
        dx = np.linalg.solve(J, -G)
        x = x + dx
        if np.max(np.abs(dx)) <= tol * max(1.0, np.max(np.abs(x))):
            break
    phi = x.reshape(n, n, n)
    om = lap(phi, h)
    mu = phi ** 3 + (1.0 - eps) * phi + 2.0 * lap(phk, h) + lap(om, h)
    return np.stack([phi, mu, om])


def fo_linear_factor(lam, eps, tau, pbar=0.0):
    """Amplification of a Fourier mode of -Delta_h-eigenvalue lam about the
    constant state pbar under the linearised first-order scheme:
    (1 + 2 tau lam^2) / (1 + tau lam (3 pbar^2 + 1 - eps + lam^2))."""
    return (1.0 + 2.0 * tau * lam * lam) / (1.0 + tau * lam * (3.0 * pbar * pbar + 1.0 - eps + lam * lam))


def _eliminated_rhs(S, h, tau):
    """phi-equation right-hand side after eliminating omega and mu:
    f1 + tau Delta f2 + tau Delta^2 f3."""
    return S[0] + tau * lap(S[1], h) + tau * lap(lap(S[2], h), h)


def _recover_mu_omega(phi, phk, S, h, eps):
    om = S[2] + 0.5 * lap(phi, h)
    mu = S[1] + g_cubic(phi, phk) + 0.5 * (1.0 - eps) * phi + lap(om, h)
    return mu, om


def _fft_precond(n, L, tau, dbar):
    lam = lap_symbol(n, L)
    sym = 1.0 - tau * lam * dbar - 0.5 * tau * lam ** 3

    def apply(v):
        return np.real(np.fft.ifftn(np.fft.fftn(v.reshape(n, n, n)) / sym)).ravel()
    return apply


def _gmres(matvec, b, prec, rtol, maxiter=400):
    P = b.size
    A = spla.LinearOperator((P, P), matvec=matvec, dtype=np.float64)
    M = spla.LinearOperator((P, P), matvec=prec, dtype=np.float64)
    x, info = spla.gmres(A, b, M=M, rtol=rtol, atol=0.0, restart=200, maxiter=maxiter)
    if info != 0:
        raise RuntimeError(f"GMRES did not converge (info={info})")
    return x


def solve_step_nk(phkm1, phk, h, eps, tau, tol=1e-14, maxit=40):
    """Newton-Krylov on the phi-equation
        phi - tau Delta(g(phi; phk) + (1-eps)/2 phi) - 1/2 tau Delta^3 phi
            = f1 + tau Delta f2 + tau Delta^2 f3,
    then omega and mu from the two linear equations.  Returns u (3,n,n,n)."""
    n = phk.shape[0]
    L = n * h
    S = source(phk, phkm1, h, eps)
    b = _eliminated_rhs(S, h, tau)

    def F(phi):
        return (phi - tau * lap(g_cubic(phi, phk) + 0.5 * (1.0 - eps) * phi, h)
                - 0.5 * tau * lap(lap(lap(phi, h), h), h) - b)

    phi = phk.copy()
    for _ in range(maxit):
        r = F(phi)
        D = g_cubic_dphi(phi, phk) + 0.5 * (1.0 - eps)

        def jv(v, D=D):
            v = v.reshape(n, n, n)
            return (v - tau * lap(D * v, h) - 0.5 * tau * lap(lap(lap(v, h), h), h)).ravel()

        du = _gmres(jv, -r.ravel(), _fft_precond(n, L, tau, float(np.mean(D))), rtol=1e-13)
        phi = phi + du.reshape(n, n, n)
        if np.max(np.abs(du)) <= tol * max(1.0, np.max(np.abs(phi))):
            break
    mu, om = _recover_mu_omega(phi, phk, S, h, eps)
    return np.stack([phi, mu, om])


def simulate_dense(phi0, h, eps, tau, steps, solver="dense"):
    """Exact (direct) time stepping from phi0 with phi^{-1} = phi^0."""
    solve = solve_step_dense if solver == "dense" else solve_step_nk
    phis = [np.array(phi0, dtype=np.float64)]
    mus = []
    prev, cur = phis[0], phis[0]
    for _ in range(steps):
        u = solve(prev, cur, h, eps, tau)
        phis.append(u[0])
        mus.append(u[1])
        prev, cur = cur, u[0]
    return phis, mus


# -------------------------------------------------------------- adjoint ---

def step_partials_dense(phi_next, phk, h, eps):
    """Dense dG/dphk, dG/dphkm1 and dG/deps for G = N(u) - S(phk, phkm1; eps)."""
    n = phk.shape[0]
    P = n ** 3
    Lm = lap_matrix(n, h).toarray()
    I = np.eye(P)
    Z = np.zeros((P, P))
    Ga = np.diag(g_cubic_da(phi_next, phk).ravel())
    dk = np.vstack([-I, -Ga - 0.5 * (1.0 - eps) * I - 3.0 * Lm, -0.5 * Lm])
    dkm1 = np.vstack([Z, Lm, Z])
    de = np.concatenate([np.zeros(P), 0.5 * (phi_next + phk).ravel(), np.zeros(P)])
    return dk, dkm1, de


def adjoint_step_dense(phkm1, phk, u_next, gbar_next, h, eps, tau):
    """Given the cotangent gbar_next of phi^{k+1}, returns the contributions
    (to phi^k, to phi^{k-1}, to eps) through one step solved exactly:
    lambda = J^{-T} (gbar_next, 0, 0), contribution = -(dG/dx)^T lambda."""
    n = phk.shape[0]
    P = n ** 3
    J = step_jacobian_dense(u_next, phk, h, eps, tau)
    rhs = np.concatenate([gbar_next.ravel(), np.zeros(2 * P)])
    lam = np.linalg.solve(J.T, rhs)
    dk, dkm1, de = step_partials_dense(u_next[0], phk, h, eps)
    return (-(dk.T @ lam)).reshape(n, n, n), (-(dkm1.T @ lam)).reshape(n, n, n), float(-de @ lam)


def rollout_loss_grad_dense(phi0, target, h, eps, tau, steps):
    """loss = sum (phi_T - target)^2 through `steps` exactly solved steps from
    phi0 (phi^{-1} = phi^0); returns (loss, dloss/dphi0, dloss/deps)."""
    phis = [np.array(phi0, dtype=np.float64)]
    us = []
    prev, cur = phis[0], phis[0]
    for _ in range(steps):
        u = solve_step_dense(prev, cur, h, eps, tau)
        us.append(u)
        phis.append(u[0])
        prev, cur = cur, u[0]
    loss = float(np.sum((phis[-1] - target) ** 2))
    gb = [np.zeros_like(phi0) for _ in range(steps + 1)]
    gb[steps] = 2.0 * (phis[-1] - target)
    geps = 0.0
    for k in range(steps - 1, -1, -1):
        phk = phis[k]
        phkm1 = phis[k - 1] if k >= 1 else phis[0]
        a, b, e = adjoint_step_dense(phkm1, phk, us[k], gb[k + 1], h, eps, tau)
        gb[k] = gb[k] + a
        if k >= 1:
            gb[k - 1] = gb[k - 1] + b
        else:
            gb[0] = gb[0] + b          # bootstrap: phi^{-1} is phi^0
        geps += e
    return loss, gb[0], geps
