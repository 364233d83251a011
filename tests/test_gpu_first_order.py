"""Parity of the first-order convex-splitting scheme on the HIP path with the
oracle, through the C ABI (same kernels as scheme (1.10), OpParams::fo set).

Kernel-level cases compare every element, cycles and steps the full fields;
at sizes the oracle does not reach, the scheme's own guarantees are checked
(F_h non-increasing at any time step, mass within the residual bound, the
graph-driven loop equal to the step loop).
"""
import math

import numpy as np
import pytest
import torch

from oracle import cfas
from paper_1611_06288_amd import inputs

pytestmark = pytest.mark.gpu

KERNEL_RTOL = 1e-13
CYCLE_RTOL = 1e-12
STEP_RTOL = 1e-11


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def make(n, L=None, eps=0.25, dt=0.5, **kw):
    from paper_1611_06288_amd import Solver
    L = n * math.pi / 4 if L is None else L
    return Solver(n, L, eps, dt, scheme=1, **kw)


def rand_state(n, seed, mean=0.285):
    g = inputs.rng(seed)
    phk = mean + 0.1 * g.uniform(-1, 1, (n, n, n))
    u = np.stack([phk + 0.02 * g.uniform(-1, 1, (n, n, n)), g.uniform(-1, 1, (n, n, n)),
                  g.uniform(-1, 1, (n, n, n))])
    f = np.stack([phk, 0.1 * g.uniform(-1, 1, (n, n, n)), 0.1 * g.uniform(-1, 1, (n, n, n))])
    return phk, u, f


@pytest.mark.parametrize("n", [6, 48])
def test_source(n):
    s = make(n)
    g = inputs.rng(3000 + n)
    a = 0.3 + 0.1 * g.uniform(-1, 1, (n, n, n))
    b = 0.3 + 0.1 * g.uniform(-1, 1, (n, n, n))
    f = host(s.source(dev(b), dev(a)))
    ref = cfas.source_fo(a, s.h)
    assert rel(f[:2], ref[:2]) < KERNEL_RTOL and np.all(f[2] == 0.0)


@pytest.mark.parametrize("n,level", [(12, 0), (12, 2), (48, 1), (128, 0), (256, 0)])
def test_residual_kernels(n, level):
    """Thread-per-point residual (r returned) and, on levels with n % 64 == 0,
    the column-tile norm of the stop test."""
    s = make(n)
    nl = s.levels[level]
    phk, u, f = rand_state(nl, 3100 + nl)
    r, m = s.residual(level, dev(u), dev(f), dev(phk))
    r_o, m_o = cfas.residual_fo(u, f, s.L / nl, s.eps, s.dt)
    assert rel(host(r), r_o) < KERNEL_RTOL
    assert m == pytest.approx(m_o, rel=1e-13)
    _, m2 = s.residual(level, dev(u), dev(f), dev(phk), want_r=False)
    assert m2 == m


@pytest.mark.parametrize("n,level,lin", [(6, 0, "newton"), (12, 1, "picard"), (48, 0, "newton"),
                                         (48, 1, "picard")])
def test_smoother_half_sweeps(n, level, lin):
    s = make(n, lin=lin)
    nl = s.levels[level]
    phk, u, f = rand_state(nl, 3200 + nl)
    ud = dev(u)
    ref = u
    for colour in (0, 1, 0):
        s.smooth(level, colour, ud, dev(f), dev(phk))
        ref = cfas.smooth_half_fo(ref, f, s.L / nl, s.eps, s.dt, colour, picard=(lin == "picard"))
        assert rel(host(ud), ref) < KERNEL_RTOL


@pytest.mark.parametrize("n,lin", [(16, "newton"), (32, "picard"), (128, "newton"),
                                   (128, "picard"), (256, "newton")])
def test_fused_sweep(n, lin):
    from paper_1611_06288_amd._lib import PFC_SWEEP_FULL
    s = make(n, lin=lin)
    phk, u, f = rand_state(n, 3300 + n)
    fd, pd = dev(f), dev(phk)
    full, halves = dev(u), dev(u)
    s.smooth(0, PFC_SWEEP_FULL, full, fd, pd)
    for colour in (0, 1):
        s.smooth(0, colour, halves, fd, pd)
    torch.cuda.synchronize()
    assert torch.equal(full, halves)
    ref = u
    for colour in (0, 1):
        ref = cfas.smooth_half_fo(ref, f, s.h, s.eps, s.dt, colour, picard=(lin == "picard"))
    assert rel(host(full), ref) < KERNEL_RTOL


@pytest.mark.parametrize("n", [4, 6, 12])
def test_coarsest_newton_solve(n):
    s = make(n)
    nc = s.levels[-1]
    hc = s.L / nc
    g = inputs.rng(3400 + n)
    u0 = np.stack([0.285 + 0.1 * g.uniform(-1, 1, (nc, nc, nc)), g.uniform(-1, 1, (nc, nc, nc)),
                   g.uniform(-1, 1, (nc, nc, nc))])
    f = cfas.apply_N_fo(u0, hc, s.eps, s.dt) + 0.05 * g.uniform(-1, 1, (3, nc, nc, nc))
    start = np.stack([u0[0], np.zeros_like(u0[0]), np.zeros_like(u0[0])])
    ud = dev(start)
    it = s.coarse_solve(ud, dev(f), dev(u0[0]))
    assert 1 <= it < 30
    ref, _ = cfas.coarse_solve_fo(start, f, hc, s.eps, s.dt)
    got = host(ud)
    assert rel(got, ref) < 1e-12
    assert np.max(np.abs(f - cfas.apply_N_fo(got, hc, s.eps, s.dt))) < 1e-11


@pytest.mark.parametrize("n,cycle", [(12, "V"), (32, "V"), (48, "F"), (128, "V")])
def test_one_cycle_matches_oracle(n, cycle):
    s = make(n, cycle=cycle)
    phk = inputs.polycrystal_phi0(n, s.L, 2, seed=3500 + n, radius_cells=4)
    f = cfas.source_fo(phk, s.h)
    mu, om = cfas.initial_guess(phk, s.h, s.eps)
    u = np.stack([phk, mu, om])
    o = cfas.Solver(n, s.L, s.eps, s.dt, cycle=cycle, scheme=1)
    ud, fd, pd = dev(u), dev(f), dev(phk)
    for _ in range(3):
        res = s.vcycle(ud, fd, pd)
        u, res_o = o.cycle(u, f, phk)
        for c in range(3):
            assert rel(host(ud)[c], u[c]) < CYCLE_RTOL
        assert res == pytest.approx(res_o, rel=1e-9)


@pytest.mark.parametrize("n,cycle,lin", [(16, "V", "newton"), (24, "F", "newton"), (16, "V", "picard"),
                                         (32, "V", "newton")])
def test_polycrystal_steps_match_oracle(n, cycle, lin):
    L = n * math.pi / 4
    phi0 = inputs.polycrystal_phi0(n, L, 2, seed=3600 + n, radius_cells=4)
    o_phis, o_infos, _ = cfas.simulate(phi0, L, 0.25, 0.5, 3, tol=1e-10, cycle=cycle, lin=lin,
                                       scheme=1)
    s = make(n, L=L, tol=1e-10, cycle=cycle, lin=lin)
    g_phis, g_infos = [], []
    s.simulate(dev(phi0), 3, callback=lambda k, p, mu, om, info: (g_phis.append(host(p)),
                                                                  g_infos.append(info)))
    for k in range(3):
        assert g_infos[k].status == 0
        assert g_infos[k].cycles == o_infos[k].cycles, (k, g_infos[k], o_infos[k].cycles)
        assert rel(g_phis[k], o_phis[k + 1]) < STEP_RTOL


def test_energy_decreases_at_large_time_step_128():
    """Convex splitting: F_h(phi^{k+1}) <= F_h(phi^k) whatever tau (here 4x the
    polycrystal benchmark's step), mass within the residual bound; and the
    graph-driven loop reproduces the step loop bit for bit."""
    n = 128
    p = inputs.polycrystal_params(n)
    s = make(n, L=p.L, eps=p.eps, dt=4 * p.dt, tol=1e-9, cycle="F", max_cycles=500)
    phi0 = dev(inputs.polycrystal_phi0(n, p.L, 4, seed=3700))
    mu, om = s.init_guess(phi0)
    prev, cur = phi0.clone(), phi0.clone()
    E = [s.energy(phi0)[0]]
    mass0 = s.energy(phi0)[2]
    bound = 1e-12 * abs(mass0)
    for _ in range(4):
        infos = s.run(prev, cur, mu, om, 1)
        assert infos[0].status == 0
        bound += s.h ** 3 * n ** 3 * infos[0].res_final
        e = s.energy(cur)
        E.append(e[0])
        assert abs(e[2] - mass0) <= bound
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(E, E[1:])), E
    # loop vs step loop
    t = make(n, L=p.L, eps=p.eps, dt=4 * p.dt, tol=1e-9, cycle="F", max_cycles=500)
    mu2, om2 = t.init_guess(phi0)
    prv, cu = phi0.clone(), phi0.clone()
    spare = torch.empty_like(cu)
    for _ in range(4):
        nxt, _ = t.step(prv, cu, mu2, om2, out=spare)
        spare, prv, cu = prv, cu, nxt
    torch.cuda.synchronize()
    assert torch.equal(cu, cur) and torch.equal(mu2, mu)


def test_refused_combinations():
    from paper_1611_06288_amd import Solver
    from paper_1611_06288_amd.solver import PFCError
    with pytest.raises(PFCError):
        Solver(16, 4 * math.pi, 0.25, 0.5, scheme=1, precision="mixed")
    with pytest.raises(PFCError):
        Solver(16, 4 * math.pi, 0.25, 0.5, scheme=1, mobility=(1.0, 0.0, -1.0, 0.05))
    s = make(16)
    phi = dev(inputs.polycrystal_phi0(16, s.L, 1, seed=3800, radius_cells=3))
    g = torch.zeros_like(phi)
    with pytest.raises(PFCError):
        s.adjoint_step(phi, phi, phi, g, g.clone(), g.clone(),
                       torch.zeros(1, dtype=torch.float64, device=phi.device))
