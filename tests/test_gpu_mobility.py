"""Parity of the variable-mobility HIP path with the CPU oracle, through the C ABI.

The first equation in flux form, phi - tau d(M(A phi*) D mu) = S1, with the
face mobility M(v) = max(mmin, m0 + m1 v + m2 v^2) at the face average of
phi* = 3/2 phi^k - 1/2 phi^{k-1} (Section 5 allows a variable mobility; its
form is this code's reading).  Kernel-level cases compare every element,
cycle and step cases the full fields; larger grids check what holds at any
size (constant M = c equals M = 1 with time step c tau; mass; energy decay).
"""
import ctypes
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

MOB = (1.0, 0.0, -1.0, 0.05)     # M(v) = max(0.05, 1 - v^2)
MOB_LIN = (0.8, 0.9, 0.0, 0.1)   # M(v) = max(0.1, 0.8 + 0.9 v)
MOB_STRONG = (-0.14, 4.0, 0.0, 0.05)  # 0.5 .. 1.5 over the polycrystal's phi range


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def make(n, mob=MOB, L=None, eps=0.25, dt=0.5, **kw):
    from paper_1611_06288_amd import Solver
    L = n * math.pi / 4 if L is None else L
    return Solver(n, L, eps, dt, mobility=mob, **kw)


def rand_state(n, seed, mean=0.285):
    """phi^k, an iterate, a right-hand side and phi* with M varying by O(1)
    (phi* in [-0.8, 1.2]: some faces reach the floor mmin)."""
    g = inputs.rng(seed)
    phk = mean + 0.1 * g.uniform(-1, 1, (n, n, n))
    u = np.stack([phk + 0.02 * g.uniform(-1, 1, (n, n, n)), g.uniform(-1, 1, (n, n, n)),
                  g.uniform(-1, 1, (n, n, n))])
    f = np.stack([phk, 0.1 * g.uniform(-1, 1, (n, n, n)), 0.1 * g.uniform(-1, 1, (n, n, n))])
    phs = g.uniform(-1, 1, (n, n, n)) + 0.2
    return phk, u, f, phs


# --------------------------------------------------------- kernel level

@pytest.mark.parametrize("n,level,mob", [(12, 0, MOB), (12, 1, MOB_LIN), (12, 2, MOB),
                                         (48, 0, MOB_LIN), (48, 2, MOB), (96, 0, MOB),
                                         (128, 0, MOB_LIN), (256, 0, MOB)])
def test_residual_kernel(n, level, mob):
    """Thread-per-point residual against the oracle; on levels with n % 64 == 0
    the norm-only call runs the column-tile kernel with its phi* ring, which
    must give the same maximum bit for bit."""
    s = make(n, mob)
    nl = s.levels[level]
    hl = s.L / nl
    phk, u, f, phs = rand_state(nl, 1100 + nl)
    s.set_phistar(level, dev(phs))
    r, m = s.residual(level, dev(u), dev(f), dev(phk))
    r_o, m_o = cfas.residual_m(u, f, phk, phs, hl, s.eps, s.dt, mob)
    assert rel(host(r), r_o) < KERNEL_RTOL
    assert m == pytest.approx(m_o, rel=1e-13)
    # the norm-only call (the stop test's kernel) gives the same maximum
    _, m2 = s.residual(level, dev(u), dev(f), dev(phk), want_r=False)
    assert m2 == m


def test_phistar_hierarchy_is_eight_child_means():
    """phi* set at level 0 reaches level 1 as 8-child means (seen through the
    level-1 residual, which depends on phi* only through M)."""
    s = make(24, MOB_LIN)
    phk, u, f, phs = rand_state(24, 1201)
    s.set_phistar(0, dev(phs))
    n1 = s.levels[1]
    phk1, u1, f1, _ = rand_state(n1, 1202)
    phs1 = cfas.restrict(phs)
    r, _ = s.residual(1, dev(u1), dev(f1), dev(phk1))
    r_o, _ = cfas.residual_m(u1, f1, phk1, phs1, s.L / n1, s.eps, s.dt, MOB_LIN)
    assert rel(host(r), r_o) < KERNEL_RTOL


@pytest.mark.parametrize("n,level,lin,mob", [(6, 0, "newton", MOB), (12, 0, "newton", MOB_LIN),
                                             (12, 1, "picard", MOB), (48, 0, "newton", MOB),
                                             (48, 1, "picard", MOB_LIN)])
def test_smoother_half_sweeps(n, level, lin, mob):
    s = make(n, mob, lin=lin)
    nl = s.levels[level]
    hl = s.L / nl
    phk, u, f, phs = rand_state(nl, 1300 + nl)
    s.set_phistar(level, dev(phs))
    ud = dev(u)
    ref = u
    for colour in (0, 1, 0):
        s.smooth(level, colour, ud, dev(f), dev(phk))
        ref = cfas.smooth_half_m(ref, f, phk, phs, hl, s.eps, s.dt, colour, mob,
                                 picard=(lin == "picard"))
        assert rel(host(ud), ref) < KERNEL_RTOL


@pytest.mark.parametrize("n,lin", [(16, "newton"), (48, "picard"), (128, "newton"),
                                   (128, "picard"), (256, "newton")])
def test_fused_sweep_equals_two_half_sweeps(n, lin):
    """Levels of >= 128^3 with n % 64 == 0 run the fused one-pass sweep with the
    phi* ring (smaller ones two half-sweeps); the full sweep must equal two
    half-sweeps bit for bit, and the oracle."""
    from paper_1611_06288_amd._lib import PFC_SWEEP_FULL
    s = make(n, MOB, lin=lin)
    phk, u, f, phs = rand_state(n, 1400 + n)
    s.set_phistar(0, dev(phs))
    fd, pd = dev(f), dev(phk)
    full, halves = dev(u), dev(u)
    s.smooth(0, PFC_SWEEP_FULL, full, fd, pd)
    for colour in (0, 1):
        s.smooth(0, colour, halves, fd, pd)
    torch.cuda.synchronize()
    assert torch.equal(full, halves)
    ref = u
    for colour in (0, 1):
        ref = cfas.smooth_half_m(ref, f, phk, phs, s.h, s.eps, s.dt, colour, MOB,
                                 picard=(lin == "picard"))
    assert rel(host(full), ref) < KERNEL_RTOL


@pytest.mark.parametrize("n,mob", [(4, MOB), (6, MOB_LIN), (8, MOB), (12, MOB_LIN)])
def test_coarsest_newton_solve(n, mob):
    s = make(n, mob)
    nc = s.levels[-1]
    hc = s.L / nc
    g = inputs.rng(1500 + n)
    phk = 0.285 + 0.1 * g.uniform(-1, 1, (nc, nc, nc))
    phs = 0.2 + g.uniform(-1, 1, (nc, nc, nc))
    u0 = np.stack([phk, g.uniform(-1, 1, (nc, nc, nc)), g.uniform(-1, 1, (nc, nc, nc))])
    f = cfas.apply_N_m(u0, phk, phs, hc, s.eps, s.dt, mob) + 0.05 * g.uniform(-1, 1, (3, nc, nc, nc))
    start = np.stack([phk, np.zeros_like(phk), np.zeros_like(phk)])
    s.set_phistar(len(s.levels) - 1, dev(phs))
    ud = dev(start)
    it = s.coarse_solve(ud, dev(f), dev(phk))
    assert 1 <= it < 30
    ref, _ = cfas.coarse_solve_m(start, f, phk, phs, hc, s.eps, s.dt, mob)
    got = host(ud)
    assert rel(got, ref) < 1e-12
    assert np.max(np.abs(f - cfas.apply_N_m(got, phk, phs, hc, s.eps, s.dt, mob))) < 1e-11


# ----------------------------------------------------------- cycle level

@pytest.mark.parametrize("n,cycle,mob", [(12, "V", MOB), (32, "V", MOB_LIN), (48, "F", MOB),
                                         (64, "V", MOB), (128, "V", MOB_LIN)])
def test_one_cycle_matches_oracle(n, cycle, mob):
    s = make(n, mob, cycle=cycle)
    phk = inputs.polycrystal_phi0(n, s.L, 2, seed=1600 + n, radius_cells=4)
    phkm1 = phk + 0.005 * inputs.random_field(n, 1601 + n)
    phs = 1.5 * phk - 0.5 * phkm1
    f = cfas.source(phk, phkm1, s.h, s.eps)
    mu, om = cfas.initial_guess(phk, s.h, s.eps)
    u = np.stack([phk, mu, om])
    o = cfas.Solver(n, s.L, s.eps, s.dt, cycle=cycle, mobility=mob)
    s.set_phistar(0, dev(phs))
    ud, fd, pd = dev(u), dev(f), dev(phk)
    for _ in range(3):
        res = s.vcycle(ud, fd, pd)
        u, res_o = o.cycle(u, f, phk, phs)
        for c in range(3):
            assert rel(host(ud)[c], u[c]) < CYCLE_RTOL
        assert res == pytest.approx(res_o, rel=1e-9)


# ------------------------------------------------------------ step level

def run_both(n, L, eps, dt, phi0, steps, mob, tol=1e-10, **kw):
    s = make(n, mob, L=L, eps=eps, dt=dt, tol=tol, **kw)
    o_phis, o_infos, _ = cfas.simulate(phi0, L, eps, dt, steps, tol=tol, cycle=kw.get("cycle", "V"),
                                       lin=kw.get("lin", "newton"), mobility=mob)
    g_phis, g_infos = [], []
    s.simulate(dev(phi0), steps, callback=lambda k, p, mu, om, info: (g_phis.append(host(p)),
                                                                      g_infos.append(info)))
    return o_phis, o_infos, g_phis, g_infos


@pytest.mark.parametrize("n,cycle,lin,mob", [(16, "V", "newton", MOB), (24, "F", "newton", MOB_LIN),
                                             (16, "V", "picard", MOB_LIN), (32, "V", "newton", MOB)])
def test_polycrystal_steps_match_oracle(n, cycle, lin, mob):
    L = n * math.pi / 4
    phi0 = inputs.polycrystal_phi0(n, L, 2, seed=1700 + n, radius_cells=4)
    o_phis, o_infos, g_phis, g_infos = run_both(n, L, 0.25, 0.5, phi0, 3, mob, cycle=cycle, lin=lin)
    for k in range(3):
        assert g_infos[k].status == 0
        assert g_infos[k].cycles == o_infos[k].cycles, (k, g_infos[k], o_infos[k].cycles)
        assert rel(g_phis[k], o_phis[k + 1]) < STEP_RTOL, k


def test_constant_mobility_is_a_rescaled_time_step_at_64():
    """M = c makes the first equation phi - (c tau) Lap mu = S1: the variable-
    mobility kernels must reproduce the M = 1 kernels run with time step c tau."""
    from paper_1611_06288_amd import Solver
    n, c = 64, 0.7
    L = n * math.pi / 4
    phi0 = dev(inputs.polycrystal_phi0(n, L, 3, seed=1800, radius_cells=6))
    a = Solver(n, L, 0.25, 0.5, tol=1e-12, mobility=(c, 0.0, 0.0, 0.01))
    b = Solver(n, L, 0.25, c * 0.5, tol=1e-12)
    _, pa, _, _, ia = a.simulate(phi0, 3)
    _, pb, _, _, ib = b.simulate(phi0, 3)
    assert all(i.status == 0 for i in ia + ib)
    assert rel(host(pa), host(pb)) < 1e-10


def test_mass_and_energy_at_128():
    """Flux form: the fluxes telescope, so the mass changes only by the sum of
    the first equation's residual (|dm| <= h^3 n^3 max|r| per step); the
    modified energy does not grow (M > 0); M varies by O(1) over the grains."""
    n = 128
    p = inputs.polycrystal_params(n)
    from paper_1611_06288_amd import Solver
    s = Solver(n, p.L, p.eps, p.dt, tol=1e-9, mobility=MOB_STRONG, cycle="F")
    phi0 = dev(inputs.polycrystal_phi0(n, p.L, 4, seed=1900))
    mass0 = s.energy(phi0)[2]
    E = []
    phis = []
    bound = [1e-12 * abs(mass0)]

    def cb(k, nxt, mu, om, info):
        assert info.status == 0
        phis.append(nxt.clone())
        E.append(s.energy(nxt, phis[-2] if len(phis) > 1 else phi0)[1])
        bound[0] += s.h ** 3 * n ** 3 * info.res_final
        assert abs(s.energy(nxt)[2] - mass0) <= bound[0], (k, bound[0])

    s.simulate(phi0, 4, callback=cb)
    assert all(E[k + 1] <= E[k] + 1e-9 * abs(E[k]) for k in range(len(E) - 1)), E
    phs = 1.5 * host(phis[-1]) - 0.5 * host(phis[-2])
    m = np.clip(MOB_STRONG[0] + MOB_STRONG[1] * phs, MOB_STRONG[3], None)
    assert m.max() - m.min() > 0.5


# ------------------------------------------------------------ errors

def test_error_cases():
    from paper_1611_06288_amd import Solver, _lib
    from paper_1611_06288_amd.solver import PFCError
    n = 16
    L = n * math.pi / 4
    phi = dev(inputs.polycrystal_phi0(n, L, 1, seed=2000, radius_cells=3))
    u3 = dev(np.zeros((3, n, n, n)))
    # phi* must be set before a kernel-level call on a variable-mobility handle
    s = make(n, MOB)
    with pytest.raises(PFCError) as e:
        s.residual(0, u3, u3, phi)
    assert e.value.status == _lib.PFC_ERR_INVALID_ARG
    with pytest.raises(PFCError):
        s.vcycle(u3.clone(), u3, phi)
    # pfc_set_phistar on a constant-mobility handle
    with pytest.raises(PFCError):
        Solver(n, L, 0.25, 0.5).set_phistar(0, phi)
    # the mixed-precision, adjoint and batched forms are M = 1 only
    with pytest.raises(PFCError):
        Solver(n, L, 0.25, 0.5, precision="mixed", mobility=MOB)
    g = torch.zeros_like(phi)
    with pytest.raises(PFCError):
        s.adjoint_step(phi, phi, phi, g, g.clone(), g.clone(), torch.zeros(1, dtype=torch.float64,
                                                                           device=phi.device))
    cfg = s.cfg
    out = ctypes.c_void_p()
    lib = _lib.lib()
    assert lib.pfc_batch_create(1, ctypes.byref(cfg), None, ctypes.byref(out)) == \
        _lib.PFC_ERR_INVALID_ARG
    # a step still works after the refused calls, and sets phi* itself
    mu, om = s.init_guess(phi)
    _, info = s.step(phi, phi, mu, om)
    assert info.status == 0
    r, _ = s.residual(0, dev(np.zeros((3, n, n, n))), dev(np.zeros((3, n, n, n))), phi)
