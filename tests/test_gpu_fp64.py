"""Parity of the FP64 HIP path with the CPU oracle, through the C ABI.

Kernel-level cases compare every element; cycle and step cases compare the
full fields after each cycle / time step.  Sizes span several workgroups and
ragged tails (n = 6 and 12 leave partial 256-thread blocks on every level).
"""
import math

import numpy as np
import pytest
import torch

from oracle import cfas
from oracle import definition as D
from paper_1611_06288_amd import inputs

pytestmark = pytest.mark.gpu

KERNEL_RTOL = 1e-13   # one kernel application: a few roundings apart
CYCLE_RTOL = 1e-12    # one multigrid cycle
STEP_RTOL = 1e-11     # converged time step (same algorithm, same cycle count)


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
    return Solver(n, L, eps, dt, **kw)


def rand_state(n, seed, mean=0.285):
    g = inputs.rng(seed)
    phk = mean + 0.1 * g.uniform(-1, 1, (n, n, n))
    u = np.stack([phk + 0.02 * g.uniform(-1, 1, (n, n, n)), g.uniform(-1, 1, (n, n, n)),
                  g.uniform(-1, 1, (n, n, n))])
    f = np.stack([phk, 0.1 * g.uniform(-1, 1, (n, n, n)), 0.1 * g.uniform(-1, 1, (n, n, n))])
    return phk, u, f


# --------------------------------------------------------- kernel level

@pytest.mark.parametrize("n", [6, 12, 48])
def test_source_and_init_guess(n):
    s = make(n)
    g = inputs.rng(n)
    a = 0.3 + 0.1 * g.uniform(-1, 1, (n, n, n))
    b = 0.3 + 0.1 * g.uniform(-1, 1, (n, n, n))
    f = host(s.source(dev(b), dev(a)))
    assert rel(f, cfas.source(a, b, s.h, s.eps)) < KERNEL_RTOL
    mu, om = s.init_guess(dev(a))
    mu_o, om_o = cfas.initial_guess(a, s.h, s.eps)
    assert rel(host(mu), mu_o) < KERNEL_RTOL and rel(host(om), om_o) < KERNEL_RTOL


@pytest.mark.parametrize("n,level", [(12, 0), (12, 1), (48, 0), (48, 2), (96, 0)])
def test_residual_kernel(n, level):
    s = make(n)
    nl = s.levels[level]
    hl = s.L / nl
    phk, u, f = rand_state(nl, 100 + nl)
    r, m = s.residual(level, dev(u), dev(f), dev(phk))
    r_o, m_o = cfas.residual(u, f, phk, hl, s.eps, s.dt)
    assert rel(host(r), r_o) < KERNEL_RTOL
    assert m == pytest.approx(m_o, rel=1e-13)


# Column-tile residual norm (levels with n % 64 == 0; n = 128 cuts columns
# into uneven plane ranges) against the thread-per-point kernel and the oracle.
@pytest.mark.parametrize("n,level", [(128, 0), (192, 0), (256, 0), (256, 1)])
def test_residual_norm_tiles(n, level):
    s = make(n)
    nl = s.levels[level]
    hl = s.L / nl
    phk, u, f = rand_state(nl, 400 + nl)
    ud, fd, pd = dev(u), dev(f), dev(phk)
    _, m_tile = s.residual(level, ud, fd, pd, want_r=False)
    r, m_thread = s.residual(level, ud, fd, pd, want_r=True)
    assert m_tile == m_thread
    if nl <= 128:
        _, m_o = cfas.residual(u, f, phk, hl, s.eps, s.dt)
        assert m_tile == pytest.approx(m_o, rel=1e-13)


@pytest.mark.parametrize("n,level,lin", [(6, 0, "newton"), (12, 0, "newton"), (12, 1, "picard"),
                                         (48, 0, "newton"), (48, 1, "picard"), (96, 0, "newton")])
def test_smoother_half_sweeps(n, level, lin):
    s = make(n, lin=lin)
    nl = s.levels[level]
    hl = s.L / nl
    phk, u, f = rand_state(nl, 200 + nl)
    ud = dev(u)
    ref = u
    for colour in (0, 1, 0):
        s.smooth(level, colour, ud, dev(f), dev(phk))
        ref = cfas.smooth_half(ref, f, phk, hl, s.eps, s.dt, colour, picard=(lin == "picard"))
        assert rel(host(ud), ref) < KERNEL_RTOL


# Full sweeps: levels of >= 128^3 with n % 64 == 0 run the fused one-pass
# sweep (n = 128 and 256 cut each column into uneven plane ranges, n = 192
# into even ones); smaller levels run two half-sweeps (a fused pass there is
# latency-bound: 11-15 us against 3-5 us per half-sweep).  The full sweep
# must equal the GPU's own two half-sweeps bitwise and the oracle's within
# rounding.
@pytest.mark.parametrize("n,lin", [(8, "newton"), (12, "newton"), (16, "picard"), (24, "newton"),
                                   (32, "newton"), (48, "newton"), (64, "picard"), (96, "newton"),
                                   (128, "newton"), (128, "picard"), (192, "newton"),
                                   (256, "newton")])
def test_full_sweep_fused(n, lin):
    from paper_1611_06288_amd._lib import PFC_SWEEP_FULL
    s = make(n, lin=lin)
    phk, u, f = rand_state(n, 300 + n)
    fd, pd = dev(f), dev(phk)
    full, halves = dev(u), dev(u)
    ref = u
    for _ in range(2):
        s.smooth(0, PFC_SWEEP_FULL, full, fd, pd)
        for colour in (0, 1):
            s.smooth(0, colour, halves, fd, pd)
            ref = cfas.smooth_half(ref, f, phk, s.h, s.eps, s.dt, colour, picard=(lin == "picard"))
        torch.cuda.synchronize()
        assert torch.equal(full, halves)
        assert rel(host(full), ref) < KERNEL_RTOL


@pytest.mark.parametrize("n,level", [(12, 0), (48, 0), (48, 1), (96, 0)])
def test_transfers(n, level):
    s = make(n)
    nf, nc = s.levels[level], s.levels[level + 1]
    g = inputs.rng(300 + n + level)
    fine = g.uniform(-1, 1, (3, nf, nf, nf))
    co = host(s.restrict(level, dev(fine), 3))
    assert rel(co, cfas.restrict(fine)) < KERNEL_RTOL
    one = g.uniform(-1, 1, (nf, nf, nf))
    assert rel(host(s.restrict(level, dev(one), 1)), cfas.restrict(one)) < KERNEL_RTOL
    v = g.uniform(-1, 1, (3, nc, nc, nc))
    ub = g.uniform(-1, 1, (3, nc, nc, nc))
    fd = dev(fine)
    s.prolong_add(level, dev(v), dev(ub), fd, 3)
    assert rel(host(fd), cfas.prolong_add(v - ub, fine)) < KERNEL_RTOL
    od = dev(one)
    s.prolong_add(level, dev(v[0]), None, od, 1)
    assert rel(host(od), cfas.prolong_add(v[0], one)) < KERNEL_RTOL


# Interpolation of all three components onto fine levels with n % 64 == 0
# runs the z-marching LDS-tiled kernel (forming v - ubar as it stages the
# coarse planes, or taking v as the error when no ubar is given); one
# component at a time runs the thread-per-pair kernel.  They must agree
# bitwise, and with the oracle.
@pytest.mark.parametrize("n,level", [(64, 0), (128, 0), (192, 0), (256, 0), (256, 1)])
def test_prolong_tiles(n, level):
    s = make(n)
    nf, nc = s.levels[level], s.levels[level + 1]
    g = inputs.rng(500 + n + level)
    fine = g.uniform(-1, 1, (3, nf, nf, nf))
    v = g.uniform(-1, 1, (3, nc, nc, nc))
    ub = g.uniform(-1, 1, (3, nc, nc, nc))
    tiled, tiled_e = dev(fine), dev(fine)
    s.prolong_add(level, dev(v), dev(ub), tiled, 3)
    s.prolong_add(level, dev(v - ub), None, tiled_e, 3)
    direct = [dev(fine[c]) for c in range(3)]
    for c in range(3):
        s.prolong_add(level, dev(v[c]), dev(ub[c]), direct[c], 1)
    torch.cuda.synchronize()
    assert torch.equal(tiled, tiled_e)
    assert torch.equal(tiled, torch.stack(direct))
    assert rel(host(tiled), cfas.prolong_add(v - ub, fine)) < KERNEL_RTOL


@pytest.mark.parametrize("n", [4, 6, 8, 12])
def test_coarsest_newton_solve(n):
    s = make(n, eps=0.25, dt=0.5)
    nc = s.levels[-1]
    hc = s.L / nc
    g = inputs.rng(400 + n)
    phk = 0.285 + 0.1 * g.uniform(-1, 1, (nc, nc, nc))
    u0 = np.stack([phk, g.uniform(-1, 1, (nc, nc, nc)), g.uniform(-1, 1, (nc, nc, nc))])
    f = D.apply_N(u0, phk, hc, s.eps, s.dt) + 0.05 * g.uniform(-1, 1, (3, nc, nc, nc))
    start = np.stack([phk, np.zeros_like(phk), np.zeros_like(phk)])
    ud = dev(start)
    it = s.coarse_solve(ud, dev(f), dev(phk))
    assert 1 <= it < 30
    ref, _ = cfas.coarse_solve(start, f, phk, hc, s.eps, s.dt)
    got = host(ud)
    assert rel(got, ref) < 1e-12
    assert np.max(np.abs(f - D.apply_N(got, phk, hc, s.eps, s.dt))) < 1e-12


@pytest.mark.parametrize("n", [6, 12, 64])
def test_energy(n):
    s = make(n)
    g = inputs.rng(500 + n)
    phi = 0.285 + 0.1 * g.uniform(-1, 1, (n, n, n))
    prev = phi + 0.01 * g.uniform(-1, 1, (n, n, n))
    got = s.energy(dev(phi), dev(prev))
    ref = cfas.energy(phi, s.h, s.eps, prev)
    for a, b in zip(got, ref):
        assert a == pytest.approx(b, rel=1e-12)
    got0 = s.energy(dev(phi))
    assert got0[1] == got0[0]


# ----------------------------------------------------------- cycle level

@pytest.mark.parametrize("n,cycle", [(12, "V"), (32, "V"), (48, "V"), (48, "F"), (64, "V"),
                                     (128, "V"), (192, "F")])
def test_one_cycle_matches_oracle(n, cycle):
    """Levels of 128 and more use the fused red-black sweep (one pass per sweep)."""
    s = make(n, cycle=cycle)
    phk = inputs.polycrystal_phi0(n, s.L, 2, seed=600 + n, radius_cells=4)
    phkm1 = phk + 0.005 * inputs.random_field(n, 601 + n)
    f = cfas.source(phk, phkm1, s.h, s.eps)
    mu, om = cfas.initial_guess(phk, s.h, s.eps)
    u = np.stack([phk, mu, om])
    o = cfas.Solver(n, s.L, s.eps, s.dt, cycle=cycle)
    ud, fd, pd = dev(u), dev(f), dev(phk)
    for _ in range(3):
        res = s.vcycle(ud, fd, pd)
        u, res_o = o.cycle(u, f, phk)
        for c in range(3):
            assert rel(host(ud)[c], u[c]) < CYCLE_RTOL
        assert res == pytest.approx(res_o, rel=1e-9)


@pytest.mark.parametrize("n,nu", [(32, (0, 2)), (32, (1, 1)), (32, (2, 1)), (128, (0, 2)),
                                  (128, (1, 3))])
def test_cycles_with_other_sweep_counts_match_oracle(n, nu):
    """V(nu1, nu2): without pre-sweeps every coarse level takes the tau
    kernel (and its copy of I u) before the coarsest solve; with them the
    coarse levels of half-sweeps form the correction in their first sweep."""
    s = make(n, nu1=nu[0], nu2=nu[1])
    phk = inputs.polycrystal_phi0(n, s.L, 2, seed=650 + n, radius_cells=4)
    phkm1 = phk + 0.005 * inputs.random_field(n, 651 + n)
    f = cfas.source(phk, phkm1, s.h, s.eps)
    mu, om = cfas.initial_guess(phk, s.h, s.eps)
    u = np.stack([phk, mu, om])
    o = cfas.Solver(n, s.L, s.eps, s.dt, nu1=nu[0], nu2=nu[1])
    ud, fd, pd = dev(u), dev(f), dev(phk)
    for _ in range(2):
        res = s.vcycle(ud, fd, pd)
        u, res_o = o.cycle(u, f, phk)
        for c in range(3):
            assert rel(host(ud)[c], u[c]) < CYCLE_RTOL
        assert res == pytest.approx(res_o, rel=1e-9)


# ------------------------------------------------------------ step level

def run_both(n, L, eps, dt, phi0, steps, tol=1e-10, **kw):
    s = make(n, L=L, eps=eps, dt=dt, tol=tol, **kw)
    o_phis, o_infos, _ = cfas.simulate(phi0, L, eps, dt, steps, tol=tol,
                                       cycle=kw.get("cycle", "V"), lin=kw.get("lin", "newton"))
    g_phis, g_infos = [], []
    s.simulate(dev(phi0), steps, callback=lambda k, p, mu, om, info: (g_phis.append(host(p)),
                                                                      g_infos.append(info)))
    return o_phis, o_infos, g_phis, g_infos


def test_smooth_mode_32_every_step():
    """32^3, L = 32, eps = 0.025, s = 0.01, 10 steps, V(2,2), tol 1e-10."""
    p = inputs.smooth_mode_params()
    phi0 = inputs.smooth_mode_phi0()
    o_phis, o_infos, g_phis, g_infos = run_both(p.n, p.L, p.eps, p.dt, phi0, p.steps, tol=p.tol)
    for k in range(p.steps):
        assert g_infos[k].status == 0
        assert g_infos[k].cycles == o_infos[k].cycles, (k, g_infos[k], o_infos[k].cycles)
        assert rel(g_phis[k], o_phis[k + 1]) < STEP_RTOL, k


@pytest.mark.parametrize("n,cycle,lin", [(24, "V", "newton"), (24, "F", "newton"), (16, "V", "picard")])
def test_polycrystal_small_steps(n, cycle, lin):
    L = n * math.pi / 4
    phi0 = inputs.polycrystal_phi0(n, L, 2, seed=700 + n, radius_cells=4)
    o_phis, o_infos, g_phis, g_infos = run_both(n, L, 0.25, 0.5, phi0, 3, cycle=cycle, lin=lin)
    for k in range(3):
        assert g_infos[k].cycles == o_infos[k].cycles
        assert rel(g_phis[k], o_phis[k + 1]) < STEP_RTOL


def test_constant_state_zero_cycles_bitwise():
    s = make(16)
    phi = torch.full((16, 16, 16), 0.285, dtype=torch.float64, device="cuda")
    mu, om = s.init_guess(phi)
    out, info = s.step(phi, phi, mu, om)
    assert info.cycles == 0
    assert torch.equal(out, phi)


def test_single_level_grid_n4():
    """n = 4 is its own coarsest level: each cycle is an exact Newton solve."""
    n, L = 4, 4.0
    phi0 = 0.2 + 0.05 * inputs.random_field(n, 9)
    o_phis, o_infos, g_phis, g_infos = run_both(n, L, 0.1, 0.1, phi0, 2, tol=1e-12)
    for k in range(2):
        assert g_infos[k].cycles == o_infos[k].cycles <= 2
        assert rel(g_phis[k], o_phis[k + 1]) < STEP_RTOL


def test_deterministic_bitwise():
    n = 32
    L = n * math.pi / 4
    phi0 = dev(inputs.polycrystal_phi0(n, L, 2, seed=5, radius_cells=4))
    outs = []
    for _ in range(2):
        s = make(n)
        _, cur, mu, om, infos = s.simulate(phi0, 2)
        outs.append((cur.clone(), mu.clone(), [i.cycles for i in infos], s.energy(cur)))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2] and outs[0][3] == outs[1][3]


def test_error_statuses():
    from paper_1611_06288_amd.solver import PFCError
    s = make(16, tol=1e-30, max_cycles=1)
    phi = dev(inputs.polycrystal_phi0(16, s.L, 1, seed=1, radius_cells=3))
    mu, om = s.init_guess(phi)
    out, info = s.step(phi, phi, mu, om, raise_on_error=False)
    assert info.status == 2 and info.cycles == 1
    bad = phi.clone()
    bad[3, 4, 5] = float("nan")
    s2 = make(16)
    mu2, om2 = s2.init_guess(phi)
    with pytest.raises(PFCError) as e:
        s2.step(bad, bad, mu2, om2)
    assert e.value.status == 3
    with pytest.raises(PFCError):
        s2.step(phi, phi, mu2, om2, out=phi)   # aliasing
    with pytest.raises(PFCError):
        make(10)
    with pytest.raises(ValueError):
        s2.step(phi[:8].contiguous(), phi, mu2, om2)


# --------------------------------------------- full-size workload checks

def test_polycrystal_128_first_steps():
    """128^3 polycrystal (3 crystallites, h = pi/4, eps = 0.25, s = 0.5):
    the first two steps against the oracle, element by element."""
    n = 128
    p = inputs.polycrystal_params(n)
    phi0 = inputs.polycrystal_128()
    o_phis, o_infos, g_phis, g_infos = run_both(n, p.L, p.eps, p.dt, phi0, 2, tol=p.tol)
    for k in range(2):
        assert g_infos[k].cycles == o_infos[k].cycles
        assert rel(g_phis[k], o_phis[k + 1]) < STEP_RTOL


def test_polycrystal_256_cycle_and_invariants():
    """256^3 (8 crystallites): one V-cycle element by element against the
    oracle, then a full GPU step checked through size-independent properties:
    mass drift bounded by the tolerance and the modified-energy identity."""
    n = 256
    p = inputs.polycrystal_params(n)
    phi0 = inputs.polycrystal_256()
    s = make(n, L=p.L, eps=p.eps, dt=p.dt, tol=p.tol)
    f = cfas.source(phi0, phi0, s.h, s.eps)
    mu, om = cfas.initial_guess(phi0, s.h, s.eps)
    u = np.stack([phi0, mu, om])
    ud = dev(u)
    s.vcycle(ud, dev(f), dev(phi0))
    o = cfas.Solver(n, p.L, p.eps, p.dt)
    u1, _ = o.cycle(u, f, phi0)
    assert rel(host(ud), u1) < CYCLE_RTOL
    del u1, ud
    pd = dev(phi0)
    mud, omd = s.init_guess(pd)
    nxt, info = s.step(pd, pd, mud, omd)
    assert info.status == 0
    m0, m1 = s.energy(pd)[2], s.energy(nxt)[2]
    assert abs(m1 - m0) <= s.h ** 3 * n ** 3 * p.tol
    Fa = s.energy(nxt, pd)[1]
    Fb = s.energy(pd, pd)[1]
    gm = D.grad_norm2(host(mud), s.h)
    second = D.grad_norm2(host(nxt) - host(pd), s.h)
    defect = Fa - Fb + s.dt * gm + 0.5 * second
    assert abs(defect) < 1e-6 * abs(Fa)
