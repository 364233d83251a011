"""The cycle loop's stop test split over the finest level's fused sweeps
(FP64, M = 1 or variable mobility, finest level of at least 128^3 with
n % 64 == 0).

The residual max-norm after a cycle is assembled from two halves: the
colour-1 points, whose residual the cycle's last post-sweep forms from the
values it has just written, and the colour-0 points, whose residual the next
cycle's first pre-sweep forms from its input while it smooths.  That sweep
runs before the loop's decision and its output is dropped when the loop
stops.  Everything here is compared with a host loop of single cycles
(pfc_fas_vcycle) and whole-level norms (pfc_residual), which never splits:
fields, cycle counts and both reported norms bit for bit, for V and F
cycles, several sweep counts, NOT_CONVERGED at small max_cycles and the
graph-driven loop; the launch counts show that the split path ran.

The same comparison at finest levels below those sizes (half-sweeps, no
split) checks that the step's kernels, which take the first source
component from phi^k itself (one buffer, loaded once), give bit for bit
what the host loop's kernels give with a separate copy of it.
"""
import math

import numpy as np
import pytest
import torch

from paper_1611_06288_amd import inputs
from paper_1611_06288_amd._lib import (PFC_KERNEL_NORM0, PFC_KERNEL_SMOOTH0,
                                       PFC_KERNEL_SWEEP_NORM0)

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def make(n, L, eps, dt, **kw):
    from paper_1611_06288_amd import Solver
    return Solver(n, L, eps, dt, **kw)


MOB = (1.0, 0.0, -1.0, 0.05)  # M(v) = max(0.05, 1 - v^2)


def host_loop(s, phi_prev, phi_cur, mu, om, tol, max_cycles, mobility=None):
    """The cycle loop of one step with a whole-level norm before each cycle."""
    if mobility is not None:  # phi* of this step, as the step computes it
        s.set_phistar(0, 1.5 * phi_cur - 0.5 * phi_prev)
    f = s.source(phi_prev, phi_cur)
    u = torch.stack([phi_cur, mu, om]).contiguous()
    _, r = s.residual(0, u, f, phi_cur, want_r=False)
    res0, c, status = r, 0, 0
    while True:
        if not math.isfinite(r):
            status = 3
            break
        if r <= tol:
            break
        if c == max_cycles:
            status = 2
            break
        r = s.vcycle(u, f, phi_cur)
        c += 1
    return u, c, status, res0, r


def workload(n, seed):
    p = inputs.polycrystal_params(n)
    phi0 = inputs.polycrystal_phi0(n, p.L, 3, seed=seed)
    return p, dev(phi0)


def check_step(n, seed, tol, max_cycles, **kw):
    p, phi = workload(n, seed)
    s = make(n, p.L, p.eps, p.dt, tol=tol, max_cycles=max_cycles, **kw)
    ref = make(n, p.L, p.eps, p.dt, tol=tol, max_cycles=max_cycles, **kw)
    mu, om = s.init_guess(phi)
    mu_r, om_r = mu.clone(), om.clone()
    # the state one step in, so that phi_prev != phi_cur; the reference handle
    # takes the same step, so both carry the same coarsest-level inverse
    cur, info = s.step(phi, phi, mu, om, raise_on_error=False)
    assert info.status in (0, 2)
    cur_r, _ = ref.step(phi, phi, mu_r, om_r, raise_on_error=False)
    torch.cuda.synchronize()
    assert torch.equal(cur, cur_r)
    prev = phi
    mu_h, om_h = mu.clone(), om.clone()
    if kw.get("mobility") is not None:
        # the host loop's pfc_set_phistar clears the coarsest level's cached
        # Newton inverse, which a step carries over: start both afresh
        s.reset_coarse_cache()
    s.timing(True)
    s.timing_reset()
    nxt, info = s.step(prev, cur, mu, om, raise_on_error=False)
    counts = {k: s.timing_get(k)[0] for k in (PFC_KERNEL_SMOOTH0, PFC_KERNEL_SWEEP_NORM0,
                                               PFC_KERNEL_NORM0)}
    s.timing(False)
    u, c, status, res0, res = host_loop(ref, prev, cur, mu_h, om_h, tol, max_cycles,
                                        kw.get("mobility"))
    torch.cuda.synchronize()
    assert (info.cycles, info.status) == (c, status)
    assert info.res0 == res0 and info.res_final == res
    assert torch.equal(nxt, u[0]) and torch.equal(mu, u[1]) and torch.equal(om, u[2])
    return s, info, counts


@pytest.mark.parametrize("n,cycle,nu", [(128, "V", (2, 2)), (128, "F", (2, 2)), (128, "V", (1, 1)),
                                        (128, "V", (3, 1)), (128, "V", (2, 1)), (192, "V", (2, 2))])
def test_step_equals_host_loop(n, cycle, nu):
    s, info, counts = check_step(n, 40 + n, 1e-10, 400, cycle=cycle, nu1=nu[0], nu2=nu[1])
    c = info.cycles
    assert info.status == 0 and c >= 3
    # the split path ran: one whole-level norm (before the first cycle), one
    # pre-sweep ahead per cycle, and every later cycle skips its first pre-sweep
    assert counts[PFC_KERNEL_NORM0] == 1
    assert counts[PFC_KERNEL_SWEEP_NORM0] == c
    assert counts[PFC_KERNEL_SMOOTH0] == c * (nu[0] + nu[1]) - (c - 1)


@pytest.mark.parametrize("n,cycle,nu", [(128, "V", (2, 2)), (128, "F", (2, 2)), (192, "V", (2, 1))])
def test_step_equals_host_loop_mobility(n, cycle, nu):
    """Variable mobility: both halves take the flux form of the first
    equation with the face mobilities of phi*."""
    s, info, counts = check_step(n, 60 + n, 1e-10, 400, cycle=cycle, nu1=nu[0], nu2=nu[1],
                                 mobility=MOB)
    c = info.cycles
    assert info.status == 0 and c >= 3
    assert counts[PFC_KERNEL_NORM0] == 1
    assert counts[PFC_KERNEL_SWEEP_NORM0] == c
    assert counts[PFC_KERNEL_SMOOTH0] == c * (nu[0] + nu[1]) - (c - 1)


@pytest.mark.parametrize("n,mobility", [(32, None), (64, None), (64, MOB)])
def test_half_sweep_levels_equal_host_loop(n, mobility):
    s, info, counts = check_step(n, 20 + n, 1e-10, 400, mobility=mobility)
    assert info.status == 0 and info.cycles >= 3
    # V(2,2) in half-sweeps: eight finest-level launches per cycle, no split
    assert counts[PFC_KERNEL_SWEEP_NORM0] == 0
    assert counts[PFC_KERNEL_SMOOTH0] == 8 * info.cycles


@pytest.mark.parametrize("max_cycles", [1, 2, 3])
def test_not_converged_equals_host_loop(max_cycles):
    """The last allowed cycle takes the whole-level norm (no sweep ahead)."""
    s, info, counts = check_step(128, 77, 1e-14, max_cycles)
    assert info.status == 2 and info.cycles == max_cycles
    assert counts[PFC_KERNEL_SWEEP_NORM0] == max_cycles - 1
    assert counts[PFC_KERNEL_NORM0] == 2


def test_picard_and_loose_tolerance():
    check_step(128, 91, 1e-6, 400, lin="picard")


def test_step_256_equals_host_loop():
    """The benchmark's size: 256^3 polycrystal, V(2,2) to 1e-10."""
    s, info, counts = check_step(256, 8, 1e-10, 400)
    assert info.status == 0 and counts[PFC_KERNEL_SWEEP_NORM0] == info.cycles


@pytest.mark.parametrize("cycle,mobility", [("V", None), ("F", None), ("V", MOB)])
def test_graph_loop_equals_host_loop(cycle, mobility):
    """pfc_run (graph replays, the colour-1 half seeded with the whole-level
    norm before a step's first replay) against the host loop, three steps."""
    n = 128
    p, phi = workload(n, 123)
    s = make(n, p.L, p.eps, p.dt, cycle=cycle, mobility=mobility)
    ref = make(n, p.L, p.eps, p.dt, cycle=cycle, mobility=mobility)
    mu, om = s.init_guess(phi)
    mu_h, om_h = mu.clone(), om.clone()
    prev, cur = phi.clone(), phi.clone()
    infos = s.run(prev, cur, mu, om, 3)
    hp, hc = phi.clone(), phi.clone()
    for k in range(3):
        u, c, status, res0, res = host_loop(ref, hp, hc, mu_h, om_h, 1e-10, 400, mobility)
        assert (infos[k].cycles, infos[k].status) == (c, status)
        assert infos[k].res0 == res0 and infos[k].res_final == res
        hp, hc = hc, u[0].clone()
        mu_h, om_h = u[1].clone(), u[2].clone()
    torch.cuda.synchronize()
    assert torch.equal(cur, hc) and torch.equal(prev, hp)
    assert torch.equal(mu, mu_h) and torch.equal(om, om_h)
