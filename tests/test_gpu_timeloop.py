"""The graph-driven time loop (pfc_run) against the step-by-step driver and
the CPU oracle.

pfc_run replays one recorded cycle (residual test, then a gated cycle) per
cycle and takes the loop's decisions on the device; it must reproduce the
pfc_step loop bit for bit, including the cycle counts and residuals it
reports.  The long run follows the polycrystal growth of Section 6.2
(eqn init2, eps = 0.25, [0, 64]^3, tau = 0.01) to t = 40 and checks what the
scheme guarantees at any length (the modified energy of Prop. prop:hu09 does
not grow; mass moves only by the residual) and what the physics fixes (the
density wave forms at |k| = 1, the fastest-growing mode of the linearised
equation).
"""
import math

import numpy as np
import pytest
import torch

from paper_1611_06288_amd import inputs

pytestmark = pytest.mark.gpu

MOB = (1.0, 0.0, -1.0, 0.05)


def step_loop(s, prev, cur, mu, om, steps):
    infos = []
    spare = torch.empty_like(cur)
    for _ in range(steps):
        nxt, info = s.step(prev, cur, mu, om, out=spare, raise_on_error=False)
        infos.append(info)
        spare, prev, cur = prev, cur, nxt
        if info.status != 0:
            break
    return prev, cur, infos


def start(s, n, seed):
    phi0 = torch.from_numpy(inputs.polycrystal_phi0(n, s.L, 2, seed=seed, radius_cells=4)).cuda()
    mu, om = s.init_guess(phi0)
    return phi0, mu, om


@pytest.mark.parametrize("n,cycle,nu,mob", [
    (64, "V", (2, 2), None),     # graph, thread-per-point levels
    (48, "F", (2, 2), None),     # graph, F-cycles
    (128, "V", (2, 2), None),    # graph, fused sweep and column tiles at the finest level
    (32, "V", (1, 2), None),     # graph, odd sweep count on half-sweep levels
    (128, "V", (1, 2), None),    # odd sweep count with fused levels: the step loop runs
    (32, "V", (2, 2), MOB),      # graph, variable mobility
])
def test_run_equals_step_loop_bitwise(n, cycle, nu, mob):
    from paper_1611_06288_amd import Solver
    L = n * math.pi / 4
    kw = dict(tol=1e-10, nu1=nu[0], nu2=nu[1], cycle=cycle, mobility=mob)
    a, b = Solver(n, L, 0.25, 0.5, **kw), Solver(n, L, 0.25, 0.5, **kw)
    phi0, mu0, om0 = start(a, n, 2100 + n)
    steps = 6
    prev_a, cur_a, mu_a, om_a = phi0.clone(), phi0.clone(), mu0.clone(), om0.clone()
    ia = a.run(prev_a, cur_a, mu_a, om_a, steps)
    mu_b, om_b = mu0.clone(), om0.clone()
    prev_b, cur_b, ib = step_loop(b, phi0.clone(), phi0.clone(), mu_b, om_b, steps)
    torch.cuda.synchronize()
    assert [i.cycles for i in ia] == [i.cycles for i in ib]
    assert [(i.res0, i.res_final) for i in ia] == [(i.res0, i.res_final) for i in ib]
    assert all(i.status == 0 for i in ia)
    for x, y in ((prev_a, prev_b), (cur_a, cur_b), (mu_a, mu_b), (om_a, om_b)):
        assert torch.equal(x, y)


@pytest.mark.parametrize("n,cycle,mob", [
    (32, "V", None),             # thread-per-point levels
    (48, "F", None),             # F-cycles, hierarchy down to 3^3
    (64, "V", None),             # the long run's size
    (32, "V", MOB),              # variable mobility
])
def test_run_matches_oracle(n, cycle, mob):
    """pfc_run (graph replays, device stop test and cycle gate) against the
    CPU oracle's time loop directly: equal cycle counts at every step,
    phi, mu and omega within 1e-11 relative (max norm), the reported final
    residual below tol.  (128^3 with fused sweeps and column tiles is
    compared with the oracle's 200-step trajectory of the 128^3 polycrystal
    in test_gpu_configs.py.)"""
    from oracle import cfas
    from paper_1611_06288_amd import Solver
    L, eps, dt, steps, tol = n * math.pi / 4, 0.25, 0.5, 6, 1e-10
    phi0 = inputs.polycrystal_phi0(n, L, 2, seed=2600 + n, radius_cells=4)
    s = Solver(n, L, eps, dt, tol=tol, cycle=cycle, mobility=mob)
    p0 = torch.from_numpy(phi0).cuda()
    mu, om = s.init_guess(p0)
    prev, cur = p0.clone(), p0.clone()
    infos = s.run(prev, cur, mu, om, steps)
    torch.cuda.synchronize()
    phis, oinfos, (omu, oom) = cfas.simulate(phi0, L, eps, dt, steps, tol=tol, cycle=cycle,
                                             mobility=mob)
    got_c, want_c = [i.cycles for i in infos], [i.cycles for i in oinfos]
    print(f"n={n} {cycle} mob={mob is not None}: cycles {got_c} (oracle {want_c})")
    assert got_c == want_c
    assert all(i.status == 0 and i.res_final <= tol for i in infos)
    for got, want in ((prev, phis[-2]), (cur, phis[-1]), (mu, omu), (om, oom)):
        g = got.cpu().numpy()
        err = float(np.max(np.abs(g - want)) / np.max(np.abs(want)))
        assert err <= 1e-11, err


@pytest.mark.parametrize("steps", [1, 2, 3, 4])
def test_run_returns_state_in_callers_buffers(steps):
    """Every step count leaves (phi^{k-1}, phi^k) in (phi_prev, phi_cur),
    whichever of the loop's three buffers they ended in."""
    from paper_1611_06288_amd import Solver
    n = 16
    s = Solver(n, n * math.pi / 4, 0.25, 0.5)
    phi0, mu0, om0 = start(s, n, 2200)
    prev, cur, mu, om = phi0.clone(), phi0.clone(), mu0.clone(), om0.clone()
    s.run(prev, cur, mu, om, steps)
    pb, cb, _ = step_loop(s, phi0.clone(), phi0.clone(), mu0.clone(), om0.clone(), steps)
    torch.cuda.synchronize()
    assert torch.equal(prev, pb) and torch.equal(cur, cb)


def test_run_after_kernel_level_sweep_rerecords():
    """A full sweep through the kernel-level entry point trades the finest
    level's buffers; the loop must notice and record its cycle again."""
    from paper_1611_06288_amd import Solver
    from paper_1611_06288_amd._lib import PFC_SWEEP_FULL
    n = 128
    L = n * math.pi / 4
    a, b = Solver(n, L, 0.25, 0.5), Solver(n, L, 0.25, 0.5)
    phi0, mu0, om0 = start(a, n, 2300)
    pa, ca, ma, oa = phi0.clone(), phi0.clone(), mu0.clone(), om0.clone()
    a.run(pa, ca, ma, oa, 2)
    u3 = torch.stack([phi0, mu0, om0]).contiguous()
    f3 = a.source(phi0, phi0)
    a.smooth(0, PFC_SWEEP_FULL, u3, f3, phi0)
    a.run(pa, ca, ma, oa, 2)
    pb, cb, mb, ob = phi0.clone(), phi0.clone(), mu0.clone(), om0.clone()
    b.run(pb, cb, mb, ob, 4)
    torch.cuda.synchronize()
    assert torch.equal(ca, cb) and torch.equal(pa, pb) and torch.equal(ma, mb)


def test_run_not_converged_and_mixed():
    from paper_1611_06288_amd import Solver
    from paper_1611_06288_amd.solver import PFCError
    n = 32
    L = n * math.pi / 4
    # max_cycles = 1 with an unreachable tolerance: the first step reports it
    a = Solver(n, L, 0.25, 0.5, tol=1e-30, max_cycles=1)
    b = Solver(n, L, 0.25, 0.5, tol=1e-30, max_cycles=1)
    phi0, mu0, om0 = start(a, n, 2400)
    pa, ca, ma, oa = phi0.clone(), phi0.clone(), mu0.clone(), om0.clone()
    infos = a.run(pa, ca, ma, oa, 3, raise_on_error=False)
    assert len(infos) == 3 and infos[0].status == 2 and infos[0].cycles == 1
    assert infos[1].cycles == 0  # not run
    pb, cb, ib = step_loop(b, phi0.clone(), phi0.clone(), mu0.clone(), om0.clone(), 3)
    assert len(ib) == 1 and ib[0].status == 2
    torch.cuda.synchronize()
    assert torch.equal(ca, cb) and torch.equal(pa, pb)
    with pytest.raises(PFCError):
        a.run(pa, ca, ma, oa, 1)
    # the mixed-precision form runs its own step loop
    m1, m2 = (Solver(n, L, 0.25, 0.5, precision="mixed") for _ in range(2))
    pa, ca, ma, oa = phi0.clone(), phi0.clone(), mu0.clone(), om0.clone()
    ia = m1.run(pa, ca, ma, oa, 3)
    pb, cb, ib = step_loop(m2, phi0.clone(), phi0.clone(), mu0.clone(), om0.clone(), 3)
    torch.cuda.synchronize()
    assert [i.cycles for i in ia] == [i.cycles for i in ib]
    assert torch.equal(ca, cb)
    # argument checks
    with pytest.raises(PFCError):
        a.run(pa, pa, ma, oa, 1)
    assert a.run(pa, ca, ma, oa, 0) == []


def test_long_polycrystal_growth_section_6_2():
    """eqn init2 on [0, 64]^3 at 64^3 (h = 1; the paper gives no grid), eps =
    0.25, tau = 0.01, 4000 steps to t = 40, the first snapshot time of the
    paper's figure."""
    from paper_1611_06288_amd import Solver
    n, L, eps, dt = 64, 64.0, 0.25, 0.01
    s = Solver(n, L, eps, dt, tol=1e-10)
    phi0 = torch.from_numpy(inputs.paper_init2(n, seed=11)).cuda()
    mu, om = s.init_guess(phi0)
    prev, cur = phi0.clone(), phi0.clone()
    h3 = (L / n) ** 3
    mass0 = s.energy(phi0)[2]
    bound = 1e-12 * abs(mass0)
    energies = []
    cycles = []
    for chunk in range(8):
        infos = s.run(prev, cur, mu, om, 500)
        assert all(i.status == 0 for i in infos)
        cycles += [i.cycles for i in infos]
        bound += sum(h3 * n ** 3 * i.res_final for i in infos)
        e = s.energy(cur, prev)
        energies.append(e[1])
        assert abs(e[2] - mass0) <= bound
        print(f"t = {(chunk + 1) * 5:3d}: modified energy {e[1]:.6f}, mean cycles "
              f"{np.mean(cycles[-500:]):.2f}", flush=True)
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(energies, energies[1:])), energies
    phi = cur.cpu().numpy()
    amp0 = float(np.std(phi0.cpu().numpy()))
    # linear theory: the noise's standard deviation grows about 14x by t = 40
    assert np.std(phi) > 5 * amp0, (np.std(phi), amp0)
    # radially averaged power spectrum peaks at |k| = 1 (wavelength 2 pi)
    F = np.abs(np.fft.fftn(phi - phi.mean())) ** 2
    k1 = 2 * np.pi * np.fft.fftfreq(n, d=L / n)
    kx, ky, kz = np.meshgrid(k1, k1, k1, indexing="ij")
    kr = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    dk = 2 * np.pi / L
    shells = np.rint(kr / dk).astype(int)
    power = np.bincount(shells.ravel(), F.ravel()) / np.maximum(np.bincount(shells.ravel()), 1)
    kpeak = np.argmax(power[1:]) * dk + dk
    print("spectrum peak at |k| =", kpeak)
    assert 0.85 <= kpeak <= 1.15


def test_run_reports_nonfinite():
    """A NaN in the state makes the device stop test report NONFINITE after
    the first norm, as the step loop does, and the loop stops there."""
    from paper_1611_06288_amd import Solver
    from paper_1611_06288_amd.solver import PFCError
    n = 16
    s = Solver(n, n * math.pi / 4, 0.25, 0.5)
    phi0, mu0, om0 = start(s, n, 2500)
    bad = phi0.clone()
    bad[3, 4, 5] = float("nan")
    prev, cur, mu, om = bad.clone(), bad.clone(), mu0.clone(), om0.clone()
    infos = s.run(prev, cur, mu, om, 3, raise_on_error=False)
    assert infos[0].status == 3 and infos[0].cycles == 0
    assert infos[1].status == 0 and infos[1].cycles == 0  # not run
    with pytest.raises(PFCError) as e:
        s.run(bad.clone(), bad.clone(), mu0.clone(), om0.clone(), 1)
    assert e.value.status == 3
    # the handle is still usable afterwards
    prev, cur, mu, om = phi0.clone(), phi0.clone(), mu0.clone(), om0.clone()
    assert all(i.status == 0 for i in s.run(prev, cur, mu, om, 2))


def test_zero_steps_leave_the_state_alone():
    """Empty input: pfc_run and pfc_batch_run over zero steps return at once,
    report nothing and leave every buffer bit for bit as it was."""
    from paper_1611_06288_amd import Solver
    from paper_1611_06288_amd.solver import Batch
    n = 32
    s = Solver(n, n * math.pi / 4, 0.25, 0.5, tol=1e-10)
    phi0, mu0, om0 = start(s, n, 2300)
    state = [phi0.clone(), (phi0 + 0.01).clone(), mu0.clone(), om0.clone()]
    before = [t.clone() for t in state]
    assert s.run(*state, 0) == []
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(state, before))
    ens = [dict(n=16, L=4 * math.pi, eps=0.25, dt=0.5,
                phi0=inputs.polycrystal_phi0(16, 4 * math.pi, 1, seed=2301, radius_cells=3)),
           dict(n=24, L=6 * math.pi, eps=0.2, dt=0.5,
                phi0=inputs.polycrystal_phi0(24, 6 * math.pi, 1, seed=2302, radius_cells=3))]
    b = Batch(ens, tol=1e-10)
    for i, p in enumerate(ens):
        b.init_state(i, torch.from_numpy(p["phi0"]).cuda())
    kept = [[t.clone() for t in b.get_state(i)] for i in range(2)]
    assert b.run(0) == [[], []]
    for i in range(2):
        assert all(torch.equal(x, y) for x, y in zip(b.get_state(i), kept[i]))
