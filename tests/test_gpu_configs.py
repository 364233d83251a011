"""The HIP path against the oracle at the polycrystal workloads' own sizes.

The references are the oracle's trajectories written by
tests/golden/make_config_goldens.py (oracle only):
  * 128^3 polycrystal (3 crystallites, seed 2), 200 steps: per-step cycles,
    residuals, mass and energies; phi on four z-planes and (phi, mu, omega)
    at 4096 seeded points at steps 50, 100, 150 and 200;
  * 256^3 polycrystal (8 crystallites, seed 3), the first 2 steps: the same
    records, phi on one z-plane and (phi, mu, omega) at 8192 points.

The FP64 bar of scheme (1.10) solved by Algorithm algorithm:FAS: the same
cycle count at every step, fields within 1e-11 relative (max norm over the
stored values), mass and energies within 1e-11 relative, every final
residual at or below tol.  Both the step loop (pfc_step) and the
graph-driven loop (pfc_run) are held to it at 128^3 over the first 100
steps.  Over a trajectory the two runs do not share inputs after the first
step: their rounding-level differences (about 1e-14 relative per step) are
carried forward and amplified by the growth dynamics, measured at about 4x
per 50 steps here (3.5e-13 at step 50, 1.4e-12 at step 100).  From step 101
on the trajectory bar is therefore 1e-9 for fields and energies (equal cycle
counts still required).  The per-step bar on identical inputs is the one at
256^3 below and in the mixed and time-loop tests.  The mixed form's per-step
max-norm error against the oracle's steps is reported at 256^3.
"""
import math
import os

import numpy as np
import pytest
import torch

from paper_1611_06288_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FIELD_REL = 1e-11
SCALAR_REL = 1e-11
LATE_REL = 1e-9      # trajectory bar after step 100 (see above)
LATE_FROM = 100


def field_bar(step):
    return FIELD_REL if step <= LATE_FROM else LATE_REL


def scalar_bar(step):
    return SCALAR_REL if step <= LATE_FROM else LATE_REL


def load(name):
    with np.load(os.path.join(GOLDEN, name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def check_snapshot(ref, ck, phi, mu, om, label, bar=FIELD_REL):
    """phi on the stored planes, (phi, mu, omega) at the stored points."""
    idx = ref["sample_index"]
    planes = ref["planes"]
    got_planes = phi[planes]
    e_pl = rel(got_planes, ref["phi_planes"][ck])
    e_pts = [rel(a.reshape(-1)[idx], ref["sample_values"][ck][c]) for c, a in enumerate((phi, mu, om))]
    print(f"{label}: phi planes {e_pl:.2e}, samples phi/mu/omega "
          f"{e_pts[0]:.2e}/{e_pts[1]:.2e}/{e_pts[2]:.2e}", flush=True)
    assert e_pl <= bar and max(e_pts) <= bar, (label, e_pl, e_pts)


def check_scalars(ref, k, energy, info, label, bar=SCALAR_REL):
    F, Ft, m = energy
    for name, got in (("energy", F), ("energy_mod", Ft), ("mass", m)):
        want = float(ref[name][k])
        assert abs(got - want) <= bar * abs(want), (label, name, got, want)
    assert info.cycles == int(ref["cycles"][k]), (label, info.cycles, int(ref["cycles"][k]))
    assert info.status == 0 and info.res_final <= float(ref["tol"])
    # both residual norms near tol are differences of O(1e2) terms: equal
    # to within their rounding
    assert abs(info.res_final - float(ref["res_final"][k])) <= 1e-12, label


def test_config2_polycrystal_128_200_steps_step_loop():
    from paper_1611_06288_amd import Solver
    ref = load("config2_polycrystal_128.npz")
    n, steps = int(ref["n"]), int(ref["steps"])
    L, eps, dt, tol = float(ref["L"]), float(ref["eps"]), float(ref["dt"]), float(ref["tol"])
    phi0 = inputs.polycrystal_128()
    s = Solver(n, L, eps, dt, tol=tol)
    checkpoints = [int(c) for c in ref["checkpoints"]]
    seen = []

    def cb(k, nxt, mu, om, info):
        prev = seen[-1] if seen else ph
        e = s.energy(nxt, prev)
        check_scalars(ref, k, e, info, f"step {k + 1}", scalar_bar(k + 1))
        if k + 1 in checkpoints:
            check_snapshot(ref, checkpoints.index(k + 1), nxt.cpu().numpy(), mu.cpu().numpy(),
                           om.cpu().numpy(), f"step {k + 1}", field_bar(k + 1))
        seen[:] = [nxt.clone()]

    ph = torch.from_numpy(phi0).cuda()
    s.simulate(ph, steps, callback=cb)
    print(f"cycles per step: first {list(ref['cycles'][:5])}, last {list(ref['cycles'][-5:])}")


def test_config2_polycrystal_128_200_steps_graph_loop():
    """pfc_run in chunks that end at the stored steps."""
    from paper_1611_06288_amd import Solver
    ref = load("config2_polycrystal_128.npz")
    n = int(ref["n"])
    L, eps, dt, tol = float(ref["L"]), float(ref["eps"]), float(ref["dt"]), float(ref["tol"])
    s = Solver(n, L, eps, dt, tol=tol)
    ph = torch.from_numpy(inputs.polycrystal_128()).cuda()
    mu, om = s.init_guess(ph)
    prev, cur = ph.clone(), ph.clone()
    done = 0
    for ck, stop in enumerate(int(c) for c in ref["checkpoints"]):
        infos = s.run(prev, cur, mu, om, stop - done)
        for j, info in enumerate(infos):
            k = done + j
            assert info.cycles == int(ref["cycles"][k]), (k, info.cycles)
            assert info.status == 0 and info.res_final <= tol
            assert abs(info.res_final - float(ref["res_final"][k])) <= 1e-12
        done = stop
        check_scalars(ref, stop - 1, s.energy(cur, prev), infos[-1], f"run to step {stop}",
                      scalar_bar(stop))
        check_snapshot(ref, ck, cur.cpu().numpy(), mu.cpu().numpy(), om.cpu().numpy(),
                       f"run to step {stop}", field_bar(stop))


def test_config3_polycrystal_256_first_steps_fp64_and_mixed():
    from paper_1611_06288_amd import Solver
    ref = load("config3_polycrystal_256.npz")
    n, steps = int(ref["n"]), int(ref["steps"])
    L, eps, dt, tol = float(ref["L"]), float(ref["eps"]), float(ref["dt"]), float(ref["tol"])
    ph = torch.from_numpy(inputs.polycrystal_256()).cuda()
    idx = ref["sample_index"]
    plane = int(ref["planes"][0])
    for precision in ("fp64", "mixed"):
        s = Solver(n, L, eps, dt, tol=tol, precision=precision)
        mu, om = s.init_guess(ph)
        prev, cur = ph.clone(), ph.clone()
        same_so_far = True
        for k in range(steps):
            nxt, info = s.step(prev, cur, mu, om)
            if precision == "fp64":
                check_scalars(ref, k, s.energy(nxt, cur), info, f"fp64 step {k + 1}")
                check_snapshot(ref, k, nxt.cpu().numpy(), mu.cpu().numpy(), om.cpu().numpy(),
                               f"fp64 step {k + 1}")
            else:
                want_c = int(ref["cycles"][k])
                got = [nxt.cpu().numpy(), mu.cpu().numpy(), om.cpu().numpy()]
                err_plane = float(np.max(np.abs(got[0][plane] - ref["phi_planes"][k][0])))
                err_pts = max(float(np.max(np.abs(a.reshape(-1)[idx] - ref["sample_values"][k][c])))
                              for c, a in enumerate(got))
                err = max(err_plane, err_pts)
                same_so_far = same_so_far and info.cycles == want_c
                print(f"mixed step {k + 1}: cycles {info.cycles} (oracle {want_c}), FP64 residual "
                      f"{info.res_final:.2e}; max-norm error vs the FP64 oracle over one "
                      f"z-plane and {idx.size} points: {err:.3e}", flush=True)
                assert info.status == 0 and info.res_final <= tol
                assert want_c <= info.cycles <= want_c + 2
                if same_so_far:
                    assert err <= 1e-12, err
            prev, cur = cur, nxt
        s.close()
