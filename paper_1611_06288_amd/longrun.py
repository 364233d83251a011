"""Long polycrystal growth run of Section 6.2 through the graph-driven time
loop (``pfc_run``), logging what the scheme guarantees at any length.

    python -m paper_1611_06288_amd.longrun --t-end 1000 --log-every 1000
    python -m paper_1611_06288_amd.longrun --t-end 5000 --resume run.npz --save run.npz

Workload: eqn init2 (0.2 + 0.005 U[0, 1], seed 11) on [0, 64]^3 at 64^3
(h = 1), eps = 0.25, tau = 0.01, V(2,2) to a max-norm residual of 1e-10.
Every ``log_every`` steps one JSON line reports t, the modified energy
F_h(phi^{k+1}) + 1/2 |grad_h(phi^{k+1} - phi^k)|^2 (Proposition prop:hu09:
non-increasing), the mass h^3 sum(phi) and its drift against the bound
sum over steps of h^3 n^3 max|r1| (the first equation's residual moves the
mass by at most that much; scheme (1.10) conserves it exactly), the standard
deviation of phi, the mean cycles per step and the steps per second.  The
last line is a summary with the checks' outcomes.

--save writes the state (phi^{k-1}, phi^k, mu, omega), the step count, the
starting energy and mass and the running mass bound to an .npz file;
--resume continues from such a file, so a long run can be split over several
processes with the checks carried across (the trajectory is the one an
uninterrupted run takes, except that the coarsest level's cached inverse is
rebuilt at the restart: a chord-iteration start, not a change of the solve's
tolerance).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--t-end", type=float, default=1000.0)
    ap.add_argument("--log-every", type=int, default=1000, help="steps between log lines")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--save", default=None, help="write the final state to this .npz file")
    ap.add_argument("--resume", default=None, help="continue from a state written by --save")
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import inputs
    from .solver import Solver

    n, L, eps, dt = args.n, float(args.n), 0.25, 0.01
    steps = int(round(args.t_end / dt))
    h3 = (L / n) ** 3
    s = Solver(n, L, eps, dt, tol=args.tol)
    if args.resume:
        with np.load(args.resume, allow_pickle=False) as z:
            if int(z["n"]) != n:
                raise SystemExit(f"--resume: state is {int(z['n'])}^3, not {n}^3")
            prev, cur, mu, om = (torch.from_numpy(np.ascontiguousarray(z[k])).cuda()
                                 for k in ("prev", "cur", "mu", "om"))
            done, e0, mass0 = int(z["steps"]), float(z["energy0"]), float(z["mass0"])
            bound, last_e = float(z["bound"]), float(z["energy_last"])
    else:
        phi0 = torch.from_numpy(inputs.paper_init2(n, seed=11)).cuda()
        mu, om = s.init_guess(phi0)
        prev, cur = phi0.clone(), phi0.clone()
        _, e0, mass0 = s.energy(phi0)
        bound = 1e-12 * abs(mass0)
        last_e = e0
        done = 0
        print(json.dumps({"t": 0.0, "energy_mod": e0, "mass": mass0, "std_phi":
                          float(phi0.std())}), flush=True)
    monotone, within = True, True
    cycles_total = 0
    start_step = done
    t_start = time.perf_counter()
    while done < steps:
        k = min(args.log_every, steps - done)
        t0 = time.perf_counter()
        infos = s.run(prev, cur, mu, om, k)
        torch.cuda.synchronize()
        dt_wall = time.perf_counter() - t0
        done += k
        cyc = sum(i.cycles for i in infos)
        cycles_total += cyc
        bound += sum(h3 * n ** 3 * i.res_final for i in infos)
        _, e, m = s.energy(cur, prev)
        monotone = monotone and e <= last_e + 1e-12 * abs(last_e)
        within = within and abs(m - mass0) <= bound
        last_e = e
        print(json.dumps({
            "t": round(done * dt, 6), "energy_mod": e, "mass": m, "mass_drift": m - mass0,
            "mass_bound": bound, "std_phi": float(cur.std()), "mean_cycles": cyc / k,
            "max_res_final": max(i.res_final for i in infos), "steps_per_s": k / dt_wall,
        }), flush=True)
    wall = time.perf_counter() - t_start
    ran = max(done - start_step, 1)
    if args.save:
        np.savez(args.save, n=n, steps=done, energy0=e0, mass0=mass0, bound=bound,
                 energy_last=last_e, prev=prev.cpu().numpy(), cur=cur.cpu().numpy(),
                 mu=mu.cpu().numpy(), om=om.cpu().numpy())
    summary = {
        "summary": True, "t_start": start_step * dt, "t_end": done * dt, "steps": done - start_step,
        "n": n, "wall_s": round(wall, 2), "steps_per_s": round(ran / wall, 2),
        "mean_cycles_per_step": round(cycles_total / ran, 3),
        "modified_energy_non_increasing": monotone, "mass_within_residual_bound": within,
        "energy_mod_start": e0, "energy_mod_end": last_e,
    }
    print(json.dumps(summary), flush=True)
    return 0 if (monotone and within and math.isfinite(last_e)) else 1


if __name__ == "__main__":
    sys.exit(main())
