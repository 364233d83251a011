"""Writes the oracle's reference trajectories of the two polycrystal
workloads (h = pi/4, eps = 0.25, s = 0.5, V(2,2) to a max-norm residual of
1e-10, bootstrap phi^{-1} = phi^0, first-step guess of the discrete chemical
potential).  Calls only oracle/ and the seeded input generator.

* ``config2_polycrystal_128.npz``: 128^3, 3 crystallites (seed 2), 200 steps.
  Per step: cycles, the residual before the first cycle and after the last,
  mass h^3 sum(phi), F_h(phi^{k+1}) and the modified energy
  F_h(phi^{k+1}) + 1/2 |grad_h(phi^{k+1} - phi^k)|^2.  At steps 50, 100, 150
  and 200: phi on the z-planes 0, 37, 64 and 101, and (phi, mu, omega) at
  4096 seeded random points.
* ``config3_polycrystal_256.npz``: 256^3, 8 crystallites (seed 3), the first
  2 steps, with the same per-step records, phi on the z-plane 100 and
  (phi, mu, omega) at 8192 seeded random points after each step.

    python tests/golden/make_config_goldens.py [2] [3]
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cfas  # noqa: E402
from paper_1611_06288_amd import inputs  # noqa: E402

EPS, DT, TOL = 0.25, 0.5, 1e-10


def sample_index(n, count, seed):
    return np.sort(inputs.rng(seed).choice(n ** 3, size=count, replace=False)).astype(np.int64)


def trajectory(phi0, n, steps, checkpoints, planes, idx, out_path):
    L = n * math.pi / 4.0
    h = L / n
    rec = {k: [] for k in ("cycles", "res0", "res_final", "mass", "energy", "energy_mod")}
    ck_planes, ck_pts = [], []
    prev = [np.ascontiguousarray(phi0)]
    t0 = time.time()

    def cb(k, nxt, mu, om, info):
        F, Ft, m = cfas.energy(nxt, h, EPS, prev[0])
        rec["cycles"].append(info.cycles)
        rec["res0"].append(info.res_hist[0])
        rec["res_final"].append(info.res_hist[-1])
        rec["mass"].append(m)
        rec["energy"].append(F)
        rec["energy_mod"].append(Ft)
        if k + 1 in checkpoints:
            ck_planes.append(np.stack([nxt[z] for z in planes]))
            ck_pts.append(np.stack([a.reshape(-1)[idx] for a in (nxt, mu, om)]))
        prev[0] = nxt
        print(f"n={n} step {k + 1}: cycles {info.cycles} res {info.res_hist[-1]:.3e} "
              f"E~ {Ft:.12e} ({time.time() - t0:.0f} s)", flush=True)

    F0, _, m0 = cfas.energy(phi0, h, EPS)
    cfas.simulate(phi0, L, EPS, DT, steps, tol=TOL, callback=cb)
    np.savez_compressed(
        out_path, n=n, L=L, eps=EPS, dt=DT, tol=TOL, steps=steps, energy0=F0, mass0=m0,
        checkpoints=np.array(checkpoints, dtype=np.int64), planes=np.array(planes, dtype=np.int64),
        sample_index=idx, phi_planes=np.stack(ck_planes), sample_values=np.stack(ck_pts),
        **{k: np.array(v) for k, v in rec.items()})
    print("wrote", out_path, flush=True)


def main():
    which = sys.argv[1:] or ["2", "3"]
    print("oracle threads", cfas.num_threads(), flush=True)
    if "3" in which:
        trajectory(inputs.polycrystal_256(), 256, 2, [1, 2], [100], sample_index(256, 8192, 33),
                   os.path.join(HERE, "config3_polycrystal_256.npz"))
    if "2" in which:
        trajectory(inputs.polycrystal_128(), 128, 200, [50, 100, 150, 200], [0, 37, 64, 101],
                   sample_index(128, 4096, 22), os.path.join(HERE, "config2_polycrystal_128.npz"))


if __name__ == "__main__":
    main()
