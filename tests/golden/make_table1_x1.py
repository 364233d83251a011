"""Writes table1_x1.npz: the oracle's solutions on the refinement path of
Table tab:cov (Section 6.1): [0, 3.2]^3, eps = 0.025, tau = 0.05 h, T = 0.16,
eqn init1, at 16^3, 32^3 and 64^3.  Calls only oracle/ and the input
generator.

Every step runs exactly 20 V(2,2) cycles.  On this path the residual stops
at a rounding floor that grows about 30x per refinement (1.2e-12 at 16^3,
3.7e-11 at 32^3 in the first step), so no one tolerance is both attainable
at 64^3 and small at 16^3; 20 cycles reach the floor at every size (the
residual falls about tenfold per cycle), and a fixed count makes the GPU
run the same iterations.  Stored: phi at T on 16^3 and 32^3, the 8-child
means of phi at T on 32^3 and 64^3 (the Cauchy differences compare a grid
with the means of the next finer one), the final residual of every step per
size, and the l2 (sqrt(h^3 sum d^2)) and max Cauchy differences.  Those are
taken on fields with their means removed: scheme (1.10) conserves the mean
exactly, so the mean's drift is the solver's rounding at the residual floor
(each step moves it by at most the first equation's residual, and the
conservative scheme never damps it), not a discretisation error; at 64^3 it
reaches 7e-12, a twentieth of the 32-64 difference.  The raw differences are
stored beside them.

    python tests/golden/make_table1_x1.py
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cfas  # noqa: E402
from paper_1611_06288_amd import inputs  # noqa: E402

L, EPS, T, CYCLES = 3.2, 0.025, 0.16, 20


def restrict(a):
    m = a.shape[0] // 2
    return a.reshape(m, 2, m, 2, m, 2).mean(axis=(1, 3, 5))


def solve(n):
    h = L / n
    dt = 0.05 * h
    steps = int(round(T / dt))
    phi0 = inputs.paper_init1(n, L)
    s = cfas.Solver(n, L, EPS, dt, tol=1e-300, max_cycles=CYCLES)
    mu, om = cfas.initial_guess(phi0, h, EPS)
    prev, cur = phi0, phi0
    res = []
    for _ in range(steps):
        nxt, mu, om, info = s.step(prev, cur, mu, om)
        assert info.cycles == CYCLES
        res.append(info.res_hist[-1])
        prev, cur = cur, nxt
    s.close()
    print(f"n={n}: {steps} steps, final residuals first {res[0]:.2e} last {res[-1]:.2e}", flush=True)
    return cur, np.array(res)


def main():
    sol, res = {}, {}
    for n in (16, 32, 64):
        sol[n], res[n] = solve(n)
    l2, mx, raw = {}, {}, {}
    for a in (16, 32):
        f, c = restrict(sol[2 * a]), sol[a]
        d = (f - f.mean()) - (c - c.mean())
        l2[a] = math.sqrt((L / a) ** 3 * float(np.sum(d * d)))
        mx[a] = float(np.max(np.abs(d)))
        raw[a] = math.sqrt((L / a) ** 3 * float(np.sum((f - c) ** 2)))
        print(f"{a}-{2 * a}: l2 {l2[a]:.4e} max {mx[a]:.4e} (with the means: l2 {raw[a]:.4e})")
    np.savez_compressed(
        os.path.join(HERE, "table1_x1.npz"), L=L, eps=EPS, T=T, dt_over_h=0.05, cycles=CYCLES,
        phi16=sol[16], phi32=sol[32], mean32=restrict(sol[32]), mean64=restrict(sol[64]),
        res16=res[16], res32=res[32], res64=res[64],
        cauchy_l2=np.array([l2[16], l2[32]]), cauchy_max=np.array([mx[16], mx[32]]),
        cauchy_l2_raw=np.array([raw[16], raw[32]]))


if __name__ == "__main__":
    main()
