#!/usr/bin/env python3
"""Throughput of the FAS multigrid time step on one MI355X.

Workload: 256^3 polycrystal growth (8 seeded crystallites of one-mode BCC
density in a noisy background, h = pi/4, eps = 0.25, s = 0.5), V(2,2) cycles to
an FP64 residual of 1e-10, synthetic inputs resident in HBM before timing.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line: time steps/s of the FP64 path (`value`), its V-cycles/s,
the same for the mixed-precision form, the variable-mobility form and the
first-order convex-splitting scheme on the same workload, the graph-driven
time loop (and the long run of Section 6.2), the batched and adjoint forms,
the finest-level
smoother's achieved HBM bandwidth against the 8 TB/s peak (kernel durations
from HIP events recorded by the library on its stream), and the CPU oracle
timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of one finest-level FP64 smoother launch at 256^3, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch, averaged over
# the step's 256^3 launches of the sweeps the smoother timing covers: plain,
# plain without the dead colour-0 writes, and norm-carrying post-sweeps) scaled
# by what the same counters read for a 1 GiB device copy (FETCH x 2.0,
# WRITE x 1.0).  Valid only for the smoother sources
# it was measured on (first 16 hex digits of the sha256 of smooth.hip, smooth.h,
# device_common.h and runtime.cpp, which chooses the buffers the sweeps read,
# concatenated); otherwise reported null.
SMOOTHER_TRAFFIC = {"sources_sha256_16": "38676dba7cbfe3e2", "n": 256,
                    "fetch_KiB": 360756, "write_KiB": 350145,
                    "fetch_scale": 2.0, "write_scale": 1.0}
SMOOTHER_SOURCES = ("smooth.hip", "smooth.h", "device_common.h", "runtime.cpp")
METRIC = "time-steps/s & V-cycles/s at 256^3 (FP64 vs mixed); smoother HBM GB/s %peak"
# (m0, m1, m2, mmin) of the variable-mobility run: M(v) = max(0.05, 1 - v^2)
MOBILITY = (1.0, 0.0, -1.0, 0.05)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="grid size (256 is the benchmark)")
    ap.add_argument("--cycle", default="V", choices=["V", "F"])
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-mobility", action="store_true",
                    help="skip the variable-mobility run of the same steps")
    ap.add_argument("--no-first-order", action="store_true",
                    help="skip the first-order convex-splitting run of the same workload")
    ap.add_argument("--no-loop", action="store_true",
                    help="skip the graph-driven time loop runs (pfc_run)")
    ap.add_argument("--long-steps", type=int, default=2000,
                    help="steps of the Section 6.2 long-run leg (64^3, tau = 0.01)")
    ap.add_argument("--long-plain-steps", type=int, default=200,
                    help="steps of that leg's step-by-step comparison run")
    ap.add_argument("--no-fcycle", action="store_true",
                    help="skip the FP64 F(2,2) run of the same steps (reported beside V)")
    ap.add_argument("--cpu-cycles", type=int, default=24,
                    help="oracle cycles timed on all threads for the CPU baseline, about 10 s "
                         "on 16 threads (0 disables it)")
    ap.add_argument("--cpu-one-core-cycles", type=int, default=3,
                    help="oracle cycles timed on one thread, about 12 s (child process; 0 skips)")
    ap.add_argument("--cpu-full-step", action="store_true",
                    help="also time the oracle's whole first step on all threads (~1-2 min at 256^3)")
    ap.add_argument("--batch-steps", type=int, default=50,
                    help="time steps of the 64-instance batched ensemble (0 skips it)")
    ap.add_argument("--adjoint-steps", type=int, default=20,
                    help="time steps of the 64^3 differentiated rollout (0 skips it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time a plain 1 GiB device-to-device copy (bandwidth ceiling and "
                         "counter calibration) and exit")
    return ap.parse_args()


def copy_ceiling(torch, nbytes=1 << 30, reps=20):
    """Device-to-device copy of `nbytes` (read + write) timed with events on
    the current stream; returns GB/s counting both directions."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3 / reps
    del src, dst
    return 2 * nbytes / sec / 1e9


def smoother_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in SMOOTHER_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1611_06288_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def smoother_traffic_bytes(n):
    t = SMOOTHER_TRAFFIC
    if t["fetch_KiB"] is None or smoother_sources_sha() != t["sources_sha256_16"] or n != t["n"]:
        return None
    return 1024.0 * (t["fetch_KiB"] * t["fetch_scale"] + t["write_KiB"] * t["write_scale"])


def kernel_stats(s, abi):
    out = {}
    for k, name in enumerate(abi.KERNEL_NAMES):
        cnt, ms, bpl = s.timing_get(k)
        if cnt == 0:
            continue
        avg_s = ms / cnt * 1e-3
        e = {"launches": cnt, "avg_us": round(avg_s * 1e6, 3)}
        if bpl > 0:
            e["alg_bytes_per_launch"] = bpl
            e["achieved_GBps"] = round(bpl / avg_s / 1e9, 1)
        out[name] = e
    return out


def run_path(Solver, abi, torch, precision, state0, p, steps, warmup, cycle, mobility=None,
             scheme=2):
    """Runs warmup + timed steps from state0 = (prev, cur, mu, om); returns a
    dict of results and the list of phi after every timed step (on device)."""
    s = Solver(p.n, p.L, p.eps, p.dt, tol=p.tol, nu1=p.nu1, nu2=p.nu2, cycle=cycle,
               precision=precision, max_cycles=1000, mobility=mobility, scheme=scheme)
    prev, cur, mu, om = (t.clone() for t in state0)
    spare = torch.empty_like(cur)
    for _ in range(warmup):
        nxt, info = s.step(prev, cur, mu, om, out=spare)
        spare, prev, cur = prev, cur, nxt
    torch.cuda.synchronize()
    s.timing_reset()
    s.timing(True)
    cycles = []
    phis = []
    t0 = time.perf_counter()
    for _ in range(steps):
        nxt, info = s.step(prev, cur, mu, om, out=spare)
        cycles.append(info.cycles)
        spare, prev, cur = prev, cur, nxt
        phis.append(cur.clone())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.timing(False)
    dt = t1 - t0
    res = {
        "steps_per_s": steps / dt,
        "v_cycles_per_s": sum(cycles) / dt,
        "ms_per_step": 1e3 * dt / steps,
        "cycles_per_step": cycles,
        "kernels": kernel_stats(s, abi),
    }
    s.close()
    return res, phis


def run_loop(Solver, torch, state0, p, steps, warmup, cycle):
    """The same steps through the graph-driven time loop (pfc_run)."""
    s = Solver(p.n, p.L, p.eps, p.dt, tol=p.tol, nu1=p.nu1, nu2=p.nu2, cycle=cycle, max_cycles=1000)
    prev, cur, mu, om = (t.clone() for t in state0)
    if warmup:
        s.run(prev, cur, mu, om, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = s.run(prev, cur, mu, om, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.close()
    return {"steps_per_s": steps / dt, "ms_per_step": 1e3 * dt / steps,
            "cycles_per_step": [i.cycles for i in infos]}, cur


def run_long(Solver, torch, inputs, steps, plain_steps=200):
    """Section 6.2 growth run (eqn init2, eps = 0.25, [0, 64]^3 at 64^3, tau =
    0.01): steps/s of the graph-driven loop against the step-by-step driver,
    from the state after min(100, steps) steps."""
    n, L, eps, dt = 64, 64.0, 0.25, 0.01
    s = Solver(n, L, eps, dt, tol=1e-10)
    phi0 = torch.from_numpy(inputs.paper_init2(n, seed=11)).cuda()
    mu, om = s.init_guess(phi0)
    prev, cur = phi0.clone(), phi0.clone()
    warm = min(100, steps)
    s.run(prev, cur, mu, om, warm)
    state = [t.clone() for t in (prev, cur, mu, om)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    spare = torch.empty_like(cur)
    for _ in range(plain_steps):
        nxt, _ = s.step(prev, cur, mu, om, out=spare)
        spare, prev, cur = prev, cur, nxt
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    prev, cur, mu, om = state
    t0 = time.perf_counter()
    infos = s.run(prev, cur, mu, om, steps)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    cyc = [i.cycles for i in infos]
    rate = steps / t_loop
    s.close()
    return {
        "workload": "eqn init2 (0.2 + 0.005 U[0,1], seed 11), 64^3 on [0,64]^3, eps=0.25, "
                    f"tau=0.01, V(2,2) to 1e-10, from t = {warm * dt:g}",
        "steps": steps,
        "graph_loop_steps_per_s": round(rate, 2),
        "step_loop_steps_per_s": round(plain_steps / t_plain, 2),
        "speedup": round(rate / (plain_steps / t_plain), 3),
        "mean_cycles_per_step": round(sum(cyc) / len(cyc), 3),
        "hours_for_t_12000": round(1.2e6 / rate / 3600, 2),
    }


def run_batched(torch, inputs, steps, warmup=1):
    """64 instances, n in {32,48,64,96}, eps in [0.02,0.3], s = 0.1, V(2,2) to
    1e-10, tile shapes from the autotuner.  Returns rates aggregated over
    the instances."""
    from paper_1611_06288_amd.solver import Batch
    ens = inputs.batched_ensemble(64, steps=steps)
    params = [dict(n=e.params.n, L=e.params.L, eps=e.params.eps, dt=e.params.dt) for e in ens]
    b = Batch(params, tol=1e-10)
    tiles = b.autotune()
    for i, e in enumerate(ens):
        b.init_state(i, torch.from_numpy(e.phi0()).cuda())
    if warmup:
        b.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = b.run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pts = sum(e.params.n ** 3 for e in ens)
    cyc = [sum(x.cycles for x in row) for row in infos]
    b.close()
    return {
        "instances": len(ens), "steps": steps, "grid_points": pts,
        "sizes": {str(n): sum(1 for e in ens if e.params.n == n) for n in (32, 48, 64, 96)},
        "instance_steps_per_s": round(len(ens) * steps / dt, 3),
        "batch_steps_per_s": round(steps / dt, 4),
        "v_cycles_per_s_summed": round(sum(cyc) / dt, 2),
        "mean_cycles_per_instance_step": round(sum(cyc) / (len(ens) * steps), 2),
        "max_cycles_per_step": max(max(x.cycles for x in row) for row in infos),
        "autotuned_schedule_threads_w_z": dict(zip(
            ["smooth", "resid_restrict", "tau", "prolong", "coarse_err"],
            [["persistent" if p else "per-tile", th, w, z] for p, th, w, z in tiles])),
    }


def run_adjoint(torch, inputs, steps):
    """d loss / d (phi0, eps) through `steps` steps at 64^3 (eps = 0.1,
    s = 0.1, checkpoints every 5 steps), forward and adjoint to 1e-10."""
    from paper_1611_06288_amd.autograd import rollout
    p = inputs.adjoint_params(64)
    params = dict(n=p.n, L=p.L, dt=p.dt, tol=1e-10, max_cycles=1000, adj_tol=1e-10)
    phi0 = torch.from_numpy(inputs.adjoint_phi0(64, seed=5)).cuda()
    with torch.no_grad():
        tgt = rollout(torch.from_numpy(inputs.adjoint_phi0(64, seed=6)).cuda(),
                      torch.tensor(0.12, dtype=torch.float64), params, steps)
    # one untimed rollout and backward first: the adjoint kernels' first launches
    # (code-object loading) and the handle's first allocations stay out of the timing
    pw = phi0.clone().requires_grad_(True)
    ew = torch.tensor(p.eps, dtype=torch.float64, requires_grad=True)
    ((rollout(pw, ew, params, steps, ckpt_every=5) - tgt) ** 2).sum().backward()
    p0 = phi0.clone().requires_grad_(True)
    e = torch.tensor(p.eps, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = rollout(p0, e, params, steps, ckpt_every=5)
    loss = ((out - tgt) ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return {"n": 64, "steps": steps, "forward_s": round(t1 - t0, 4),
            "backward_s": round(t2 - t1, 4),
            "gradient_steps_per_s": round(steps / (t2 - t0), 3),
            "loss": float(loss.detach()), "dloss_deps": float(e.grad)}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


# Run by the one-core leg in a child process whose OpenMP runtime starts
# with one thread: one untimed cycle (first touch of the hierarchy), then
# `cycles` timed V(2,2) cycles of the first step of the workload.
_ONE_CORE_CHILD = """
import json, math, sys, time
sys.path.insert(0, sys.argv[1])
import numpy as np
from oracle import cfas
from paper_1611_06288_amd import inputs
n, cycles = int(sys.argv[2]), int(sys.argv[3])
p = inputs.polycrystal_params(n)
phi0 = inputs.polycrystal_256() if n == 256 else inputs.polycrystal_phi0(n, p.L, 8, seed=3)
h = p.L / n
f = cfas.source(phi0, phi0, h, p.eps)
mu, om = cfas.initial_guess(phi0, h, p.eps)
o = cfas.Solver(n, p.L, p.eps, p.dt, tol=p.tol)
u, _ = o.cycle(np.stack([phi0, mu, om]), f, phi0)
t0 = time.perf_counter()
for _ in range(cycles):
    u, _ = o.cycle(u, f, phi0)
dt = time.perf_counter() - t0
print(json.dumps({"threads": cfas.num_threads(), "seconds": dt, "cycles": cycles}))
"""


def cpu_oracle_legs(cfas, phi0, p, cycles, one_core_cycles, full_step):
    """Times the CPU oracle on the workload's first step: `cycles` V(2,2)
    cycles on every thread the oracle's OpenMP runtime uses, `one_core_cycles`
    on one thread (child process), and, with `full_step`, the whole first
    step on every thread.  Runs before the GPU is touched."""
    import numpy as np
    n = phi0.shape[0]
    h = p.L / n
    out = {"threads_all": cfas.num_threads(), "cpu_model": _cpu_model(),
           "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}
    f = cfas.source(phi0, phi0, h, p.eps)
    mu, om = cfas.initial_guess(phi0, h, p.eps)
    o = cfas.Solver(n, p.L, p.eps, p.dt, tol=p.tol)
    u, _ = o.cycle(np.stack([phi0, mu, om]), f, phi0)      # first touch, untimed
    t0 = time.perf_counter()
    for _ in range(cycles):
        u, _ = o.cycle(u, f, phi0)
    out["all_cycles"], out["all_seconds"] = cycles, time.perf_counter() - t0
    o.close()
    if one_core_cycles > 0:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", _ONE_CORE_CHILD, ROOT, str(n), str(one_core_cycles)],
                           env=env, capture_output=True, text=True, timeout=600)
        if r.returncode == 0:
            one = json.loads(r.stdout.strip().splitlines()[-1])
            out["one_threads"], out["one_cycles"], out["one_seconds"] = (
                one["threads"], one["cycles"], one["seconds"])
        else:
            out["one_core_error"] = r.stderr.strip()[-300:]
    if full_step:
        t0 = time.perf_counter()
        _, infos, _ = cfas.simulate(phi0, p.L, p.eps, p.dt, 1, tol=p.tol)
        out["full_step_seconds"] = time.perf_counter() - t0
        out["full_step_cycles"] = infos[0].cycles
    return out


def cpu_baseline(legs, cycles_per_step, n):
    """The bench line's cpu_baseline object from the timed legs: V-cycles/s
    on all threads, converted to steps/s with the GPU run's mean cycles per
    step over its timed steps (the oracle and the GPU take the same number
    of cycles per step: the parity tests require equal counts)."""
    cps = legs["all_cycles"] / legs["all_seconds"]
    res = {
        "value": cps / cycles_per_step,
        "unit": "time-steps/s",
        "v_cycles_per_s": cps,
        "cores": legs["threads_all"],
        "kind": "oracle",
        "cpu_model": legs["cpu_model"],
        "nproc": legs["nproc"],
        "affinity_cpus": legs["affinity_cpus"],
        "sample": (f"{legs['all_cycles']} V(2,2) cycles of the first step at {n}^3 on "
                   f"{legs['threads_all']} threads ({legs['all_seconds']:.1f} s), converted with "
                   f"the GPU run's mean of {cycles_per_step:.1f} cycles per timed step"),
    }
    if "one_seconds" in legs:
        c1 = legs["one_cycles"] / legs["one_seconds"]
        res["one_core"] = {"threads": legs["one_threads"], "v_cycles_per_s": c1,
                           "value": c1 / cycles_per_step,
                           "sample": f"{legs['one_cycles']} cycle(s) of the same step on one "
                                     f"thread ({legs['one_seconds']:.1f} s)"}
    elif "one_core_error" in legs:
        res["one_core"] = {"error": legs["one_core_error"]}
    if "full_step_seconds" in legs:
        res["first_step_in_full"] = {
            "seconds": legs["full_step_seconds"], "cycles": legs["full_step_cycles"],
            "steps_per_s": 1.0 / legs["full_step_seconds"],
            "v_cycles_per_s": legs["full_step_cycles"] / legs["full_step_seconds"]}
    return res


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on one GPU; more than one (--gpus > 1) is not "
              "implemented (the z-slab decomposition is a design note, not code)", file=sys.stderr)
        sys.exit(2)

    from paper_1611_06288_amd import inputs

    n = args.n
    p = inputs.polycrystal_params(n)
    phi0 = inputs.polycrystal_256() if n == 256 else inputs.polycrystal_phi0(n, p.L, 8, seed=3)
    # the CPU oracle legs run first, before anything touches the GPU (the
    # one-core leg is a child process)
    cpu_legs = None
    if args.cpu_cycles > 0 and not args.copy_probe:
        from oracle import cfas
        cpu_legs = cpu_oracle_legs(cfas, phi0, p, args.cpu_cycles, args.cpu_one_core_cycles,
                                   args.cpu_full_step)
        print(f"cpu oracle: {cpu_legs}", file=sys.stderr, flush=True)

    import torch

    from paper_1611_06288_amd import _lib as abi
    from paper_1611_06288_amd.solver import PFCError, Solver

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    abi.lib()   # fails loudly if the HIP library is not built
    if args.copy_probe:
        print(json.dumps({"copy_GBps": round(copy_ceiling(torch), 1), "bytes": 1 << 30}), flush=True)
        return
    ceiling = copy_ceiling(torch)

    ph = torch.from_numpy(phi0).cuda()
    boot = Solver(n, p.L, p.eps, p.dt, tol=p.tol)
    mu, om = boot.init_guess(ph)
    boot.close()
    state0 = (ph.clone(), ph.clone(), mu, om)
    torch.cuda.synchronize()

    fp64, phis64 = run_path(Solver, abi, torch, "fp64", state0, p, args.steps, args.warmup, args.cycle)
    print(f"fp64: {fp64['steps_per_s']:.3f} steps/s, cycles {fp64['cycles_per_step']}",
          file=sys.stderr, flush=True)

    fcyc = None
    if args.cycle == "V" and not args.no_fcycle:
        # the same steps solved to the same tolerance with F(2,2) cycles; on
        # this workload the point smoother is divergent on smooth modes and
        # the F-cycle's second coarse visit needs about a third of the cycles
        fres, phisf = run_path(Solver, abi, torch, "fp64", state0, p, args.steps, args.warmup, "F")
        fcyc = {
            "steps_per_s": round(fres["steps_per_s"], 4),
            "f_cycles_per_s": round(fres["v_cycles_per_s"], 3),
            "ms_per_step": round(fres["ms_per_step"], 3),
            "cycles_per_step": fres["cycles_per_step"],
            "speedup_vs_v_per_step": round(fres["steps_per_s"] / fp64["steps_per_s"], 4),
            "max_abs_diff_vs_v_per_step": [float((a - b).abs().max()) for a, b in zip(phisf, phis64)],
        }
        print(f"fp64 F-cycles: {fres['steps_per_s']:.3f} steps/s, cycles {fres['cycles_per_step']}",
              file=sys.stderr, flush=True)

    mixed = None
    if not args.no_mixed:
        try:
            mres, phism = run_path(Solver, abi, torch, "mixed", state0, p, args.steps, args.warmup,
                                   args.cycle)
            errs = [float((a - b).abs().max()) for a, b in zip(phism, phis64)]
            mixed = {
                "steps_per_s": round(mres["steps_per_s"], 4),
                "v_cycles_per_s": round(mres["v_cycles_per_s"], 3),
                "ms_per_step": round(mres["ms_per_step"], 3),
                "cycles_per_step": mres["cycles_per_step"],
                "speedup_vs_fp64_per_step": round(mres["steps_per_s"] / fp64["steps_per_s"], 4),
                "max_abs_err_vs_fp64_gpu_per_step": errs,
                "kernels": mres["kernels"],
            }
            print(f"mixed: {mres['steps_per_s']:.3f} steps/s", file=sys.stderr, flush=True)
        except PFCError as e:
            mixed = {"unavailable": str(e)}

    mobility = None
    if not args.no_mobility:
        # the same steps with the flux form of the first equation and face
        # mobility M = max(0.05, 1 - v^2) at the face average v of phi*
        mres, _ = run_path(Solver, abi, torch, "fp64", state0, p, args.steps, args.warmup,
                           args.cycle, mobility=MOBILITY)
        mobility = {
            "mobility": {"m0": MOBILITY[0], "m1": MOBILITY[1], "m2": MOBILITY[2],
                         "mmin": MOBILITY[3]},
            "steps_per_s": round(mres["steps_per_s"], 4),
            "v_cycles_per_s": round(mres["v_cycles_per_s"], 3),
            "ms_per_step": round(mres["ms_per_step"], 3),
            "cycles_per_step": mres["cycles_per_step"],
            "kernels": mres["kernels"],
        }
        print(f"variable mobility: {mres['steps_per_s']:.3f} steps/s, cycles "
              f"{mres['cycles_per_step']}", file=sys.stderr, flush=True)

    first = None
    if not args.no_first_order:
        # the first-order convex-splitting scheme on the same workload
        fres, _ = run_path(Solver, abi, torch, "fp64", state0, p, args.steps, args.warmup,
                           args.cycle, scheme=1)
        first = {
            "scheme": "first-order convex splitting",
            "steps_per_s": round(fres["steps_per_s"], 4),
            "v_cycles_per_s": round(fres["v_cycles_per_s"], 3),
            "ms_per_step": round(fres["ms_per_step"], 3),
            "cycles_per_step": fres["cycles_per_step"],
            "kernels": fres["kernels"],
        }
        print(f"first-order scheme: {fres['steps_per_s']:.3f} steps/s, cycles "
              f"{fres['cycles_per_step']}", file=sys.stderr, flush=True)

    loop = None
    if not args.no_loop:
        lres, cur_l = run_loop(Solver, torch, state0, p, args.steps, args.warmup, args.cycle)
        loop = {
            "steps_per_s": round(lres["steps_per_s"], 4),
            "ms_per_step": round(lres["ms_per_step"], 3),
            "cycles_per_step": lres["cycles_per_step"],
            "speedup_vs_step_loop": round(lres["steps_per_s"] / fp64["steps_per_s"], 4),
            "max_abs_diff_vs_step_loop": float((cur_l - phis64[-1]).abs().max()),
        }
        print(f"graph loop: {lres['steps_per_s']:.3f} steps/s", file=sys.stderr, flush=True)
        if args.long_steps > 0:
            loop["long_run"] = run_long(Solver, torch, inputs, args.long_steps,
                                        args.long_plain_steps)
            print(f"long run: {loop['long_run']['graph_loop_steps_per_s']} steps/s", file=sys.stderr,
                  flush=True)

    batched = run_batched(torch, inputs, args.batch_steps) if args.batch_steps > 0 else None
    if batched:
        print(f"batched: {batched['instance_steps_per_s']} instance-steps/s", file=sys.stderr, flush=True)
    adjoint = run_adjoint(torch, inputs, args.adjoint_steps) if args.adjoint_steps > 0 else None
    if adjoint:
        print(f"adjoint: {adjoint['gradient_steps_per_s']} steps/s", file=sys.stderr, flush=True)

    sm = fp64["kernels"].get("smooth0", {})
    achieved = sm.get("achieved_GBps")
    roofline = {
        "kernel": ("finest-level fused red-black sweep (one full sweep per launch; 64 B/pt, 56 "
                   "where the next sweep makes colour-0 mu, omega dead; mean over launches)"),
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
        "traffic": smoother_traffic_bytes(n),
        "copy_ceiling_GBps": round(ceiling, 1),
        "frac_of_copy_ceiling": round(achieved / ceiling, 4) if achieved else None,
        "alg_bytes_per_launch": sm.get("alg_bytes_per_launch"),
        "avg_launch_us": sm.get("avg_us"),
    }

    cpu = None
    if cpu_legs is not None:
        mean_cyc = sum(fp64["cycles_per_step"]) / len(fp64["cycles_per_step"])
        cpu = cpu_baseline(cpu_legs, mean_cyc, n)

    line = {
        "metric": METRIC,
        "value": round(fp64["steps_per_s"], 4),
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fp64["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"polycrystal {n}^3, 8 crystallites, h=pi/4, eps=0.25, s=0.5, "
                        f"{args.cycle}(2,2) to FP64 residual 1e-10",
            "n": n, "L": p.L, "eps": p.eps, "dt": p.dt, "tol": p.tol,
            "cycle": args.cycle, "nu1": p.nu1, "nu2": p.nu2, "parallelism": "single GPU",
        },
        "v_cycles_per_s": round(fp64["v_cycles_per_s"], 3),
        "cycles_per_step": fp64["cycles_per_step"],
        "kernels": fp64["kernels"],
        "fp64_fcycle": fcyc,
        "mixed": mixed,
        "variable_mobility": mobility,
        "first_order_scheme": first,
        "fp64_graph_loop": loop,
        "batched": batched,
        "adjoint": adjoint,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
