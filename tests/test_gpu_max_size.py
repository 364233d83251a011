"""The largest grids the library accepts: one time step at 512^3 and at
1024^3 (the size limit), checked against the oracle.

Input: a 32^3 polycrystal (2 crystallites of radius 4h, seed 9; h = pi/4,
eps = 0.25, tau = 0.5, tol = 1e-10) tiled T times along each axis, i.e. a
field of period 32 cells on the (32 T)^3 grid with L = 32 T h.  The discrete
operator of scheme (1.10) commutes with periodic shifts, the red-black
colouring and the 8-child coarsening keep a period of 32 cells (32 is even
at every level down to a period of one cell), so the step from the tiled
input is the tiled step of the 32^3 problem, which the oracle computes in a
second.  The oracle itself was checked the same way on the CPU (64^3 tiled
from 32^3: the same 72 cycles, fields equal to 1e-14).

What is checked at the large sizes:
  * status OK and a final max-norm residual at or below tol;
  * the result is periodic: every 32^3 tile equals the first to within
    1e-13 relative (measured: bit for bit; the bar allows the coarsest
    dense solve to round differently at points that are images of each
    other once a level's period is one cell);
  * the first tile equals the oracle's 32^3 step to 1e-11 relative when the
    cycle counts agree (the FP64 bar of every other step test), else to
    1e-9 (two solves stopped at tol = 1e-10 sit within about 4e-11 of the
    exact step at this size, measured with the oracle at tol 1e-13);
  * energy, modified energy and mass equal T^3 times the oracle's.
An indexing error at a large size (an overflow, a tile or plane range)
breaks the periodicity or the agreement by far more than these bars.
The 1024^3 case needs about 180 GB of device memory and is skipped with a
message on a device with less free memory.
"""
import gc
import math

import pytest
import torch

from paper_1611_06288_amd import inputs

pytestmark = pytest.mark.gpu

BASE = 32
H = math.pi / 4.0
EPS, DT, TOL = 0.25, 0.5, 1e-10


@pytest.fixture(scope="module")
def base_step():
    from oracle import cfas
    L = BASE * H
    phi0 = inputs.polycrystal_phi0(BASE, L, 2, seed=9, radius_cells=4)
    phis, infos, (mu, om) = cfas.simulate(phi0, L, EPS, DT, 1, tol=TOL)
    energy = cfas.energy(phis[1], H, EPS, phi_prev=phi0)
    return phi0, (phis[1], mu, om), infos[0], energy


def rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def free_device_bytes():
    gc.collect()
    torch.cuda.empty_cache()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("T,precision", [(16, "fp64"), (16, "mixed"), (32, "fp64")])
def test_tiled_step_at_the_largest_sizes(base_step, T, precision):
    from paper_1611_06288_amd import Solver
    n = BASE * T
    need = (180 if n == 1024 else 30) * 2**30
    free = free_device_bytes()
    if free < need:
        pytest.skip(f"{n}^3 needs about {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} free")
    phi0, want, oinfo, oenergy = base_step
    print(f"n = {n} ({precision}): tiling the 32^3 input {T}x per axis", flush=True)
    ph = torch.from_numpy(phi0).cuda().repeat(T, T, T)
    s = Solver(n, n * H, EPS, DT, tol=TOL, precision=precision)
    try:
        mu, om = s.init_guess(ph)
        nxt, info = s.step(ph, ph, mu, om)
        torch.cuda.synchronize()
        print(f"n = {n} ({precision}): cycles {info.cycles} (oracle at 32^3: {oinfo.cycles}), "
              f"residual {info.res_final:.3e}", flush=True)
        assert info.status == 0 and info.res_final <= TOL
        same = info.cycles == oinfo.cycles
        bar = 1e-11 if same else 1e-9
        for name, got, ref in zip(("phi", "mu", "omega"), (nxt, mu, om), want):
            tiles = got.view(T, BASE, T, BASE, T, BASE)
            first = tiles[0, :, 0, :, 0, :]
            per = float((tiles - first[None, :, None, :, None, :]).abs().max() / first.abs().max())
            err = rel(first.cpu(), torch.from_numpy(ref))
            print(f"  {name}: periodicity {per:.2e}, first tile vs oracle {err:.2e}", flush=True)
            assert per <= 1e-13, (name, per)
            assert err <= bar, (name, err, bar)
            del tiles, first
        F, Ft, m = s.energy(nxt, ph)
        scale = T ** 3
        for label, got, ref in (("energy", F, oenergy[0]), ("energy_mod", Ft, oenergy[1]),
                                ("mass", m, oenergy[2])):
            r = abs(got - scale * ref) / abs(scale * ref)
            print(f"  {label}: {got:.12e} vs {scale} x oracle, relative {r:.2e}", flush=True)
            assert r <= (1e-11 if same else 1e-9), (label, r)
    finally:
        s.close()
        del ph
        gc.collect()
        torch.cuda.empty_cache()
