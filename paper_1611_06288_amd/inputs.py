"""Seeded synthetic inputs for the 3D phase field crystal (PFC) solver.

This module only builds initial density fields and run parameters; it holds
none of the scheme's arithmetic, so both the CPU oracle tests and the HIP path
can draw their inputs from it.

Grid convention (Section 2 of the paper, shifted to 0-based indices): a cubic
periodic box of side ``L`` with ``n`` cells per axis, spacing ``h = L / n``,
cell-centred values at ``x_i = (i + 1/2) h``.  Arrays are C-ordered
``[k][j][i]`` (z slowest, x fastest), FP64.

Random numbers come from ``numpy.random.Generator(PCG64(seed))`` and are drawn
in C order, so a given seed gives the same field on every machine.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def cell_centres(n: int, L: float):
    """Return (z, y, x) coordinate arrays of shape (n, n, n)."""
    h = L / n
    c = (np.arange(n, dtype=np.float64) + 0.5) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return z, y, x


@dataclasses.dataclass
class RunParams:
    """Parameters of one simulation, named as in the paper's problem statement."""

    n: int            # cells per axis (grid n^3)
    L: float          # box side
    eps: float        # epsilon in the PFC energy
    dt: float         # time step (tau in Section 3, s in Section 6)
    steps: int
    tol: float = 1e-10
    nu1: int = 2
    nu2: int = 2

    @property
    def h(self) -> float:
        return self.L / self.n


# --------------------------------------------------------------------------
# Smooth single-mode field plus noise (32^3 parity workload)
# --------------------------------------------------------------------------

def smooth_mode_phi0(n: int = 32, L: float = 32.0, seed: int = 1,
                     mean: float = 0.07, amp: float = 0.1,
                     noise: float = 0.01) -> np.ndarray:
    """mean + amp*sin(2 pi x/L) cos(2 pi y/L) sin(2 pi z/L) + noise*U(-1,1)."""
    z, y, x = cell_centres(n, L)
    k = 2.0 * math.pi / L
    phi = mean + amp * np.sin(k * x) * np.cos(k * y) * np.sin(k * z)
    if noise:
        phi = phi + noise * rng(seed).uniform(-1.0, 1.0, size=(n, n, n))
    return np.ascontiguousarray(phi)


def smooth_mode_params() -> RunParams:
    return RunParams(n=32, L=32.0, eps=0.025, dt=0.01, steps=10)


# --------------------------------------------------------------------------
# The paper's own initial data (Section 6)
# --------------------------------------------------------------------------

def paper_init1(n: int, L: float = 3.2) -> np.ndarray:
    """0.2 + 0.05 cos(2 pi x/3.2) cos(2 pi y/3.2) cos(2 pi z/3.2) (eqn init1)."""
    z, y, x = cell_centres(n, L)
    k = 2.0 * math.pi / 3.2
    return np.ascontiguousarray(0.2 + 0.05 * np.cos(k * x) * np.cos(k * y) * np.cos(k * z))


def paper_init2(n: int, seed: int) -> np.ndarray:
    """0.2 + 0.005 * U[0, 1] (eqn init2, the polycrystal start of Section 6.2)."""
    return np.ascontiguousarray(0.2 + 0.005 * rng(seed).uniform(0.0, 1.0, size=(n, n, n)))


# --------------------------------------------------------------------------
# Polycrystal seeds (128^3 and 256^3 workloads)
# --------------------------------------------------------------------------

def _rotation_from_quaternion(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def polycrystal_phi0(n: int, L: float, n_crystals: int, seed: int,
                     mean: float = 0.285, noise: float = 0.02, amp: float = 0.1,
                     radius_cells: float = 12.0,
                     q: float = 1.0 / math.sqrt(2.0)) -> np.ndarray:
    """Background ``mean + noise*U(-1,1)`` with spherical crystallites.

    Each crystallite has a centre drawn uniformly in [0, L)^3 and a uniformly
    random rotation (normalised Gaussian quaternion); inside radius
    ``radius_cells * h`` (minimum-image distance) the density is the one-mode
    BCC profile ``mean + amp*(cos qx'cos qy' + cos qx'cos qz' + cos qy'cos qz')``
    with ``x' = Rot (x - c)``.  Later crystallites overwrite earlier ones.
    """
    g = rng(seed)
    h = L / n
    phi = mean + noise * g.uniform(-1.0, 1.0, size=(n, n, n))
    coord = (np.arange(n, dtype=np.float64) + 0.5) * h
    R = radius_cells * h
    for _ in range(n_crystals):
        c = g.uniform(0.0, L, size=3)                 # (cx, cy, cz)
        rot = _rotation_from_quaternion(g.standard_normal(4))
        # candidate cells: the sphere's bounding box, wrapped (every cell
        # within the radius is in it); the formula is evaluated only there
        idx = []
        for ax in range(3):
            lo = int(math.floor((c[ax] - R) / h)) - 1
            hi = int(math.ceil((c[ax] + R) / h)) + 2
            idx.append(np.unique(np.arange(lo, hi) % n))
        ix, iy, iz = idx
        dx = (coord[ix] - c[0])[None, None, :]
        dy = (coord[iy] - c[1])[None, :, None]
        dz = (coord[iz] - c[2])[:, None, None]
        dx = dx - L * np.round(dx / L)
        dy = dy - L * np.round(dy / L)
        dz = dz - L * np.round(dz / L)
        inside = dx * dx + dy * dy + dz * dz <= R * R
        px = rot[0, 0] * dx + rot[0, 1] * dy + rot[0, 2] * dz
        py = rot[1, 0] * dx + rot[1, 1] * dy + rot[1, 2] * dz
        pz = rot[2, 0] * dx + rot[2, 1] * dy + rot[2, 2] * dz
        cx, cy, cz = np.cos(q * px), np.cos(q * py), np.cos(q * pz)
        crystal = mean + amp * (cx * cy + cx * cz + cy * cz)
        sub = phi[np.ix_(iz, iy, ix)]
        phi[np.ix_(iz, iy, ix)] = np.where(inside, crystal, sub)
    return np.ascontiguousarray(phi)


def polycrystal_params(n: int) -> RunParams:
    """h = pi/4, eps = 0.25, s = 0.5 (200 steps at 128^3, 100 at 256^3)."""
    return RunParams(n=n, L=n * math.pi / 4.0, eps=0.25, dt=0.5,
                     steps=200 if n <= 128 else 100)


def polycrystal_128() -> np.ndarray:
    return polycrystal_phi0(128, 128 * math.pi / 4.0, 3, seed=2)


def polycrystal_256() -> np.ndarray:
    return polycrystal_phi0(256, 256 * math.pi / 4.0, 8, seed=3)


# --------------------------------------------------------------------------
# Batched ensemble (64 instances of uneven n and epsilon)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Instance:
    params: RunParams
    phi_mean: float
    seed: int

    def phi0(self) -> np.ndarray:
        n = self.params.n
        return np.ascontiguousarray(
            self.phi_mean + 0.05 * rng(self.seed).uniform(-1.0, 1.0, size=(n, n, n)))


def batched_ensemble(count: int = 64, seed0: int = 1000,
                     sizes=(32, 48, 64, 96), steps: int = 50) -> List[Instance]:
    """Instance i draws (n, eps, mean) from seed ``seed0 + i``; L = n pi / 4."""
    out = []
    for i in range(count):
        g = rng(seed0 + i)
        n = int(sizes[int(g.integers(0, len(sizes)))])
        eps = float(g.uniform(0.02, 0.3))
        mean = float(g.uniform(0.05, 0.3))
        p = RunParams(n=n, L=n * math.pi / 4.0, eps=eps, dt=0.1, steps=steps)
        # the field itself uses a derived seed so that it does not reuse the
        # parameter stream
        out.append(Instance(params=p, phi_mean=mean, seed=10_000_000 + seed0 + i))
    return out


# --------------------------------------------------------------------------
# Adjoint workload (64^3)
# --------------------------------------------------------------------------

def adjoint_params(n: int = 64) -> RunParams:
    return RunParams(n=n, L=n * math.pi / 4.0, eps=0.1, dt=0.1, steps=20)


def adjoint_phi0(n: int = 64, seed: int = 5) -> np.ndarray:
    return np.ascontiguousarray(0.2 + 0.05 * rng(seed).uniform(-1.0, 1.0, size=(n, n, n)))


def unit_direction(shape, seed: int = 7) -> np.ndarray:
    v = rng(seed).standard_normal(shape)
    return np.ascontiguousarray(v / np.linalg.norm(v))


def random_field(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.ascontiguousarray(rng(seed).uniform(lo, hi, size=(n, n, n)))
