"""ctypes binding to the C oracle (``pfc_oracle.c``).  Test infrastructure only.

Every function takes and returns numpy FP64 arrays in C order ``[k][j][i]``;
a triple ``u`` is an array of shape ``(3, n, n, n)`` ordered (phi, mu, omega).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import build as _build

_lib = None
_dp = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(force=True)
        L = C.CDLL(path)
        d, i, vp = C.c_double, C.c_int, C.c_void_p
        L.orc_laplacian.argtypes = [i, d, _dp, _dp]
        L.orc_apply_N.argtypes = [i, d, d, d, _dp, _dp, _dp]
        L.orc_source.argtypes = [i, d, d, _dp, _dp, _dp]
        L.orc_residual.argtypes = [i, d, d, d, _dp, _dp, _dp, _dp]
        L.orc_residual.restype = d
        L.orc_local_solve.argtypes = [d, d, d, i, d, d, d, d, d, d, d, d, _dp, _dp, _dp]
        L.orc_smooth_half.argtypes = [i, d, d, d, i, i, _dp, _dp, _dp]
        L.orc_sweep.argtypes = [i, d, d, d, i, _dp, _dp, _dp]
        L.orc_restrict.argtypes = [i, _dp, _dp]
        L.orc_prolong_add.argtypes = [i, _dp, _dp]
        L.orc_coarse_solve.argtypes = [i, d, d, d, _dp, _dp, _dp]
        L.orc_coarse_solve.restype = i
        L.orc_num_levels.argtypes = [i]
        L.orc_num_levels.restype = i
        L.orc_create.argtypes = [i, d, d, d, d, i, i, i, i, i]
        L.orc_create.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_level_n.argtypes = [vp, i]
        L.orc_level_n.restype = i
        L.orc_levels.argtypes = [vp]
        L.orc_levels.restype = i
        L.orc_cycle.argtypes = [vp, _dp, _dp, _dp]
        L.orc_cycle.restype = d
        L.orc_step.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, C.POINTER(C.c_int), _dp]
        L.orc_step.restype = i
        L.orc_initial_guess.argtypes = [i, d, d, _dp, _dp, _dp]
        L.orc_energy.argtypes = [i, d, d, _dp, _dp, _dp]
        L.orc_num_threads.restype = i
        mob = [d, d, d, d]
        L.orc_apply_N_m.argtypes = [i, d, d, d, _dp, _dp, _dp] + mob + [_dp]
        L.orc_residual_m.argtypes = [i, d, d, d, _dp, _dp, _dp, _dp] + mob + [_dp]
        L.orc_residual_m.restype = d
        L.orc_local_solve_m.argtypes = [d, d, d, i, d, d, d, d, d, d, d, d, d, _dp, _dp, _dp]
        L.orc_smooth_half_m.argtypes = [i, d, d, d, i, i, _dp, _dp, _dp, _dp] + mob
        L.orc_coarse_solve_m.argtypes = [i, d, d, d, _dp, _dp, _dp, _dp] + mob
        L.orc_coarse_solve_m.restype = i
        L.orc_set_mobility.argtypes = [vp] + mob
        L.orc_cycle_m.argtypes = [vp, _dp, _dp, _dp, _dp]
        L.orc_cycle_m.restype = d
        L.orc_apply_N_fo.argtypes = [i, d, d, d, _dp, _dp]
        L.orc_source_fo.argtypes = [i, d, _dp, _dp]
        L.orc_residual_fo.argtypes = [i, d, d, d, _dp, _dp, _dp]
        L.orc_residual_fo.restype = d
        L.orc_local_solve_fo.argtypes = [d, d, d, i, d, d, d, d, d, d, d, _dp, _dp, _dp]
        L.orc_smooth_half_fo.argtypes = [i, d, d, d, i, i, _dp, _dp]
        L.orc_coarse_solve_fo.argtypes = [i, d, d, d, _dp, _dp]
        L.orc_coarse_solve_fo.restype = i
        L.orc_set_first_order.argtypes = [vp]
        L.orc_set_first_order.restype = i
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    """OpenMP threads used by the oracle's parallel loops."""
    return lib().orc_num_threads()


def num_levels(n: int) -> int:
    return lib().orc_num_levels(n)


def laplacian(v, h):
    v = _f64(v)
    out = np.empty_like(v)
    lib().orc_laplacian(v.shape[0], h, _p(v), _p(out))
    return out


def apply_N(u, phk, h, eps, tau):
    u, phk = _f64(u), _f64(phk)
    out = np.empty_like(u)
    lib().orc_apply_N(phk.shape[0], h, eps, tau, _p(u), _p(phk), _p(out))
    return out


def source(phk, phkm1, h, eps):
    phk, phkm1 = _f64(phk), _f64(phkm1)
    n = phk.shape[0]
    f = np.empty((3, n, n, n))
    lib().orc_source(n, h, eps, _p(phk), _p(phkm1), _p(f))
    return f


def residual(u, f, phk, h, eps, tau):
    """Returns (r, max|r|)."""
    u, f, phk = _f64(u), _f64(f), _f64(phk)
    r = np.empty_like(u)
    m = lib().orc_residual(phk.shape[0], h, eps, tau, _p(u), _p(f), _p(phk), _p(r))
    return r, m


def local_solve(h, eps, tau, picard, phin, phk, f1, f2, f3, smu, som, sphi):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().orc_local_solve(h, eps, tau, int(picard), phin, phk, f1, f2, f3, smu, som, sphi,
                          C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def smooth_half(u, f, phk, h, eps, tau, colour, picard=False):
    u = _f64(u).copy()
    f, phk = _f64(f), _f64(phk)
    lib().orc_smooth_half(phk.shape[0], h, eps, tau, int(picard), int(colour), _p(u), _p(f), _p(phk))
    return u


def restrict(fine):
    fine = _f64(fine)
    nf = fine.shape[-1]
    if fine.ndim == 4:
        return np.stack([restrict(fine[c]) for c in range(fine.shape[0])])
    out = np.empty((nf // 2,) * 3)
    lib().orc_restrict(nf, _p(fine), _p(out))
    return out


def prolong_add(ec, fine):
    """Returns fine + P ec (inputs untouched)."""
    ec = _f64(ec)
    fine = _f64(fine).copy()
    if ec.ndim == 4:
        for c in range(ec.shape[0]):
            fc = np.ascontiguousarray(fine[c])
            lib().orc_prolong_add(ec.shape[-1], _p(np.ascontiguousarray(ec[c])), _p(fc))
            fine[c] = fc
        return fine
    lib().orc_prolong_add(ec.shape[-1], _p(ec), _p(fine))
    return fine


def coarse_solve(u, f, phk, h, eps, tau):
    u = _f64(u).copy()
    f, phk = _f64(f), _f64(phk)
    it = lib().orc_coarse_solve(phk.shape[0], h, eps, tau, _p(u), _p(f), _p(phk))
    return u, it


# ------------------------------------------------------------------
# Variable mobility M(v) = max(mmin, m0 + m1 v + m2 v^2) on the faces,
# evaluated at the face average of phi* (mob = (m0, m1, m2, mmin)).

def apply_N_m(u, phk, phs, h, eps, tau, mob):
    u, phk, phs = _f64(u), _f64(phk), _f64(phs)
    out = np.empty_like(u)
    lib().orc_apply_N_m(phk.shape[0], h, eps, tau, _p(u), _p(phk), _p(phs), *mob, _p(out))
    return out


def residual_m(u, f, phk, phs, h, eps, tau, mob):
    """Returns (r, max|r|)."""
    u, f, phk, phs = _f64(u), _f64(f), _f64(phk), _f64(phs)
    r = np.empty_like(u)
    m = lib().orc_residual_m(phk.shape[0], h, eps, tau, _p(u), _p(f), _p(phk), _p(phs), *mob, _p(r))
    return r, m


def local_solve_m(h, eps, tau, picard, phin, phk, f1, f2, f3, msum, smu, som, sphi):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().orc_local_solve_m(h, eps, tau, int(picard), phin, phk, f1, f2, f3, msum, smu, som, sphi,
                            C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def smooth_half_m(u, f, phk, phs, h, eps, tau, colour, mob, picard=False):
    u = _f64(u).copy()
    f, phk, phs = _f64(f), _f64(phk), _f64(phs)
    lib().orc_smooth_half_m(phk.shape[0], h, eps, tau, int(picard), int(colour), _p(u), _p(f),
                            _p(phk), _p(phs), *mob)
    return u


def coarse_solve_m(u, f, phk, phs, h, eps, tau, mob):
    u = _f64(u).copy()
    f, phk, phs = _f64(f), _f64(phk), _f64(phs)
    it = lib().orc_coarse_solve_m(phk.shape[0], h, eps, tau, _p(u), _p(f), _p(phk), _p(phs), *mob)
    return u, it


# ------------------------------------------------------------------
# First-order convex-splitting scheme: N1 = phi - tau Lap mu,
# N2 = mu - phi^3 - (1-eps) phi - Lap omega, N3 = omega - Lap phi;
# S = (phi^k, 2 Lap phi^k, 0).

def apply_N_fo(u, h, eps, tau):
    u = _f64(u)
    out = np.empty_like(u)
    lib().orc_apply_N_fo(u.shape[1], h, eps, tau, _p(u), _p(out))
    return out


def source_fo(phk, h):
    phk = _f64(phk)
    f = np.empty((3,) + phk.shape)
    lib().orc_source_fo(phk.shape[0], h, _p(phk), _p(f))
    return f


def residual_fo(u, f, h, eps, tau):
    """Returns (r, max|r|)."""
    u, f = _f64(u), _f64(f)
    r = np.empty_like(u)
    m = lib().orc_residual_fo(u.shape[1], h, eps, tau, _p(u), _p(f), _p(r))
    return r, m


def local_solve_fo(h, eps, tau, picard, phin, f1, f2, f3, smu, som, sphi):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().orc_local_solve_fo(h, eps, tau, int(picard), phin, f1, f2, f3, smu, som, sphi,
                             C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def smooth_half_fo(u, f, h, eps, tau, colour, picard=False):
    u = _f64(u).copy()
    f = _f64(f)
    lib().orc_smooth_half_fo(u.shape[1], h, eps, tau, int(picard), int(colour), _p(u), _p(f))
    return u


def coarse_solve_fo(u, f, h, eps, tau):
    u = _f64(u).copy()
    f = _f64(f)
    it = lib().orc_coarse_solve_fo(u.shape[1], h, eps, tau, _p(u), _p(f))
    return u, it


def initial_guess(phi0, h, eps):
    phi0 = _f64(phi0)
    mu = np.empty_like(phi0)
    om = np.empty_like(phi0)
    lib().orc_initial_guess(phi0.shape[0], h, eps, _p(phi0), _p(mu), _p(om))
    return mu, om


def energy(phi, h, eps, phi_prev=None):
    """Returns (F_h(phi), F_h(phi) + 1/2|grad_h(phi - phi_prev)|^2, mass)."""
    phi = _f64(phi)
    pp = None if phi_prev is None else _f64(phi_prev)
    out = np.zeros(3)
    lib().orc_energy(phi.shape[0], h, eps, _p(phi), _p(pp), _p(out))
    return float(out[0]), float(out[1]), float(out[2])


class OracleError(RuntimeError):
    pass


@dataclass
class StepInfo:
    status: int
    cycles: int
    res_hist: List[float] = field(default_factory=list)


class Solver:
    """FAS solver of one time step of scheme (1.10) (C oracle); ``mobility``
    selects the variable-mobility flux form, ``scheme=1`` the first-order
    convex-splitting scheme."""

    def __init__(self, n, L, eps, dt, tol=1e-10, nu1=2, nu2=2, max_cycles=200,
                 cycle="V", lin="newton", mobility=None, scheme=2):
        self.n, self.L, self.eps, self.dt, self.tol = n, L, eps, dt, tol
        self.h = L / n
        self.max_cycles = max_cycles
        self._s = lib().orc_create(n, L, eps, dt, tol, nu1, nu2, max_cycles,
                                   1 if cycle == "F" else 0, 1 if lin == "picard" else 0)
        if not self._s:
            raise OracleError(f"invalid oracle configuration n={n}")
        self.mobility = mobility
        if mobility is not None:
            lib().orc_set_mobility(self._s, *[float(x) for x in mobility])
        self.scheme = scheme
        if scheme == 1 and lib().orc_set_first_order(self._s) != 0:
            raise OracleError("the first-order scheme has constant mobility only")

    def close(self):
        if self._s:
            lib().orc_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def levels(self):
        return [lib().orc_level_n(self._s, l) for l in range(lib().orc_levels(self._s))]

    def cycle(self, u, f, phk, phs=None):
        """One cycle from (u, f, phk) (and phi* with variable mobility);
        returns (u_new, residual after)."""
        u = _f64(u).copy()
        f, phk = _f64(f), _f64(phk)
        if self.mobility is not None:
            res = lib().orc_cycle_m(self._s, _p(u), _p(f), _p(phk), _p(_f64(phs)))
        else:
            res = lib().orc_cycle(self._s, _p(u), _p(f), _p(phk))
        return u, res

    def step(self, phkm1, phk, mu, omega):
        """One time step; returns (phi_next, mu, omega, StepInfo)."""
        phkm1, phk = _f64(phkm1), _f64(phk)
        mu, omega = _f64(mu).copy(), _f64(omega).copy()
        out = np.empty_like(phk)
        cyc = C.c_int(0)
        hist = np.zeros(self.max_cycles + 2)
        st = lib().orc_step(self._s, _p(phkm1), _p(phk), _p(out), _p(mu), _p(omega),
                            C.byref(cyc), _p(hist))
        info = StepInfo(status=st, cycles=cyc.value, res_hist=list(hist[:cyc.value + 1]))
        return out, mu, omega, info


def simulate(phi0, L, eps, dt, steps, tol=1e-10, nu1=2, nu2=2, cycle="V", lin="newton",
             max_cycles=400, callback=None, mobility=None, scheme=2):
    """Runs `steps` time steps from phi0 with the bootstrap phi^{-1} = phi^0.

    Returns (list of phi^0..phi^steps, list of StepInfo, final (mu, omega))."""
    n = phi0.shape[0]
    s = Solver(n, L, eps, dt, tol, nu1, nu2, max_cycles, cycle, lin, mobility, scheme)
    mu, om = initial_guess(phi0, L / n, eps)
    phis = [_f64(phi0).copy()]
    infos = []
    prev, cur = phis[0], phis[0]
    for k in range(steps):
        nxt, mu, om, info = s.step(prev, cur, mu, om)
        if info.status != 0:
            raise OracleError(f"oracle step {k} status {info.status}")
        infos.append(info)
        phis.append(nxt)
        if callback:
            callback(k, nxt, mu, om, info)
        prev, cur = cur, nxt
    s.close()
    return phis, infos, (mu, om)
