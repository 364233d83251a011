"""Python front end of the HIP solver: torch tensors in, device pointers out.

Only argument marshalling happens here; every step of the method runs in the
HIP kernels of ``libpfc_hip.so`` on the stream torch currently uses.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import torch

from . import _lib as abi


class PFCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


@dataclasses.dataclass
class StepInfo:
    cycles: int
    status: int
    res0: float
    res_final: float


def _ptr(t: Optional[torch.Tensor], numel: int, name: str):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return C.c_void_p(t.data_ptr())


class Solver:
    """One time step of scheme (1.10) by FAS multigrid on an n^3 periodic grid.

    Parameters follow the paper's statement of the problem: n, L, eps, time
    step dt, residual tolerance tol, smoothing counts nu1/nu2.  ``mobility``
    (m0, m1, m2, mmin) selects the flux form of the first equation with face
    mobility M(v) = max(mmin, m0 + m1 v + m2 v^2) at the face average v of
    phi* = 3/2 phi^k - 1/2 phi^{k-1}; None is M = 1.  ``scheme`` 2 is scheme
    (1.10), 1 the first-order convex splitting (phi_prev then unused)."""

    def __init__(self, n: int, L: float, eps: float, dt: float, tol: float = 1e-10,
                 nu1: int = 2, nu2: int = 2, max_cycles: int = 400, cycle: str = "V",
                 lin: str = "newton", precision: str = "fp64", device=None, mobility=None,
                 scheme: int = 2):
        if not torch.cuda.is_available():
            raise RuntimeError("the PFC solver needs a GPU (torch.cuda.is_available() is False)")
        self.lib = abi.lib()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.n, self.L, self.eps, self.dt, self.tol = n, float(L), float(eps), float(dt), float(tol)
        self.h = self.L / n
        self.P = n ** 3
        cfg = abi.PfcConfig()
        cfg.n, cfg.nu1, cfg.nu2, cfg.max_cycles = n, nu1, nu2, max_cycles
        cfg.cycle = {"V": abi.PFC_CYCLE_V, "F": abi.PFC_CYCLE_F}[cycle]
        cfg.lin = {"newton": abi.PFC_LIN_NEWTON, "picard": abi.PFC_LIN_PICARD}[lin]
        cfg.precision = {"fp64": abi.PFC_FP64, "mixed": abi.PFC_MIXED}[precision]
        cfg.L, cfg.eps, cfg.dt, cfg.tol = self.L, self.eps, self.dt, self.tol
        cfg.scheme = {2: abi.PFC_SCHEME_CS2, 1: abi.PFC_SCHEME_CS1}[scheme]
        self.scheme = scheme
        self.mobility = None if mobility is None else tuple(float(x) for x in mobility)
        if self.mobility is None:
            cfg.mobility = abi.PFC_MOBILITY_ONE
        else:
            cfg.mobility = abi.PFC_MOBILITY_QUADRATIC
            cfg.mob_m0, cfg.mob_m1, cfg.mob_m2, cfg.mob_min = self.mobility
        self.cfg = cfg
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            st = self.lib.pfc_create(C.byref(cfg), C.c_void_p(stream), C.byref(self._h))
        if st != abi.PFC_OK:
            raise PFCError(st, self.lib.pfc_last_error(None).decode())

    # ---------------------------------------------------------------- utils
    def _check(self, st: int):
        if st != abi.PFC_OK:
            raise PFCError(st, self.lib.pfc_last_error(self._h).decode())

    def _sync_stream(self):
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self.lib.pfc_set_stream(self._h, C.c_void_p(stream))

    def close(self):
        if self._h:
            self.lib.pfc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def levels(self):
        return [self.lib.pfc_level_size(self._h, l) for l in range(self.lib.pfc_num_levels(self._h))]

    def field(self, n: Optional[int] = None, comps: int = 1) -> torch.Tensor:
        n = self.n if n is None else n
        shape = (n, n, n) if comps == 1 else (comps, n, n, n)
        return torch.empty(shape, dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------- method
    def init_guess(self, phi0: torch.Tensor):
        self._sync_stream()
        mu, om = torch.empty_like(phi0), torch.empty_like(phi0)
        self._check(self.lib.pfc_init_guess(self._h, _ptr(phi0, self.P, "phi0"),
                                            _ptr(mu, self.P, "mu"), _ptr(om, self.P, "omega")))
        return mu, om

    def step(self, phi_prev, phi_cur, mu, omega, out=None, raise_on_error=True):
        """Returns (phi_next, StepInfo); mu and omega are updated in place."""
        self._sync_stream()
        if out is None:
            out = torch.empty_like(phi_cur)
        info = abi.PfcStepInfo()
        st = self.lib.pfc_step(self._h, _ptr(phi_prev, self.P, "phi_prev"),
                               _ptr(phi_cur, self.P, "phi_cur"), _ptr(out, self.P, "phi_next"),
                               _ptr(mu, self.P, "mu"), _ptr(omega, self.P, "omega"), C.byref(info))
        si = StepInfo(info.cycles, info.status, info.res0, info.res_final)
        if raise_on_error and st != abi.PFC_OK:
            self._check(st)
        return out, si

    def run(self, phi_prev, phi_cur, mu, omega, steps, raise_on_error=True):
        """Advances (phi_prev, phi_cur, mu, omega) in place by `steps` steps of
        the graph-driven time loop; returns the list of StepInfo."""
        self._sync_stream()
        infos = (abi.PfcStepInfo * max(1, steps))()
        P = self.P
        st = self.lib.pfc_run(self._h, _ptr(phi_prev, P, "phi_prev"), _ptr(phi_cur, P, "phi_cur"),
                              _ptr(mu, P, "mu"), _ptr(omega, P, "omega"), int(steps), infos)
        out = [StepInfo(i.cycles, i.status, i.res0, i.res_final) for i in infos[:steps]]
        if raise_on_error and st != abi.PFC_OK:
            self._check(st)
        return out

    def vcycle(self, u3, f3, phi_cur):
        """One multigrid cycle in place on u3; returns the residual after it."""
        self._sync_stream()
        res = C.c_double()
        self._check(self.lib.pfc_fas_vcycle(self._h, _ptr(u3, 3 * self.P, "u3"),
                                            _ptr(f3, 3 * self.P, "f3"),
                                            _ptr(phi_cur, self.P, "phi_cur"), C.byref(res)))
        return res.value

    def energy(self, phi, phi_prev=None):
        self._sync_stream()
        out = (C.c_double * 3)()
        self._check(self.lib.pfc_energy(self._h, _ptr(phi, self.P, "phi"),
                                        _ptr(phi_prev, self.P, "phi_prev"), out))
        return out[0], out[1], out[2]

    def adjoint_step(self, phi_prev, phi_cur, phi_next, gbar_next, gbar_cur, gbar_prev, geps,
                     adj_tol=1e-12):
        """Accumulates the step's adjoint into gbar_cur, gbar_prev and geps (1-element)."""
        self._sync_stream()
        cyc = C.c_int32()
        P = self.P
        self._check(self.lib.pfc_adjoint_step(
            self._h, _ptr(phi_prev, P, "phi_prev"), _ptr(phi_cur, P, "phi_cur"),
            _ptr(phi_next, P, "phi_next"), _ptr(gbar_next, P, "gbar_next"),
            _ptr(gbar_cur, P, "gbar_cur"), _ptr(gbar_prev, P, "gbar_prev"),
            _ptr(geps, 1, "geps"), float(adj_tol), C.byref(cyc)))
        return cyc.value

    def simulate(self, phi0: torch.Tensor, steps: int, callback=None):
        """Runs `steps` steps from phi0 with phi^{-1} = phi^0 and the first-step
        guess of init_guess.  Returns (phi_prev, phi_cur, mu, omega, infos)."""
        mu, om = self.init_guess(phi0)
        prev, cur = phi0.clone(), phi0.clone()
        spare = torch.empty_like(phi0)
        infos = []
        for k in range(steps):
            nxt, info = self.step(prev, cur, mu, om, out=spare)
            infos.append(info)
            if callback:
                callback(k, nxt, mu, om, info)
            spare = prev
            prev, cur = cur, nxt
        return prev, cur, mu, om, infos

    # ------------------------------------------------- kernel-level access
    def level_n(self, level):
        return self.lib.pfc_level_size(self._h, level)

    def source(self, phi_prev, phi_cur):
        self._sync_stream()
        f3 = self.field(comps=3)
        self._check(self.lib.pfc_source(self._h, _ptr(phi_prev, self.P, "phi_prev"),
                                        _ptr(phi_cur, self.P, "phi_cur"), _ptr(f3, 3 * self.P, "f3")))
        return f3

    def residual(self, level, u3, f3, phk, want_r=True):
        self._sync_stream()
        n = self.level_n(level)
        P = n ** 3
        r = self.field(n, 3) if want_r else None
        m = C.c_double()
        self._check(self.lib.pfc_residual(self._h, level, _ptr(u3, 3 * P, "u3"), _ptr(f3, 3 * P, "f3"),
                                          _ptr(phk, P, "phk"), _ptr(r, 3 * P, "r3"), C.byref(m)))
        return r, m.value

    def smooth(self, level, colour, u3, f3, phk):
        self._sync_stream()
        P = self.level_n(level) ** 3
        self._check(self.lib.pfc_smooth(self._h, level, colour, _ptr(u3, 3 * P, "u3"),
                                        _ptr(f3, 3 * P, "f3"), _ptr(phk, P, "phk")))

    def restrict(self, level, fine, ncomp):
        self._sync_stream()
        nf, nc = self.level_n(level), self.level_n(level + 1)
        coarse = self.field(nc, ncomp)
        self._check(self.lib.pfc_restrict(self._h, level, _ptr(fine, ncomp * nf ** 3, "fine"),
                                          _ptr(coarse, ncomp * nc ** 3, "coarse"), ncomp))
        return coarse

    def prolong_add(self, level, coarse_v, coarse_ubar, fine, ncomp):
        self._sync_stream()
        nf, nc = self.level_n(level), self.level_n(level + 1)
        self._check(self.lib.pfc_prolong_add(self._h, level, _ptr(coarse_v, ncomp * nc ** 3, "v"),
                                             _ptr(coarse_ubar, ncomp * nc ** 3, "ubar"),
                                             _ptr(fine, ncomp * nf ** 3, "fine"), ncomp))

    def reset_coarse_cache(self):
        """Forgets the cached coarsest Newton inverse (``pfc_reset_coarse_cache``)."""
        self._sync_stream()
        self._check(self.lib.pfc_reset_coarse_cache(self._h))

    def set_phistar(self, level, phs):
        """Variable mobility: phi* at `level` (and its 8-child means below)."""
        self._sync_stream()
        P = self.level_n(level) ** 3
        self._check(self.lib.pfc_set_phistar(self._h, level, _ptr(phs, P, "phs")))

    def coarse_solve(self, u3, f3, phk):
        self._sync_stream()
        nc = self.levels[-1]
        P = nc ** 3
        it = C.c_int32()
        self._check(self.lib.pfc_coarse_solve(self._h, _ptr(u3, 3 * P, "u3"), _ptr(f3, 3 * P, "f3"),
                                              _ptr(phk, P, "phk"), C.byref(it)))
        return it.value

    # ------------------------------------------------------ instrumentation
    def timing(self, on: bool):
        self._check(self.lib.pfc_timing_enable(self._h, 1 if on else 0))

    def timing_reset(self):
        self._check(self.lib.pfc_timing_reset(self._h))

    def timing_get(self, kernel: int):
        cnt, ms, b = C.c_int64(), C.c_double(), C.c_double()
        self._check(self.lib.pfc_timing_get(self._h, kernel, C.byref(cnt), C.byref(ms), C.byref(b)))
        return cnt.value, ms.value, b.value


class Batch:
    """Many independent simulations advanced together (``pfc_batch_*``).

    ``instances``: list of dicts with keys n, L, eps, dt.  The cycle
    parameters (tol, nu1, nu2, cycle, lin, max_cycles) are shared."""

    def __init__(self, instances, tol=1e-10, nu1=2, nu2=2, max_cycles=400, cycle="V",
                 lin="newton", device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the PFC solver needs a GPU (torch.cuda.is_available() is False)")
        self.lib = abi.lib()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.count = len(instances)
        self.sizes = [int(p["n"]) for p in instances]
        cfgs = (abi.PfcConfig * self.count)()
        for c, p in zip(cfgs, instances):
            c.n, c.nu1, c.nu2, c.max_cycles = int(p["n"]), nu1, nu2, max_cycles
            c.cycle = {"V": abi.PFC_CYCLE_V, "F": abi.PFC_CYCLE_F}[cycle]
            c.lin = {"newton": abi.PFC_LIN_NEWTON, "picard": abi.PFC_LIN_PICARD}[lin]
            c.precision, c.mobility = abi.PFC_FP64, abi.PFC_MOBILITY_ONE
            c.L, c.eps, c.dt, c.tol = float(p["L"]), float(p["eps"]), float(p["dt"]), float(tol)
        self._b = C.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        st = self.lib.pfc_batch_create(self.count, cfgs, C.c_void_p(stream), C.byref(self._b))
        if st != abi.PFC_OK:
            raise PFCError(st, self.lib.pfc_batch_last_error(None).decode())

    def _check(self, st):
        if st != abi.PFC_OK:
            raise PFCError(st, self.lib.pfc_batch_last_error(self._b).decode())

    def close(self):
        if self._b:
            self.lib.pfc_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_state(self, i, phi0):
        self._check(self.lib.pfc_batch_init_state(self._b, i, _ptr(phi0, self.sizes[i] ** 3, "phi0")))

    def set_state(self, i, phi_prev, phi_cur, mu, omega):
        P = self.sizes[i] ** 3
        self._check(self.lib.pfc_batch_set_state(self._b, i, _ptr(phi_prev, P, "phi_prev"),
                                                 _ptr(phi_cur, P, "phi_cur"), _ptr(mu, P, "mu"),
                                                 _ptr(omega, P, "omega")))

    def get_state(self, i):
        n = self.sizes[i]
        out = [torch.empty((n, n, n), dtype=torch.float64, device=self.device) for _ in range(4)]
        self._check(self.lib.pfc_batch_get_state(self._b, i, *[_ptr(t, n ** 3, "state") for t in out]))
        return tuple(out)

    def run(self, steps, raise_on_error=True):
        """Returns infos[i][k] (instance i, step k)."""
        infos = (abi.PfcStepInfo * (self.count * steps))()
        st = self.lib.pfc_batch_run(self._b, steps, infos)
        if raise_on_error:
            self._check(st)
        return [[StepInfo(infos[i * steps + k].cycles, infos[i * steps + k].status,
                          infos[i * steps + k].res0, infos[i * steps + k].res_final)
                 for k in range(steps)] for i in range(self.count)]

    def autotune(self, cache_path=None):
        """Schedules and tile shapes of (smooth, residual+coarsening, tau,
        interpolation, coarse error): a list of five (persistent, threads per
        workgroup, items per plane W, planes Z) tuples; an interpolation run
        as column tiles reads (False, 64, 64, coarse planes per tile)."""
        chosen = (C.c_int32 * 20)()
        path = None if cache_path is None else str(cache_path).encode()
        self._check(self.lib.pfc_batch_autotune(self._b, path, chosen))
        return [(bool(chosen[4 * k]), chosen[4 * k + 1], chosen[4 * k + 2], chosen[4 * k + 3])
                for k in range(5)]
