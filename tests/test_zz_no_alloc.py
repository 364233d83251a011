"""pfc_energy_static (the allocation-free energy entry point) against
pfc_energy through the C ABI: two calls in a row on one GPU, the second on
a smaller grid, each equal bit for bit to the handle's result (same kernels,
same reduction order); with and without phi_prev; sizes beyond the limit
rejected before any GPU work."""
import ctypes as C
import math

import numpy as np
import pytest
import torch

from paper_1611_06288_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _static(n, L, eps, phi, prev, out3):
    lib = _lib.lib()
    stream = torch.cuda.current_stream().cuda_stream
    return lib.pfc_energy_static(n, L, eps, C.c_void_p(phi.data_ptr()),
                                 None if prev is None else C.c_void_p(prev.data_ptr()),
                                 C.c_void_p(out3.data_ptr()), C.c_void_p(stream))


def test_energy_static_equals_pfc_energy_twice_shrinking():
    from paper_1611_06288_amd import Solver
    out3 = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
    for n, seed in ((96, 71), (32, 72)):
        L, eps = n * math.pi / 4, 0.25
        g = inputs.rng(seed)
        phi = torch.from_numpy(0.285 + 0.1 * g.uniform(-1, 1, (n, n, n))).cuda()
        prev = torch.from_numpy(0.285 + 0.1 * g.uniform(-1, 1, (n, n, n))).cuda()
        s = Solver(n, L, eps, 0.5)
        for pv in (prev, None):
            want = s.energy(phi, pv)
            out3.fill_(float("nan"))
            st = _static(n, L, eps, phi, pv, out3)
            assert st == _lib.PFC_OK, _lib.lib().pfc_last_error(None)
            torch.cuda.synchronize()
            got = out3.cpu().tolist()
            print(f"n={n} prev={'yes' if pv is not None else 'no'}: {got} vs {list(want)}")
            assert got == list(want), (n, got, want)
        s.close()


def test_energy_static_rejects_sizes_beyond_the_limit():
    lib = _lib.lib()
    buf = torch.zeros(8, dtype=torch.float64, device="cuda")
    for n in (_lib.PFC_ENERGY_STATIC_MAX_N + 2, 2):
        st = _static(n, 1.0, 0.25, buf, None, buf)
        assert st == _lib.PFC_ERR_INVALID_ARG
        assert b"n must be in" in lib.pfc_last_error(None)
    assert lib.pfc_energy_static(8, 1.0, 0.25, None, None, C.c_void_p(buf.data_ptr()), None) \
        == _lib.PFC_ERR_INVALID_ARG
