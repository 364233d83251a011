"""Host-side checks of the C-ABI library (no GPU work)."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_1611_06288_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+char\s*\*|pfc_status|int32_t)\s*(pfc_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("pfc_step", "pfc_fas_vcycle", "pfc_energy", "pfc_adjoint_step", "pfc_create",
                 "pfc_destroy", "pfc_batch_run"):
        assert must in names


def test_library_loads_and_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("HIP library not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the ctypes table covers exactly the declared functions
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_header_constants_match_the_binding():
    text = open(HEADER).read()
    consts = dict((k, int(v)) for k, v in re.findall(r"^#define\s+(PFC_\w+)\s+(-?\d+)", text, flags=re.M))
    assert "PFC_SWEEP_FULL" in consts and "PFC_KERNEL_COUNT" in consts
    for name, value in consts.items():
        assert getattr(_lib, name) == value, name


def test_status_strings_and_create_errors_without_gpu_work():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("HIP library not built")
    L = _lib.lib()
    assert L.pfc_status_string(0) == b"ok"
    assert b"converged" in L.pfc_status_string(2)
    cfg = _lib.PfcConfig(n=10, nu1=2, nu2=2, max_cycles=10, cycle=0, lin=0, precision=0, mobility=0,
                         L=10.0, eps=0.1, dt=0.1, tol=1e-10)
    h = ctypes.c_void_p()
    # validation happens before any device call
    assert L.pfc_create(ctypes.byref(cfg), None, ctypes.byref(h)) == _lib.PFC_ERR_INVALID_ARG
    assert b"3*2^k" in L.pfc_last_error(None)
    for field, bad in (("n", 7), ("dt", 0.0), ("L", -1.0), ("tol", -1.0), ("nu1", -1),
                       ("max_cycles", 0), ("cycle", 5), ("precision", 9)):
        c = _lib.PfcConfig.from_buffer_copy(cfg)
        c.n = 16
        setattr(c, field, bad)
        assert L.pfc_create(ctypes.byref(c), None, ctypes.byref(h)) == _lib.PFC_ERR_INVALID_ARG, field
    c = _lib.PfcConfig.from_buffer_copy(cfg)
    c.n, c.precision, c.lin = 16, _lib.PFC_MIXED, _lib.PFC_LIN_PICARD
    assert L.pfc_create(ctypes.byref(c), None, ctypes.byref(h)) == _lib.PFC_ERR_INVALID_ARG
    for prec, bad in ((_lib.PFC_FP64, 5), (_lib.PFC_MIXED, _lib.PFC_SCHEME_CS1)):
        c = _lib.PfcConfig.from_buffer_copy(cfg)
        c.n, c.precision, c.scheme = 16, prec, bad
        assert L.pfc_create(ctypes.byref(c), None, ctypes.byref(h)) == _lib.PFC_ERR_INVALID_ARG
        assert b"scheme" in L.pfc_last_error(None)
    # variable mobility: enum, FP64 only, mob_min > 0, finite coefficients
    for field, bad, why in (("mobility", 7, b"unknown mobility"),
                            ("precision", _lib.PFC_MIXED, b"FP64"),
                            ("mob_min", 0.0, b"mob_min"),
                            ("mob_m1", float("inf"), b"finite"),
                            ("scheme", _lib.PFC_SCHEME_CS1, b"first-order")):
        c = _lib.PfcConfig.from_buffer_copy(cfg)
        c.n, c.mobility, c.mob_m0, c.mob_min = 16, _lib.PFC_MOBILITY_QUADRATIC, 1.0, 0.05
        setattr(c, field, bad)
        assert L.pfc_create(ctypes.byref(c), None, ctypes.byref(h)) == _lib.PFC_ERR_INVALID_ARG
        assert why in L.pfc_last_error(None), (field, L.pfc_last_error(None))
    assert L.pfc_step(None, None, None, None, None, None, None) == _lib.PFC_ERR_INVALID_ARG
    # sizes: 2^k (k >= 2) or 3 * 2^k (k >= 1), at most 1024
    for bad_n in (0, 2, 6 * 7, 2048, 1536, 1025):
        c = _lib.PfcConfig.from_buffer_copy(cfg)
        c.n = bad_n
        assert L.pfc_create(ctypes.byref(c), None, ctypes.byref(h)) == _lib.PFC_ERR_INVALID_ARG, bad_n


def test_batch_create_errors_without_gpu_work():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("HIP library not built")
    L = _lib.lib()
    b = ctypes.c_void_p()
    good = _lib.PfcConfig(n=16, nu1=2, nu2=2, max_cycles=10, cycle=0, lin=0, precision=0, mobility=0,
                          L=16.0, eps=0.1, dt=0.1, tol=1e-10)
    # an empty batch, or more instances than the tables hold
    for count in (0, -1, 4097):
        assert L.pfc_batch_create(count, ctypes.byref(good), None, ctypes.byref(b)) == \
            _lib.PFC_ERR_INVALID_ARG, count
        assert b.value is None
    assert b"count" in L.pfc_batch_last_error(None)
    arr = (_lib.PfcConfig * 2)(good, good)
    for field, bad, why in (("n", 10, b"instance 1"), ("precision", _lib.PFC_MIXED, b"FP64"),
                            ("nu1", 3, b"must agree")):
        arr[1] = _lib.PfcConfig.from_buffer_copy(good)
        setattr(arr[1], field, bad)
        assert L.pfc_batch_create(2, arr, None, ctypes.byref(b)) == _lib.PFC_ERR_INVALID_ARG, field
        assert why in L.pfc_batch_last_error(None), (field, L.pfc_batch_last_error(None))


def test_config_struct_layout_matches_the_header():
    """Offsets and size of pfc_config as the C compiler lays it out."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f for f, _ in _lib.PfcConfig._fields_]
    src = "#include <stddef.h>\n#include <stdio.h>\n#include \"pfc.h\"\nint main(void){\n"
    src += 'printf("%zu\\n", sizeof(pfc_config));\n'
    for f in fields:
        src += f'printf("%zu\\n", offsetof(pfc_config, {f}));\n'
    src += "return 0;}\n"
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c_path, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(c_path, "w").write(src)
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), c_path, "-o", exe], check=True)
        out = [int(x) for x in subprocess.run([exe], check=True, capture_output=True,
                                              text=True).stdout.split()]
    assert out[0] == ctypes.sizeof(_lib.PfcConfig)
    assert out[1:] == [getattr(_lib.PfcConfig, f).offset for f in fields]


def test_solver_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_1611_06288_amd import Solver
    with pytest.raises(RuntimeError):
        Solver(16, 16.0, 0.1, 0.1)
