"""The C ABI on the CPU: the library loads, exports every function that
include/mcr.h declares, validates arguments before touching the device, and
its host step-size helper agrees with the oracle's rule."""
import ctypes
import math
import subprocess

import numpy as np
import pytest

from paper_2410_10503_amd import _lib
from oracle import spdhg


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_function(lib):
    declared = _lib.header_functions()
    assert len(declared) >= 19
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    for f in declared:
        assert hasattr(lib, f)


def test_binding_declares_every_function():
    declared = set(_lib.header_functions()) - {"mcr_last_error"}
    assert declared == set(_lib.SIGNATURES)


@pytest.mark.parametrize("N,alpha", [(1, 1e-3), (4, 1e-2), (16, 1e-3)])
def test_step_sizes_match_oracle(lib, N, alpha):
    rng = np.random.default_rng(N)
    norms = list(3.7e5 * (1 + 0.03 * rng.random(N)))
    sig = (ctypes.c_double * N)()
    tau, th, rate = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    arr = (ctypes.c_double * N)(*norms)
    _lib.check(lib.mcr_step_sizes(0, N, arr, alpha, sig, ctypes.byref(tau), ctypes.byref(th), ctypes.byref(rate)))
    s_o, t_o, th_o, rho = spdhg.step_sizes_spdhg(norms, alpha, N)
    np.testing.assert_allclose(list(sig), s_o, rtol=1e-14)
    assert math.isclose(tau.value, t_o, rel_tol=1e-14) and math.isclose(th.value, th_o, rel_tol=1e-14)
    assert math.isclose(rate.value, spdhg.rate(max(norms) / (alpha * N), N), rel_tol=1e-12)
    stacked = (ctypes.c_double * 1)(N * 3.8e5)
    _lib.check(lib.mcr_step_sizes(1, N, stacked, alpha, sig, ctypes.byref(tau), ctypes.byref(th), ctypes.byref(rate)))
    s_o, t_o, th_o, rho = spdhg.step_sizes_pdhg(N * 3.8e5, alpha, N)
    np.testing.assert_allclose(list(sig), s_o, rtol=1e-14)
    assert math.isclose(tau.value, t_o, rel_tol=1e-14) and math.isclose(th.value, th_o, rel_tol=1e-14)
    assert math.isclose(rate.value, spdhg.rate(N * 3.8e5 / (alpha * N), 1), rel_tol=1e-12)


def _create(lib, geo, n_gates, motion, dtype=0):
    h = ctypes.c_void_p()
    st = lib.mcr_create(ctypes.byref(geo) if geo is not None else None, n_gates, motion, dtype, None,
                        ctypes.byref(h))
    return st, h


def _motions(*ms):
    arr = (_lib.Motion * len(ms))()
    for i, m in enumerate(ms):
        arr[i] = m
    return arr


RIGID = _lib.Motion(_lib.MOTION_RIGID, (ctypes.c_double * 3)(0.1, 1.0, -2.0), None)


@pytest.mark.parametrize("geo,ng,mot,dtype,needle", [
    (None, 1, _motions(RIGID), 0, "geometry"),
    (_lib.Geometry(0, 10, 10), 1, _motions(RIGID), 0, "n = 0"),
    (_lib.Geometry(16, 0, 10), 1, _motions(RIGID), 0, "n_angles"),
    (_lib.Geometry(16, 10, 20000), 1, _motions(RIGID), 0, "n_det"),
    (_lib.Geometry(16, 10, 24), 0, _motions(RIGID), 0, "n_gates"),
    (_lib.Geometry(16, 10, 24), 1, None, 0, "motion is null"),
    (_lib.Geometry(16, 10, 24), 1, _motions(_lib.Motion(7, (ctypes.c_double * 3)(0, 0, 0), None)), 0, "kind"),
    (_lib.Geometry(16, 10, 24), 1, _motions(_lib.Motion(1, (ctypes.c_double * 3)(float("nan"), 0, 0), None)), 0,
     "not finite"),
    (_lib.Geometry(16, 10, 24), 1, _motions(_lib.Motion(2, (ctypes.c_double * 3)(0, 0, 0), None)), 0, "field"),
    (_lib.Geometry(16, 10, 24), 1, _motions(RIGID), 5, "dtype"),
])
def test_create_rejects_bad_arguments_before_device_work(lib, geo, ng, mot, dtype, needle):
    st, h = _create(lib, geo, ng, mot, dtype)
    assert st == _lib.MCR_ERR_ARG
    assert not h.value
    assert needle in lib.mcr_last_error().decode()


def test_null_handle_is_an_argument_error(lib):
    assert lib.mcr_apply_Ai(None, 0, None, None) == _lib.MCR_ERR_ARG
    assert b"null handle" in lib.mcr_last_error()
    assert lib.mcr_spdhg_epoch(None, None, None, 1.0, None, 1.0, 1.0, None, None) == _lib.MCR_ERR_ARG
    assert lib.mcr_destroy(None) == _lib.MCR_OK


@pytest.mark.parametrize("algo,N,norms,alpha", [(2, 1, [1.0], 1.0), (0, 0, [1.0], 1.0), (0, 2, [1.0, -1.0], 1.0),
                                                (1, 2, [float("inf")], 1.0), (0, 1, [1.0], 0.0)])
def test_step_sizes_reject_bad_arguments(lib, algo, N, norms, alpha):
    sig = (ctypes.c_double * max(N, 1))()
    assert lib.mcr_step_sizes(algo, N, (ctypes.c_double * len(norms))(*norms), alpha, sig, None, None,
                              None) == _lib.MCR_ERR_ARG


@pytest.mark.parametrize("N,M,alpha", [(1, 1, 1e-3), (4, 3, 0.5), (16, 4, 1e-3)])
def test_block_step_sizes_match_oracle(lib, N, M, alpha):
    from oracle import subsets
    rng = np.random.default_rng(N * 10 + M)
    norms = list(3.7e5 / M * (1 + 0.05 * rng.random(N * M)))
    nb = N * M
    sig = (ctypes.c_double * nb)()
    tau, th, rate = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _lib.check(lib.mcr_step_sizes_blocks(N, M, (ctypes.c_double * nb)(*norms), alpha, sig, ctypes.byref(tau),
                                         ctypes.byref(th), ctypes.byref(rate)))
    s_o, t_o, th_o, rho = subsets.step_sizes(norms, alpha, N)
    np.testing.assert_allclose(list(sig), s_o, rtol=1e-14)
    assert math.isclose(tau.value, t_o, rel_tol=1e-14) and math.isclose(th.value, th_o, rel_tol=1e-14)
    assert math.isclose(rate.value, subsets.epoch_rate(norms, alpha, N), rel_tol=1e-12)
    bad = (ctypes.c_double * nb)(*([0.0] + norms[1:]))
    assert lib.mcr_step_sizes_blocks(N, M, bad, alpha, sig, None, None, None) == _lib.MCR_ERR_ARG
    assert lib.mcr_step_sizes_blocks(N, 0, (ctypes.c_double * nb)(*norms), alpha, sig, None, None,
                                     None) == _lib.MCR_ERR_ARG


def test_set_subsets_rejects_null_handle(lib):
    assert lib.mcr_set_subsets(None, 2) == _lib.MCR_ERR_ARG


def test_register_rigid_rejects_null_handle(lib):
    th = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    assert lib.mcr_register_rigid(None, 0, None, None, th, 10, 1e-6, None, None) == _lib.MCR_ERR_ARG
    assert b"null handle" in lib.mcr_last_error()


def test_register_affine_rejects_null_handle(lib):
    th = (ctypes.c_double * 6)()
    assert lib.mcr_register_affine(None, 0, None, None, th, 10, 1e-6, None, None) == _lib.MCR_ERR_ARG
    assert b"null handle" in lib.mcr_last_error()


def test_register_field_rejects_null_handle(lib):
    assert lib.mcr_register_field(None, 0, None, None, None, 0.1, None, 0, 10, 1e-4, None, None) == _lib.MCR_ERR_ARG


def test_project_noalloc_validates_before_device_work(lib):
    # sizes beyond the fixed scratch array, a null geometry and null pointers
    # are refused before anything touches a device (this runs without a GPU)
    dummy = ctypes.c_void_p(0x1000)
    for geo, msg in ((_lib.Geometry(1025, 10, 10), b"n = 1025"), (_lib.Geometry(64, 4097, 10), b"n_angles = 4097"),
                     (_lib.Geometry(64, 10, 16385), b"n_det = 16385"), (_lib.Geometry(0, 10, 10), b"n = 0")):
        st = lib.mcr_project_noalloc(ctypes.byref(geo), dummy, dummy, None)
        assert st == _lib.MCR_ERR_ARG
        assert msg in lib.mcr_last_error()
    assert lib.mcr_project_noalloc(None, dummy, dummy, None) == _lib.MCR_ERR_ARG
    geo = _lib.Geometry(64, 10, 10)
    assert lib.mcr_project_noalloc(ctypes.byref(geo), None, dummy, None) == _lib.MCR_ERR_ARG
    assert lib.mcr_project_noalloc(ctypes.byref(geo), dummy, None, None) == _lib.MCR_ERR_ARG


def test_probe_library_exports_every_declared_function():
    import os
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    header = open(os.path.join(root, "include", "mcr_probes.h")).read()
    declared = re.findall(r"^int (mcr_probe_\w+)\(", header, flags=re.M)
    assert len(declared) >= 4
    path = os.path.join(root, "paper_2410_10503_amd", "libmcr_probes.so")
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert not [f for f in declared if f not in exported]


def test_probe_lds_pattern_validates_before_device_work():
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    probes = ctypes.CDLL(os.path.join(root, "paper_2410_10503_amd", "libmcr_probes.so"))
    probes.mcr_probe_lds_pattern.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_double)]
    v = ctypes.c_double()
    assert probes.mcr_probe_lds_pattern(None, 1, 1, ctypes.byref(v)) == 1
    bad = (ctypes.c_int * 64)(*([0] * 63 + [64]))
    assert probes.mcr_probe_lds_pattern(bad, 1, 1, ctypes.byref(v)) == 1
    ok = (ctypes.c_int * 64)(*range(64))
    assert probes.mcr_probe_lds_pattern(ok, 0, 1, ctypes.byref(v)) == 1
