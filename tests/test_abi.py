"""C ABI of libuot.so: loads, exports every function declared in include/*.h, and rejects
invalid arguments on the host before any launch (CPU only; no compute calls)."""
import ctypes
import glob
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2201_00730_amd as uot

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for mt in re.finditer(r"\b(uot_[a-z0-9_]+)\s*\(", text):
            names.add(mt.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(uot.library_path()):
        pytest.fail("libuot.so is not built (run __graft_entry__.build())")
    return uot.load_library()


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for required in ("uot_sinkhorn", "uot_ti_sinkhorn", "uot_dual_value", "uot_plan_apply",
                     "uot_backward", "uot_workspace_bytes", "uot_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", uot.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for name in _declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def _cost(kind=1, n=10, m=12, d=3, p=2.0, ldc=0):
    c = uot._Cost()
    c.kind, c.n, c.m, c.d = kind, n, m, d
    c.C = ctypes.c_void_p(0x1000) if kind == 0 else None
    c.ldc = ldc if ldc else m
    c.x = ctypes.c_void_p(0x1000) if kind == 1 else None
    c.y = ctypes.c_void_p(0x2000) if kind == 1 else None
    c.p = p
    return c


def test_workspace_bytes_host_only(lib):
    c = _cost()
    assert lib.uot_workspace_bytes(ctypes.byref(c), 0) > 0
    big = _cost(n=20000, m=20000)
    assert lib.uot_workspace_bytes(ctypes.byref(big), 0) > lib.uot_workspace_bytes(ctypes.byref(c), 0)
    dense = _cost(kind=0, n=64, m=100, d=0)
    assert lib.uot_workspace_bytes(ctypes.byref(dense), 0) > 0
    for bad in (_cost(n=0), _cost(m=0), _cost(d=0), _cost(d=65), _cost(p=0.5),
                _cost(p=float("nan")), _cost(kind=0, ldc=5), _cost(kind=7)):
        assert lib.uot_workspace_bytes(ctypes.byref(bad), 0) == 0
    assert lib.uot_workspace_bytes(ctypes.byref(c), 9) == 0
    assert lib.uot_workspace_bytes(None, 0) == 0


@pytest.mark.parametrize("field,value", [("eps", 0.0), ("eps", -1.0), ("eps", float("inf")),
                                         ("rho1", 0.0), ("rho2", float("nan")), ("max_iter", 0),
                                         ("tol", -1.0), ("check_every", 0)])
def test_solver_rejects_bad_params_before_any_launch(lib, field, value):
    c = _cost()
    prm = uot._Params(0.1, 1.0, 1.0, 10, 0.0, 1, 0)
    setattr(prm, field, value)
    for fn in (lib.uot_sinkhorn, lib.uot_ti_sinkhorn):
        st = fn(ctypes.byref(c), None, None, ctypes.byref(prm), None, None, None, 0, None, None)
        assert st == uot.UOT_ERR_INVALID
        assert lib.uot_last_error()


@pytest.mark.parametrize("k,r", [(1, 1e-7), (9, 1e-7), (0, 1e-7), (4, 0.0), (4, -1e-7),
                                 (4, float("nan")), (4, float("inf"))])
def test_anderson_rejects_bad_settings_before_any_launch(lib, k, r):
    c = _cost()
    prm = uot._Params(0.1, 1.0, 1.0, 10, 0.0, 1, 0)
    acc = uot._Anderson(k, r)
    for fn in (lib.uot_sinkhorn_anderson, lib.uot_ti_sinkhorn_anderson):
        st = fn(ctypes.byref(c), None, None, ctypes.byref(prm), ctypes.byref(acc), None, None, None,
                0, None, None)
        assert st == uot.UOT_ERR_INVALID
        assert b"anderson" in lib.uot_last_error()
        assert fn(ctypes.byref(c), None, None, ctypes.byref(prm), None, None, None, None, 0, None,
                  None) == uot.UOT_ERR_INVALID


def test_anderson_workspace_is_larger(lib):
    c = _cost(n=1000, m=900)
    solve = lib.uot_workspace_bytes(ctypes.byref(c), uot.UOT_WS_SOLVE)
    acc = lib.uot_workspace_bytes(ctypes.byref(c), uot.UOT_WS_ANDERSON)
    assert acc >= solve + 9 * 1000 * 4


def test_points_kernel_switch_keeps_workspace_size(lib):
    """Every p = 2 softmin variant (4: direct differences) fits the same workspace, so a
    workspace sized under one setting serves the others."""
    sizes = []
    prev = uot.set_points_kernel(uot.POINTS_KERNEL_AUTO)
    try:
        for v in (0, 1, 2, 3, uot.POINTS_KERNEL_DIRECT):
            assert uot.set_points_kernel(v) in (0, 1, 2, 3, 4)
            sizes.append([lib.uot_workspace_bytes(ctypes.byref(_cost(n=1000, m=900, d=d)),
                                                  uot.UOT_WS_SOLVE) for d in (1, 3, 16, 20)])
        with pytest.raises(ValueError):
            uot.set_points_kernel(5)
    finally:
        uot.set_points_kernel(prev)
    assert all(s == sizes[0] for s in sizes), sizes


def test_grad_kernel_switch_keeps_workspace_size(lib):
    """Both backward implementations fit the same workspace; unknown settings are refused."""
    prev = uot.set_grad_kernel(uot.GRAD_KERNEL_MFMA)
    sizes = []
    try:
        for v in (uot.GRAD_KERNEL_MFMA, uot.GRAD_KERNEL_VALU):
            assert uot.set_grad_kernel(v) in (0, 1)
            sizes.append([lib.uot_workspace_bytes(ctypes.byref(_cost(n=1000, m=900, d=d)),
                                                  uot.UOT_WS_BACKWARD) for d in (3, 12, 16)])
        assert lib.uot_set_grad_kernel(2) == -1 and lib.uot_set_grad_kernel(-1) == -1
        with pytest.raises(ValueError):
            uot.set_grad_kernel(2)
    finally:
        uot.set_grad_kernel(prev)
    assert sizes[0] == sizes[1], sizes


def test_solver_rejects_bad_cost(lib):
    prm = uot._Params(0.1, 1.0, 1.0, 10, 0.0, 1, 0)
    for bad in (_cost(n=0), _cost(d=100), _cost(p=0.0), _cost(kind=0, ldc=3)):
        assert lib.uot_ti_sinkhorn(ctypes.byref(bad), None, None, ctypes.byref(prm), None, None, None,
                                   0, None, None) == uot.UOT_ERR_INVALID
    assert lib.uot_ti_sinkhorn(None, None, None, ctypes.byref(prm), None, None, None, 0, None,
                               None) == uot.UOT_ERR_INVALID


def test_other_entry_points_reject_bad_scalars(lib):
    c = _cost()
    v = ctypes.c_double(0)
    assert lib.uot_dual_value(ctypes.byref(c), None, None, -1.0, 1.0, 1.0, None, None, None, 0,
                              ctypes.byref(v), None) == uot.UOT_ERR_INVALID
    assert lib.uot_dual_value(ctypes.byref(c), None, None, 0.1, 1.0, 1.0, None, None, None, 0,
                              None, None) == uot.UOT_ERR_INVALID
    assert lib.uot_plan_apply(ctypes.byref(c), None, None, 0.1, None, None, 0, None, 0, 1, None, 1,
                              None, 0, None) == uot.UOT_ERR_INVALID  # k = 0
    assert lib.uot_plan_apply(ctypes.byref(c), None, None, 0.1, None, None, 0, None, 2, 2, None, 2,
                              None, 0, None) == uot.UOT_ERR_INVALID  # V = NULL with k = 2
    assert lib.uot_plan_apply(ctypes.byref(c), None, None, 0.1, None, None, 2, None, 1, 1, None, 1,
                              None, 0, None) == uot.UOT_ERR_INVALID  # transpose = 2
    dense = _cost(kind=0, d=0)
    assert lib.uot_backward(ctypes.byref(dense), None, None, 0.1, 1.0, 1.0, None, None, 1.0,
                            ctypes.c_void_p(0x1000), None, None, None, None, 0,
                            None) == uot.UOT_ERR_INVALID  # dx with a dense cost
    assert lib.uot_backward(ctypes.byref(c), None, None, 0.1, 1.0, 1.0, None, None,
                            float("nan"), None, None, None, None, None, 0, None) == uot.UOT_ERR_INVALID


def test_status_strings(lib):
    for s in range(5):
        assert lib.uot_status_string(s)
    assert lib.uot_status_string(99) == b"unknown status"


def test_python_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        uot.ti_sinkhorn(torch.ones(3), torch.ones(3), x=torch.zeros(3, 1), y=torch.zeros(3, 1),
                        eps=0.1, rho1=1.0)


@pytest.mark.parametrize("entropy,variant", [(2, 0), (-1, 0), (0, 2), (1, -1)])
def test_phi_rejects_bad_settings_before_any_launch(lib, entropy, variant):
    c = _cost()
    prm = uot._Params(0.1, 1.0, 1.0, 10, 0.0, 1, 0)
    phi = uot._Phi(entropy, variant)
    assert lib.uot_sinkhorn_phi(ctypes.byref(c), None, None, ctypes.byref(prm), ctypes.byref(phi),
                                None, None, None, 0, None, None) == uot.UOT_ERR_INVALID
    assert b"phi" in lib.uot_last_error()
    assert lib.uot_sinkhorn_phi(ctypes.byref(c), None, None, ctypes.byref(prm), None, None, None,
                                None, 0, None, None) == uot.UOT_ERR_INVALID


def test_fw1d_rejects_bad_arguments_before_any_launch(lib):
    offN = np.array([0, 3, 5], dtype=np.int64)
    offM = np.array([0, 2, 6], dtype=np.int64)
    assert lib.uot_fw1d_workspace_bytes(2, offN.ctypes.data, offM.ctypes.data) > 0
    bad = np.array([0, 3, 3], dtype=np.int64)  # an empty problem
    assert lib.uot_fw1d_workspace_bytes(2, bad.ctypes.data, offM.ctypes.data) == 0
    assert lib.uot_fw1d_workspace_bytes(0, offN.ctypes.data, offM.ctypes.data) == 0
    for p, ls, it, tol in ((0.5, 0, 10, 0.0), (2.0, 2, 10, 0.0), (2.0, 0, 0, 0.0),
                           (2.0, 0, 10, -1.0), (float("nan"), 0, 10, 0.0)):
        st = lib.uot_fw1d_batched(2, offN.ctypes.data, offM.ctypes.data, None, None, None, None,
                                  None, None, p, ls, it, tol, None, None, None, None, None, None,
                                  0, None)
        assert st == uot.UOT_ERR_INVALID
        assert lib.uot_last_error()


def test_barycenter_rejects_bad_arguments_before_any_launch(lib):
    off = np.array([0, 3, 5, 9], dtype=np.int64)
    assert lib.uot_fw1d_barycenter_workspace_bytes(1, 3, off.ctypes.data) > 0
    assert lib.uot_fw1d_barycenter_workspace_bytes(1, 1, off.ctypes.data) == 0     # K < 2
    assert lib.uot_fw1d_barycenter_workspace_bytes(1, 17, off.ctypes.data) == 0    # K > 16
    bad = np.array([0, 3, 3, 9], dtype=np.int64)  # an empty measure
    assert lib.uot_fw1d_barycenter_workspace_bytes(1, 3, bad.ctypes.data) == 0
    for it, tol in ((0, 0.0), (10, -1.0), (10, float("inf"))):
        st = lib.uot_fw1d_barycenter(1, 3, off.ctypes.data, None, None, None, None, it, tol, None,
                                     None, None, None, None, None, None, 0, None)
        assert st == uot.UOT_ERR_INVALID
        assert lib.uot_last_error()


def test_rate_estimate_of_a_geometric_sequence():
    """The bench's rate estimate (median log ratio of consecutive errors) returns the ratio of
    a geometric sequence exactly, ignores errors under the floor, and is None without pairs."""
    import bench
    assert abs(bench.kappa([0.8 ** t for t in range(30)]) - 0.8) < 1e-12
    assert abs(bench.kappa([0.5 ** t for t in range(10)] + [1e-7, 1e-7]) - 0.5) < 1e-12
    assert bench.kappa([1e-6, 1e-7]) is None


def test_anderson_rejects_bad_normalize_flag(lib):
    c = _cost()
    prm = uot._Params(0.1, 1.0, 1.0, 10, 0.0, 1, 0)
    for flag in (2, -1):
        acc = uot._Anderson(4, 1e-7, flag)
        st = lib.uot_ti_sinkhorn_anderson(ctypes.byref(c), None, None, ctypes.byref(prm),
                                          ctypes.byref(acc), None, None, None, 0, None, None)
        assert st == uot.UOT_ERR_INVALID
        assert b"normalize" in lib.uot_last_error()


def test_noalloc_backward_rejects_a_problem_beyond_its_scratch_array(lib):
    """The allocation-free backward refuses, before any launch, a problem whose backward
    workspace exceeds UOT_NOALLOC_BYTES (96 MiB), and one with a bad cost."""
    big = _cost(n=400000, m=400000, d=3)
    assert lib.uot_workspace_bytes(ctypes.byref(big), uot.UOT_WS_BACKWARD) > 96 << 20
    st = lib.uot_backward_noalloc(ctypes.byref(big), None, None, 0.1, 1.0, 1.0, None, None, 1.0,
                                  None, None, None, None, None)
    assert st == uot.UOT_ERR_WORKSPACE
    assert b"allocation-free" in lib.uot_last_error()
    assert lib.uot_backward_noalloc(ctypes.byref(_cost(n=0)), None, None, 0.1, 1.0, 1.0, None,
                                    None, 1.0, None, None, None, None, None) == uot.UOT_ERR_INVALID
