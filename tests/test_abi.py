"""C-ABI contract on the CPU: the library loads, exports every function the
header declares, sizes workspaces, and rejects bad arguments with the
documented status before anything is enqueued.  Every call here fails
validation (or is a documented no-op), so nothing touches a device; the
pointers passed are never dereferenced."""
import ctypes
import os
import re

import pytest

from paper_1302_4000_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clusco.h")
FAKE = ctypes.c_void_p(0x10000)        # never dereferenced
FAKE_ODD = ctypes.c_void_p(0x10002)


def declared_functions():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(clusco_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return binding.lib()


@pytest.fixture(scope="module")
def h(L):
    hh = ctypes.c_void_p()
    assert L.clusco_create(ctypes.byref(hh), 0) == binding.OK
    yield hh
    L.clusco_destroy(hh)


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    for s, name in enumerate(["CLUSCO_OK", "CLUSCO_ERR_INVALID_ARG", "CLUSCO_ERR_WORKSPACE",
                              "CLUSCO_ERR_UNSUPPORTED", "CLUSCO_ERR_HIP"]):
        assert L.clusco_status_string(s).decode() == name


def test_create_rejects_bad_arguments(L):
    assert L.clusco_create(None, 0) == binding.ERR_INVALID_ARG
    hh = ctypes.c_void_p()
    assert L.clusco_create(ctypes.byref(hh), -1) == binding.ERR_INVALID_ARG


def test_workspace_sizes(L, h):
    s1 = L.clusco_crmsd_workspace_size(h, 200, 100, 0)
    s2 = L.clusco_crmsd_workspace_size(h, 20000, 150, 1)
    assert s1 > 0 and s2 > s1 and s1 % 256 == 0 and s2 % 256 == 0
    # operands alone: 3 planes x Np x Lp (FP32) / two halves per value (split)
    assert s1 >= 3 * 256 * 104 * 4
    assert s2 >= 2 * 2 * 3 * 20032 * 160
    assert L.clusco_crmsd_workspace_size(h, 10, 0, 0) == 0
    assert L.clusco_crmsd_workspace_size(h, -1, 5, 0) == 0
    assert L.clusco_crmsd_workspace_size(h, 10, 5, 9) == 0
    assert L.clusco_crmsd_workspace_size(None, 10, 5, 0) == 0


def test_matrix_argument_errors(L, h):
    f = L.clusco_crmsd_matrix
    need = L.clusco_crmsd_workspace_size(h, 100, 50, 0)
    assert f(None, FAKE, 100, 50, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 0, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, -3, 50, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 50, 7, FAKE, FAKE, need, None) == binding.ERR_UNSUPPORTED
    assert f(h, None, 100, 50, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 50, 0, None, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE_ODD, 100, 50, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 50, 0, FAKE, None, need, None) == binding.ERR_WORKSPACE
    assert f(h, FAKE, 100, 50, 0, FAKE, FAKE, need - 1, None) == binding.ERR_WORKSPACE
    assert f(h, FAKE, 100, 50, 0, FAKE, ctypes.c_void_p(0x10040), need, None) == \
        binding.ERR_INVALID_ARG
    assert b"256" in L.clusco_last_error(h)
    assert f(h, FAKE, 1 << 21, 50, 0, FAKE, FAKE, need, None) == binding.ERR_UNSUPPORTED
    # N in {0, 1}: nothing to compute, nothing enqueued, pointers unused
    assert f(h, None, 0, 50, 0, None, None, 0, None) == binding.OK
    assert f(h, None, 1, 50, 3, None, None, 0, None) == binding.OK


def test_set_tolerance(L, h):
    assert L.clusco_set_tolerance(h, 0, 1e-4) == binding.OK
    assert L.clusco_set_tolerance(h, 11, 1e-4) == binding.ERR_UNSUPPORTED
    assert L.clusco_set_tolerance(None, 0, 1e-4) == binding.ERR_INVALID_ARG


def test_binding_refuses_cpu_tensors():
    import torch
    from paper_1302_4000_amd import crmsd_matrix
    with pytest.raises(TypeError):
        crmsd_matrix(torch.zeros(4, 5, 3))


def test_cross_argument_errors(L, h):
    f = L.clusco_crmsd_cross
    need = L.clusco_crmsd_cross_workspace_size(h, 50, 1, 30, 0)
    assert need > 0
    assert f(h, FAKE, 50, FAKE, 1, 0, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, -1, FAKE, 1, 30, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, None, 50, FAKE, 1, 30, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 50, None, 1, 30, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 50, FAKE, 1, 30, 0, FAKE, FAKE, need - 1, None) == binding.ERR_WORKSPACE
    assert f(h, FAKE, 50, FAKE, 1, 30, 5, FAKE, FAKE, need, None) == binding.ERR_UNSUPPORTED
    assert f(h, None, 0, None, 7, 30, 0, None, None, 0, None) == binding.OK
    assert f(h, None, 7, None, 0, 30, 0, None, None, 0, None) == binding.OK


def _arr(vals):
    a = (ctypes.c_int64 * len(vals))(*vals)
    return a


def test_batched_argument_errors_and_sizes(L, h):
    N, Ls = _arr([100, 1, 300]), _arr([50, 20, 120])
    co, oo = _arr([0, 15000, 15060]), _arr([0, 4950, 4950])
    size = L.clusco_crmsd_batched_workspace_size(h, 3, N, Ls, 1)
    # at least the two real ensembles' operands
    assert size >= 2 * 2 * 3 * (128 * 64 + 320 * 128)
    assert L.clusco_crmsd_batched_workspace_size(h, 3, None, Ls, 1) == 0
    bad = _arr([100, -1, 300])
    assert L.clusco_crmsd_batched_workspace_size(h, 3, bad, Ls, 1) == 0
    f = L.clusco_crmsd_batched
    assert f(h, -1, N, Ls, co, oo, FAKE, 1, FAKE, FAKE, size, None) == binding.ERR_INVALID_ARG
    assert f(h, 3, N, Ls, None, oo, FAKE, 1, FAKE, FAKE, size, None) == binding.ERR_INVALID_ARG
    assert f(h, 3, N, Ls, co, oo, None, 1, FAKE, FAKE, size, None) == binding.ERR_INVALID_ARG
    assert f(h, 3, N, Ls, co, oo, FAKE, 1, FAKE, FAKE, size - 1, None) == binding.ERR_WORKSPACE
    assert f(h, 3, N, Ls, _arr([0, -5, 0]), oo, FAKE, 1, FAKE, FAKE, size, None) == \
        binding.ERR_INVALID_ARG
    assert f(h, 3, N, Ls, co, oo, FAKE, 9, FAKE, FAKE, size, None) == binding.ERR_UNSUPPORTED
    # nothing to compute: E = 0, or every ensemble below two models
    assert f(h, 0, None, None, None, None, None, 1, None, None, 0, None) == binding.OK
    ones = _arr([1, 0])
    assert f(h, 2, ones, _arr([5, 5]), _arr([0, 15]), _arr([0, 0]), None, 1, None, None, 0,
             None) == binding.OK


def test_backward_argument_errors(L, h):
    f = L.clusco_crmsd_backward
    need = L.clusco_crmsd_backward_workspace_size(h, 64, 40, 0)
    assert need > L.clusco_crmsd_workspace_size(h, 64, 40, 0)
    assert need >= 12 * 4 * 64 * 63 // 2
    assert f(h, FAKE, 64, 0, FAKE, FAKE, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 64, 40, None, FAKE, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 64, 40, FAKE, FAKE, 0, None, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 64, 40, FAKE, FAKE, 0, FAKE, FAKE, need - 1, None) == binding.ERR_WORKSPACE
    assert f(h, FAKE, 64, 40, FAKE, FAKE, 8, FAKE, FAKE, need, None) == binding.ERR_UNSUPPORTED
    assert f(h, None, 0, 40, None, None, 0, None, None, 0, None) == binding.OK
    g = L.clusco_crmsd_cross_backward
    needc = L.clusco_crmsd_cross_backward_workspace_size(h, 64, 1, 40, 1)
    assert needc > 0
    assert g(h, FAKE, 64, FAKE, 1, 40, FAKE, FAKE, 1, None, FAKE, FAKE, needc, None) == \
        binding.ERR_INVALID_ARG
    assert g(h, FAKE, 64, FAKE, 1, 40, FAKE, FAKE, 1, FAKE, FAKE, FAKE, needc - 1, None) == \
        binding.ERR_WORKSPACE
    assert g(h, None, 64, FAKE, 1, 40, FAKE, FAKE, 1, FAKE, FAKE, FAKE, needc, None) == \
        binding.ERR_INVALID_ARG


def test_drmsd_sizes_and_argument_errors(L, h):
    s = L.clusco_drmsd_workspace_size(h, 1000, 150, 1)
    K = 150 * 149 // 2
    assert s % 256 == 0 and s >= 4 * 1024 * K          # operand vectors, 4 bytes a value
    assert L.clusco_drmsd_workspace_size(h, 1000, 150, 3) < 1024 * K   # FP64 keeps no operands
    assert L.clusco_drmsd_workspace_size(h, 10, 4097, 1) == 0
    assert L.clusco_drmsd_workspace_size(h, 10, 0, 1) == 0
    f = L.clusco_drmsd_matrix
    need = L.clusco_drmsd_workspace_size(h, 100, 50, 0)
    assert f(None, FAKE, 100, 50, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 0, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 50, 7, FAKE, FAKE, need, None) == binding.ERR_UNSUPPORTED
    assert f(h, FAKE, 100, 5000, 0, FAKE, FAKE, need, None) == binding.ERR_UNSUPPORTED
    assert f(h, None, 100, 50, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE_ODD, 100, 50, 0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 50, 0, FAKE, FAKE, need - 1, None) == binding.ERR_WORKSPACE
    assert f(h, FAKE, 100, 50, 0, FAKE, ctypes.c_void_p(0x10040), need, None) == \
        binding.ERR_INVALID_ARG
    assert f(h, None, 1, 50, 1, None, None, 0, None) == binding.OK


def test_kmedoids_sizes_and_argument_errors(L, h):
    assert L.clusco_cluster_workspace_size(h, 1000, 20) == 256 + 8192   # 8 N, 256-byte units
    assert L.clusco_cluster_workspace_size(h, 10, 11) == 0
    assert L.clusco_cluster_workspace_size(h, 10, 0) == 0
    f = L.clusco_kmedoids
    init = (ctypes.c_int32 * 3)(0, 5, 9)
    need = L.clusco_cluster_workspace_size(h, 10, 3)
    args = lambda **kw: [kw.get("h", h), kw.get("D", FAKE), kw.get("N", 10), kw.get("k", 3),
                         kw.get("init", init), kw.get("it", 50), kw.get("chk", 4), FAKE, FAKE,
                         FAKE, FAKE, FAKE, kw.get("ws", FAKE), kw.get("wsb", need), None]
    assert f(*args(h=None)) == binding.ERR_INVALID_ARG
    assert f(*args(k=11)) == binding.ERR_INVALID_ARG
    assert f(*args(it=-1)) == binding.ERR_INVALID_ARG
    assert f(*args(chk=-1)) == binding.ERR_INVALID_ARG
    assert f(*args(init=None)) == binding.ERR_INVALID_ARG
    assert f(*args(init=(ctypes.c_int32 * 3)(0, 5, 5))) == binding.ERR_INVALID_ARG   # not distinct
    assert f(*args(init=(ctypes.c_int32 * 3)(0, 5, 10))) == binding.ERR_INVALID_ARG  # out of range
    assert b"distinct" in L.clusco_last_error(h)
    assert f(*args(D=None)) == binding.ERR_INVALID_ARG
    assert f(*args(D=FAKE_ODD)) == binding.ERR_INVALID_ARG
    assert f(*args(wsb=need - 1)) == binding.ERR_WORKSPACE
    assert f(*args(ws=ctypes.c_void_p(0x10040))) == binding.ERR_INVALID_ARG


def test_cmo_sizes_and_argument_errors(L, h):
    K = 150 * 149 // 2
    s = L.clusco_cmo_workspace_size(h, 1000, 150)
    assert s % 256 == 0 and s >= 1024 * K                # one byte per (model, atom pair)
    assert L.clusco_cmo_workspace_size(h, 10, 4097) == 0
    assert L.clusco_cmo_workspace_size(h, 10, 0) == 0
    f = L.clusco_cmo_matrix
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_float,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    need = L.clusco_cmo_workspace_size(h, 100, 50)
    assert f(None, FAKE, 100, 50, 8.0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 0, 8.0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 50, -1.0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 50, float("nan"), FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 50, float("inf"), FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 5000, 8.0, FAKE, FAKE, need, None) == binding.ERR_UNSUPPORTED
    assert f(h, None, 100, 50, 8.0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE_ODD, 100, 50, 8.0, FAKE, FAKE, need, None) == binding.ERR_INVALID_ARG
    assert f(h, FAKE, 100, 50, 8.0, FAKE, FAKE, need - 1, None) == binding.ERR_WORKSPACE
    assert f(h, None, 1, 50, 8.0, None, None, 0, None) == binding.OK


def test_only_declared_functions_are_exported(L):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    c_names = {ln.split()[-1] for ln in out.splitlines()
               if ln.split()[1] == "T" and not ln.split()[-1].startswith("_")}
    assert c_names == set(declared_functions())


def test_flag_epsilon_model(L, h):
    """The error model's shape: none in FP64, the accumulation part growing
    with sqrt(steps), the x3 split above x4 (its dropped lo*lo' term)."""
    def eps(p, n):
        e = ctypes.c_double(-1.0)
        assert L.clusco_flag_epsilon(h, p, n, ctypes.byref(e)) == binding.OK
        return e.value
    assert eps(3, 150) == 0.0
    for p in (0, 1, 2, 4):
        assert 0.0 < eps(p, 150) < 1e-5
    assert eps(1, 150) > eps(4, 150) > 0.0
    assert eps(0, 600) > eps(0, 150) > eps(0, 16)
    assert eps(4, 640) > eps(4, 160)
    e = ctypes.c_double()
    assert L.clusco_flag_epsilon(h, 9, 150, ctypes.byref(e)) == binding.ERR_UNSUPPORTED
    assert L.clusco_flag_epsilon(h, 0, 0, ctypes.byref(e)) == binding.ERR_INVALID_ARG
    assert L.clusco_flag_epsilon(h, 0, 150, None) == binding.ERR_INVALID_ARG
