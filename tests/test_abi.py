"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, sizes workspaces, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

import paper_2604_02130_amd as fd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "fdet.h")).read()
    return sorted(set(re.findall(r"\b(fd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fd.LIB_PATH):
        from paper_2604_02130_amd import build
        build.build()
    return fd.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_symbols()
    assert "fd_greens" in names and "fd_force_batched" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(fd.SYMBOLS)


def test_version_and_strerror(lib):
    assert "gfx950" in fd.version()
    assert fd.strerror(fd.FD_ERR_SINGULAR) == "M is singular"
    assert fd.strerror(12345) == "unknown code"


def prob(N=18, Nt=16, dk=0.125, K=0x1000, phi=0x2000):
    return fd.FdProblem(N, Nt, dk, K, phi)


def test_workspace_sizes_grow_with_problem(lib):
    small = fd.workspace_bytes([prob(18, 16)], fd.FD_WHAT_GREENS)
    big = fd.workspace_bytes([prob(128, 16)], fd.FD_WHAT_GREENS)
    seg = fd.workspace_bytes([prob(128, 16)], fd.FD_WHAT_GREENS, segments=4)
    force = fd.workspace_bytes([prob(128, 256)], fd.FD_WHAT_FORCE, checkpoint=16)
    batch = fd.workspace_bytes([prob(18, 16), prob(128, 16)], fd.FD_WHAT_GREENS)
    assert 0 < small < big < seg
    assert force > big
    assert batch > big
    assert batch % 256 == 0


@pytest.mark.parametrize("bad", [
    dict(N=0), dict(N=fd.MAX_N + 1), dict(Nt=0), dict(K=0), dict(phi=0),
])
def test_invalid_problem_rejected(lib, bad):
    args = dict(N=18, Nt=16, dk=0.125, K=0x1000, phi=0x2000)
    args.update(bad)
    p = prob(**args)
    o = fd.FdOptions(4, 16, 1, 0)
    rc = lib.fd_logdet(ctypes.byref(p), ctypes.byref(o), 0x3000, 0x10000, 1 << 30, 0x4000, None)
    assert rc == fd.FD_ERR_INVALID_ARG
    assert lib.fd_last_error().decode()


def test_nonfinite_dk_rejected(lib):
    p = prob(dk=float("nan"))
    rc = lib.fd_logdet(ctypes.byref(p), None, 0x3000, 0x10000, 1 << 30, 0x4000, None)
    assert rc == fd.FD_ERR_NONFINITE


def test_workspace_errors(lib):
    p = prob()
    need = fd.workspace_bytes([p], fd.FD_WHAT_LOGDET)
    rc = lib.fd_logdet(ctypes.byref(p), None, 0x3000, 0x10000, need - 1, 0x4000, None)
    assert rc == fd.FD_ERR_WORKSPACE and "too small" in lib.fd_last_error().decode()
    rc = lib.fd_logdet(ctypes.byref(p), None, 0x3000, 0x10008, need, 0x4000, None)
    assert rc == fd.FD_ERR_WORKSPACE and "aligned" in lib.fd_last_error().decode()
    rc = lib.fd_logdet(ctypes.byref(p), None, 0x3000, None, need, 0x4000, None)
    assert rc == fd.FD_ERR_WORKSPACE


def test_missing_outputs_rejected(lib):
    p = prob()
    rc = lib.fd_greens(ctypes.byref(p), None, 0x3000, None, 0x10000, 1 << 30, 0x4000, None)
    assert rc == fd.FD_ERR_INVALID_ARG
    rc = lib.fd_force(ctypes.byref(p), None, None, None, None, 0x10000, 1 << 30, 0x4000, None)
    assert rc == fd.FD_ERR_INVALID_ARG
    rc = lib.fd_logdet(ctypes.byref(p), None, 0x3000, 0x10000, 1 << 30, None, None)
    assert rc == fd.FD_ERR_INVALID_ARG


def test_bad_options_rejected(lib):
    p = prob()
    o = fd.FdOptions(0, 100, 0, 0)
    rc = lib.fd_force(ctypes.byref(p), ctypes.byref(o), None, 0x3000, None, 0x10000, 1 << 30,
                      0x4000, None)
    assert rc == fd.FD_ERR_INVALID_ARG


def test_python_layer_requires_gpu_tensors():
    import torch
    K = torch.zeros((4, 4), dtype=torch.float64)
    phi = torch.zeros((2, 4), dtype=torch.float64)
    with pytest.raises(fd.FdError):
        fd.greens(K, phi, 0.1)
