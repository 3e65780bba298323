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
    from paper_2604_02130_amd import build
    if build.is_stale(fd.LIB_PATH):
        build.build()
    return fd.load_library()


def test_library_matches_sources(lib):
    """The digest compiled into the library is that of the sources beside it."""
    from paper_2604_02130_amd import build
    assert fd.version().endswith("src " + build.source_digest())


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


def test_tune_table_roundtrip(lib, tmp_path):
    """The tuned-choice table loads, saves and steers the default segments."""
    fd.tune_clear()
    p = prob(128, 16)
    auto = fd.workspace_bytes([p], fd.FD_WHAT_GREENS)
    eight = fd.workspace_bytes([p], fd.FD_WHAT_GREENS, segments=8)
    assert auto != eight
    src = tmp_path / "t.txt"
    # what maxN maxNt nprob dk_micro s segments ms
    src.write_text("fdet-tune 1\n1 128 16 1 125000 4 8 1.5\n2 18 16 1 125000 16 1 0.25\n")
    assert fd.tune_load(str(src)) == 2
    assert fd.workspace_bytes([p], fd.FD_WHAT_GREENS) == eight
    out = tmp_path / "u.txt"
    fd.tune_save(str(out))
    lines = out.read_text().split("\n")
    assert lines[0] == "fdet-tune 1"
    assert "1 128 16 1 125000 4 8 1.5" in lines
    fd.tune_clear()
    assert fd.workspace_bytes([p], fd.FD_WHAT_GREENS) == auto
    bad = tmp_path / "bad.txt"
    bad.write_text("fdet-tune 1\n1 128 16 1 125000 0 8 1.5\n")
    with pytest.raises(fd.FdError):
        fd.tune_load(str(bad))
    bad.write_text("something else\n")
    with pytest.raises(fd.FdError):
        fd.tune_load(str(bad))
    fd.tune_clear()


def test_plan_and_autotune_reject_bad_arguments(lib):
    p = prob()
    o = fd.FdOptions(0, 0, 0, 0)
    h = ctypes.c_void_p(0)
    assert lib.fd_plan_create(fd.FD_WHAT_GREENS, ctypes.byref(p), 1, ctypes.byref(o), 0x10, 0x20,
                              None, None, 0x10000, 1 << 30, 0x40, None, None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_plan_create(fd.FD_WHAT_UDV, ctypes.byref(p), 1, ctypes.byref(o), 0x10, 0x20,
                              None, None, 0x10000, 1 << 30, 0x40, None,
                              ctypes.byref(h)) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_plan_create(fd.FD_WHAT_FORCE, ctypes.byref(p), 1, ctypes.byref(o), 0x10, None,
                              None, None, 0x10000, 1 << 30, 0x40, None,
                              ctypes.byref(h)) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_plan_launch(None, None) == fd.FD_ERR_INVALID_ARG
    best = fd.FdOptions()
    assert lib.fd_autotune(fd.FD_WHAT_UDV, ctypes.byref(p), 1, None, None, ctypes.byref(best),
                           None) == fd.FD_ERR_INVALID_ARG


@pytest.mark.parametrize("Nt", [1, 5, 16, 17, 33, 256, 512])
@pytest.mark.parametrize("c", [1, 3, 16, 64])
def test_force_plan_layout(lib, Nt, c):
    """The force plan (interval chains, prefix / suffix scans, checkpoint
    items) fits the descriptor region it counted, for ragged N_t / c."""
    n = fd.workspace_bytes([prob(18, Nt)], fd.FD_WHAT_FORCE, checkpoint=c)
    m = fd.workspace_bytes([prob(18, Nt), prob(50, Nt + 3)], fd.FD_WHAT_FORCE, checkpoint=c)
    assert 0 < n < m and n % 256 == 0


def test_response_trace_workspace_and_argument_checks(lib):
    """Observables entry point: workspace size per 32 x 32 tile, and every bad
    argument rejected on the host before a launch."""
    assert lib.fd_response_trace_workspace_bytes(0) == 0
    assert lib.fd_response_trace_workspace_bytes(fd.MAX_N + 1) == 0
    assert lib.fd_response_trace_workspace_bytes(1) == 256
    assert lib.fd_response_trace_workspace_bytes(72) == 512          # 9 tiles x 32 B, rounded up
    assert lib.fd_response_trace_workspace_bytes(512) == 256 * 32    # 256 tiles x 32 B
    ws = 0x10000
    assert lib.fd_response_trace(0, 0x1000, 0, 0x2000, ws, 4096, None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_response_trace(8, 0, 0, 0x2000, ws, 4096, None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_response_trace(8, 0x1000, 0, 0, ws, 4096, None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_response_trace(8, 0x1000, 0, 0x2000, 0, 4096, None) == fd.FD_ERR_WORKSPACE
    assert lib.fd_response_trace(8, 0x1000, 0, 0x2000, ws + 8, 4096, None) == fd.FD_ERR_WORKSPACE
    assert lib.fd_response_trace(72, 0x1000, 0, 0x2000, ws, 255, None) == fd.FD_ERR_WORKSPACE


def test_hmc_workspace_and_argument_checks(lib):
    """Leapfrog entry point: its workspace holds the force's and more; bad
    arguments are rejected on the host before a launch."""
    P = prob(18, 16)
    force = fd.workspace_bytes([P], fd.FD_WHAT_FORCE, checkpoint=8)
    hmc = fd.workspace_bytes([P], fd.FD_WHAT_HMC, checkpoint=8)
    assert hmc >= force + 18 * 16 * 8 and hmc % 256 == 0
    arr = (fd.FdProblem * 1)(P)
    o = fd.FdOptions(4, 8, 0, 0)
    ws, pi, dH, st = 0x100000, 0x1000, 0x2000, 0x3000
    call = lambda **kw: lib.fd_hmc_leapfrog(
        arr, kw.get("n", 1), ctypes.byref(o), kw.get("dU", 0.75), kw.get("eps", 0.1),
        kw.get("steps", 3), kw.get("pi", pi), kw.get("dH", dH), ws, hmc, kw.get("st", st), None)
    assert call(dU=0.0) == fd.FD_ERR_INVALID_ARG
    assert call(dU=float("inf")) == fd.FD_ERR_INVALID_ARG
    assert call(eps=float("nan")) == fd.FD_ERR_INVALID_ARG
    assert call(steps=0) == fd.FD_ERR_INVALID_ARG
    assert call(pi=0) == fd.FD_ERR_INVALID_ARG
    assert call(dH=0) == fd.FD_ERR_INVALID_ARG
    assert call(st=0) == fd.FD_ERR_INVALID_ARG
    assert call(n=0) == fd.FD_ERR_INVALID_ARG


def test_diag_response_argument_checks(lib):
    f, fi, out = 0x1000, 0x2000, 0x3000
    assert lib.fd_diag_response(0, 8, f, fi, 0, out, None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_diag_response(4, 0, f, fi, 0, out, None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_diag_response(4, fd.MAX_N + 1, f, fi, 0, out, None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_diag_response(4, 8, 0, fi, 0, out, None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_diag_response(4, 8, f, 0, 0, out, None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_diag_response(4, 8, f, fi, 0, 0, None) == fd.FD_ERR_INVALID_ARG


def test_hmc_plan_argument_checks(lib):
    P = prob(18, 16)
    arr = (fd.FdProblem * 1)(P)
    o = fd.FdOptions(4, 8, 0, 0)
    hmc = fd.workspace_bytes([P], fd.FD_WHAT_HMC, checkpoint=8)
    h = ctypes.c_void_p(0)
    ws, pi, dH, st = 0x100000, 0x1000, 0x2000, 0x3000
    assert lib.fd_hmc_plan_create(arr, 1, ctypes.byref(o), 0.75, 0.1, 3, pi, dH, ws, hmc, st, None,
                                  None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_hmc_plan_create(arr, 1, ctypes.byref(o), -1.0, 0.1, 3, pi, dH, ws, hmc, st, None,
                                  ctypes.byref(h)) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_hmc_plan_create(arr, 1, ctypes.byref(o), 0.75, 0.1, 0, pi, dH, ws, hmc, st, None,
                                  ctypes.byref(h)) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_hmc_plan_create(arr, 1, ctypes.byref(o), 0.75, 0.1, 3, 0, dH, ws, hmc, st, None,
                                  ctypes.byref(h)) == fd.FD_ERR_INVALID_ARG
    assert not h.value
    assert lib.fd_hmc_plan_launch(None, None) == fd.FD_ERR_INVALID_ARG
    lib.fd_hmc_plan_destroy(None)


def test_header_is_plain_c(lib, tmp_path):
    """include/fdet.h compiles as strict C99 (no C++ in the boundary), and a C
    program links against the library's exported names."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    src = tmp_path / "use.c"
    src.write_text('#include "fdet.h"\n'
                   "int main(void) {\n"
                   "  fd_options o = {0, 0, 0, 0};\n"
                   "  (void)o;\n"
                   "  return fd_response_trace_workspace_bytes(0) == 0 ? 0 : 1;\n"
                   "}\n")
    inc = os.path.join(ROOT, "include")
    res = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", inc,
                          "-o", str(tmp_path / "use"), str(src), fd.LIB_PATH,
                          f"-Wl,-rpath,{os.path.dirname(fd.LIB_PATH)}"],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    run = subprocess.run([str(tmp_path / "use")], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0, run.stderr[-2000:]


def test_greens_noalloc_argument_checks(lib):
    """fd_greens_noalloc rejects missing outputs and a call larger than its
    fixed array before it looks up a device (no GPU needed)."""
    p = prob(N=512, Nt=512, dk=0.125)
    o = fd.FdOptions(16, 0, 32, 0)
    rc = lib.fd_greens_noalloc(ctypes.byref(p), ctypes.byref(o), 0x3000, 0x5000, 0x4000, None)
    assert rc == fd.FD_ERR_WORKSPACE
    assert "fixed" in lib.fd_last_error().decode()
    p = prob()
    assert lib.fd_greens_noalloc(ctypes.byref(p), None, 0x3000, None, 0x4000, None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_greens_noalloc(ctypes.byref(p), None, 0x3000, 0x5000, None, None) == fd.FD_ERR_INVALID_ARG
    # within the limit: the workspace the call would use fits the fixed array
    assert 0 < lib.fd_workspace_bytes(ctypes.byref(p), 1, None, fd.FD_WHAT_GREENS) <= (64 << 20)


def test_single_launch_flag_is_switched_off(lib):
    """FD_SINGLE_LAUNCH returns FD_ERR_UNSUPPORTED before anything is enqueued."""
    p = prob()
    o = fd.FdOptions(4, 0, 0, fd.FD_SINGLE_LAUNCH)
    rc = lib.fd_logdet(ctypes.byref(p), ctypes.byref(o), 0x3000, 0x10000, 1 << 30, 0x4000, None)
    assert rc == fd.FD_ERR_UNSUPPORTED
    assert "switched off" in lib.fd_last_error().decode()


def test_displaced_argument_checks(lib):
    p = prob(N=18, Nt=16)
    assert lib.fd_displaced_workspace_bytes(ctypes.byref(p), None, 0) == 0
    n1 = lib.fd_displaced_workspace_bytes(ctypes.byref(p), None, 1)
    n3 = lib.fd_displaced_workspace_bytes(ctypes.byref(p), None, 3)
    assert 0 < n1 < n3
    t = (ctypes.c_int32 * 2)(1, 17)
    t0 = (ctypes.c_int32 * 2)(1, 1)
    rc = lib.fd_greens_displaced(ctypes.byref(p), None, 2, t, t0, 0x5000, 0x10000, 1 << 30,
                                 0x4000, None)
    assert rc == fd.FD_ERR_INVALID_ARG and "outside" in lib.fd_last_error().decode()
    t = (ctypes.c_int32 * 2)(1, 16)
    assert lib.fd_greens_displaced(ctypes.byref(p), None, 2, t, t0, None, 0x10000, 1 << 30,
                                   0x4000, None) == fd.FD_ERR_INVALID_ARG
    assert lib.fd_greens_displaced(ctypes.byref(p), None, 2, t, t0, 0x5000, 0x10000, 256,
                                   0x4000, None) == fd.FD_ERR_WORKSPACE


def test_force_response_argument_checks(lib):
    p = prob(N=18, Nt=16)
    for A, tr in ((None, 0x5000), (0x5000, None)):
        rc = lib.fd_force_response(ctypes.byref(p), None, A, tr, None, 0x6000, None, 0x10000,
                                   1 << 30, 0x4000, None)
        assert rc == fd.FD_ERR_INVALID_ARG and "A and trace" in lib.fd_last_error().decode()
    rc = lib.fd_force_response(ctypes.byref(p), None, 0x5000, 0x5000, None, None, None, 0x10000,
                               1 << 30, 0x4000, None)
    assert rc == fd.FD_ERR_INVALID_ARG


def test_force_response_rejects_blocked_class(lib):
    p = prob(N=162, Nt=16)
    rc = lib.fd_force_response(ctypes.byref(p), None, 0x5000, 0x5000, None, 0x6000, None, 0x10000,
                               1 << 30, 0x4000, None)
    assert rc == fd.FD_ERR_UNSUPPORTED and "N > 128" in lib.fd_last_error().decode()


def test_sparse_argument_checks(lib):
    p = prob(N=18, Nt=16, K=0)
    h = fd.FdEll(3, 0x1000, 0x2000)
    o = fd.FdOptions(8, 0, 0, 0)
    assert lib.fd_sparse_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), fd.FD_WHAT_GREENS) > 0
    assert lib.fd_sparse_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), fd.FD_WHAT_FORCE) == 0
    args = (0x5000, 0x6000, 0x10000, 1 << 30, 0x4000, None)
    assert lib.fd_sparse_greens(ctypes.byref(p), ctypes.byref(h), 9, ctypes.byref(o), *args) \
        == fd.FD_ERR_INVALID_ARG
    bad = fd.FdEll(0, 0x1000, 0x2000)
    assert lib.fd_sparse_greens(ctypes.byref(p), ctypes.byref(bad), 4, ctypes.byref(o), *args) \
        == fd.FD_ERR_INVALID_ARG
    o2 = fd.FdOptions(32, 0, 0, 0)
    assert lib.fd_sparse_greens(ctypes.byref(p), ctypes.byref(h), 4, ctypes.byref(o2), *args) \
        == fd.FD_ERR_INVALID_ARG and "s <= 16" in lib.fd_last_error().decode()
    o3 = fd.FdOptions(8, 0, 0, fd.FD_KEEP_CHECKPOINTS)
    assert lib.fd_sparse_greens(ctypes.byref(p), ctypes.byref(h), 4, ctypes.byref(o3), *args) \
        == fd.FD_ERR_INVALID_ARG
    assert lib.fd_sparse_greens(ctypes.byref(p), ctypes.byref(h), 4, ctypes.byref(o),
                                0x5000, 0x6000, 0x10000, 256, 0x4000, None) == fd.FD_ERR_WORKSPACE
