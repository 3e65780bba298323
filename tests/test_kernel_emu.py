"""The library's HIP kernels built for the host and run on the CPU under
checkers (tests/kernel_emu): no GPU involved, and nothing here is loaded by the
package.

Two builds of the unmodified sources in paper_2604_02130_amd/csrc:
  asan  AddressSanitizer + array-bounds: overflows of device buffers, of
        per-lane private arrays, of shared-memory objects and past member
        arrays of the shared-memory struct (the smaller classes' layouts
        reinterpreted inside a larger class's included);
  race  races between waves of a workgroup, between lanes of one wave (no
        barrier between a write and another lane's access: the compiler may
        reorder a lane's own accesses), between workgroups of one launch (work
        items that share workspace), and shared-memory reads before any write
        in the workgroup.
Both run every lane as a fiber, so they also catch barriers that some lanes
never reach and wave-level operations (MFMA, DPP, shuffles) taken by part of a
wave.  The launch classes built are 32 and 128 (register QR, LDS products)
and 512 (blocked QR, MFMA products from device memory).  Class 128 runs a
mixed batch (N = 18 to 128 in one launch: each item on its own class's code
and the class-128 shared-memory layout); class 512 runs through batches with
one N = 130 problem, whose smaller members then run the blocked code too.
The other entry points run at class 32: prepared plans (launched twice, bit
for bit the eager calls, also with FD_REUSE_E), FD_KEEP_CHECKPOINTS, fd_udv,
the slice exponential, the observables, the leapfrog and its prepared
trajectory, and the allocation-free G (bit for bit fd_greens).
With FDET_EMU_ALL=1 every class is built, and the mixed batch's force and a
class-80 force run as well (a few minutes more).
FDET_EMU_FULL=1 adds the named workloads at full size (lowT_L6 det + G with
32 segments, force_L8) and the HMC step's N = 512 shape (field 0's first 32
slices, s = c = 16): tens of minutes.
Every case is also compared with the oracle (relative deviation at most
1e-10), and the checkers are pinned by a self-test that plants each kind of
mistake in a small kernel and expects it reported.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "kernel_emu")
sys.path.insert(0, EMU)
emu_build = pytest.importorskip("emu_build", reason="tests/kernel_emu is not present")

pytestmark = pytest.mark.slow

CASES = ["greens", "force_windows", "force_scans", "response", "displaced", "sparse",
         "batch_greens", "batch_force", "b512_greens", "b512_force", "b512_force_scans",
         "b512_displaced", "b512_sparse",
         "plans", "keep_checkpoints", "udv_exp", "observables", "leapfrog", "noalloc"]
FULL = os.environ.get("FDET_EMU_FULL") == "1"
ALL = FULL or os.environ.get("FDET_EMU_ALL") == "1"
CLASSES = emu_build.ALL_CLASSES if ALL else (32, 128, 512)
CASES += ["mixed_greens"]
if ALL:
    CASES += ["mixed_force", "class80_force"]
if FULL:
    CASES += ["full_lowT_L6", "full_force_L8", "full_n512_force"]
MODES = ["asan", "race"]
TOL = 1e-10
TIMEOUT = 7200 if FULL else 900

# planted mistake -> (build, text the report must contain)
SELFTEST = {
    "wave_race": ("race", "another wave"),
    "group_race": ("race", "another workgroup"),
    "uninit_shared": ("race", "never wrote"),
    "member_oob": ("asan", "out of bounds for type 'double[512]'"),
    "heap_oob": ("asan", "heap-buffer-overflow"),
    "private_oob": ("asan", "out of bounds for type 'double[4]'"),
    "divergent_wave": ("asan", "deadlock"),
    "lane_race": ("race", "another lane of the wave"),
}


def _env(preload):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    env["ASAN_OPTIONS"] = "detect_leaks=0:detect_stack_use_after_return=0"
    if preload:   # a Python process loading the shared-runtime ASan library
        env["LD_PRELOAD"] = emu_build.asan_runtime()
    return env


def _run(cmd, preload):
    try:
        p = subprocess.run(cmd, capture_output=True, text=True, timeout=TIMEOUT, env=_env(preload))
        return p.returncode, p.stdout, p.stderr
    except subprocess.TimeoutExpired:
        return -1, "", f"timed out after {TIMEOUT} s"


@pytest.fixture(scope="module")
def emu():
    if emu_build.clang() is None or emu_build.asan_runtime() is None:
        pytest.skip("clang++ with its AddressSanitizer runtime is not installed")
    with cf.ThreadPoolExecutor(4) as ex:
        libs = {m: ex.submit(emu_build.build, m, CLASSES, None, 4) for m in MODES}
        exes = {m: ex.submit(emu_build.build_selftest, m) for m in MODES}
        libs = {m: f.result() for m, f in libs.items()}
        exes = {m: f.result() for m, f in exes.items()}
    jobs = {}
    workers = max(2, min(8, os.cpu_count() or 2))
    with cf.ThreadPoolExecutor(workers) as ex:
        # the longest cases first
        for case in sorted(CASES, key=lambda c: (not c.startswith("full"),
                                                 not c.startswith(("b512", "mixed", "class80")))):
            for m in MODES:
                jobs[("case", m, case)] = ex.submit(
                    _run, [sys.executable, os.path.join(EMU, "emu_cases.py"), libs[m], case], m == "asan")
        # the self-test programs link their sanitizer runtime statically
        for mode, (m, _) in SELFTEST.items():
            jobs[("self", m, mode)] = ex.submit(_run, [exes[m], mode], False)
        for m in MODES:
            jobs[("self", m, "ok")] = ex.submit(_run, [exes[m], "ok"], False)
        return {k: f.result() for k, f in jobs.items()}


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", CASES)
def test_host_build_case(emu, mode, case):
    rc, out, err = emu[("case", mode, case)]
    assert rc == 0, f"exit status {rc}\n{err[-4000:]}"
    for bad in ("EMU ERROR", "EMU RACE", "runtime error", "AddressSanitizer"):
        assert bad not in err, err[-4000:]
    rec = json.loads(out.strip().splitlines()[-1])
    assert rec["status"] == [0] * len(rec["status"])
    assert rec["worst"] <= TOL, rec
    assert rec["barrier_site_mismatch"] == 0, rec
    if mode == "race":
        assert rec["races"] == 0 and rec["lane_races"] == 0 and rec["checked_accesses"] > 0, rec


@pytest.mark.parametrize("mode", MODES)
def test_selftest_clean_kernel(emu, mode):
    rc, out, err = emu[("self", mode, "ok")]
    assert rc == 0, err[-2000:]
    rec = json.loads(out.strip().splitlines()[-1])
    assert rec["races"] == 0 and rec["lane_races"] == 0 and rec["barrier_site_mismatch"] == 0
    assert "EMU" not in err and "runtime error" not in err


@pytest.mark.parametrize("planted", sorted(SELFTEST))
def test_selftest_reports_planted_mistake(emu, planted):
    mode, text = SELFTEST[planted]
    rc, out, err = emu[("self", mode, planted)]
    assert text in err, f"exit {rc}; stderr:\n{err[-2000:]}"
