"""Build libfdet.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2604_02130_amd.build

The kernels are compiled once per launch class (-DFDET_NC=...), each into an
object of its own, in parallel; the library is then linked from the objects.
A digest of the sources under csrc/ and include/ is compiled into the library
(fd_version), so that the binding can refuse a library built from other
sources.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfdet.so")

KERNEL_CLASSES = (32, 64, 80, 96, 128, 512)
OTHER_SOURCES = ["fdet_obs.hip", "fdet_hmc.hip", "fdet_noalloc.hip", "fdet_abi.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-variable",
]


def source_digest() -> str:
    """sha256 (first 16 hex digits) over the names and bytes of every file in
    csrc/ and include/, in sorted order."""
    h = hashlib.sha256()
    for d in (CSRC, INCLUDE):
        for name in sorted(os.listdir(d)):
            path = os.path.join(d, name)
            if os.path.isfile(path):
                with open(path, "rb") as f:
                    h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def library_digest(path: str = LIB) -> str | None:
    """The source digest compiled into a built library (read from the file,
    without loading it), or None."""
    import re
    try:
        with open(path, "rb") as f:
            data = f.read()
    except OSError:
        return None
    m = re.search(rb"fdet \d+\.\d+\.\d+ \(gfx950\) src ([0-9a-f]{16})", data)
    return m.group(1).decode() if m else None


def is_stale(path: str = LIB) -> bool:
    """True if the library is missing or was built from other sources."""
    return library_digest(path) != source_digest()


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP/C++ source and link libfdet.so next to this file."""
    cc = hipcc()
    digest = source_digest()
    jobs = jobs or min(8, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="fdet_build_") as tmpd:
        units = [(os.path.join(CSRC, "fdet_kernels.hip"), [f"-DFDET_NC={c}"], f"k{c}.o")
                 for c in (512, 128, 96, 80, 64, 32)]
        units += [(os.path.join(CSRC, s), [f'-DFDET_SRC_DIGEST="{digest}"'], s + ".o")
                  for s in OTHER_SOURCES]
        pending = list(units)
        running = []
        objs = []
        failed = None
        while pending or running:
            while pending and len(running) < jobs and failed is None:
                src, extra, obj = pending.pop(0)
                out = os.path.join(tmpd, obj)
                cmd = [cc, *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-c", "-o", out, src]
                if verbose:
                    print(" ".join(cmd), flush=True)
                running.append((subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                 stderr=subprocess.STDOUT, text=True), out))
                objs.append(out)
            if failed is not None and not running:
                break
            proc, out = running.pop(0)
            text, _ = proc.communicate()
            if proc.returncode != 0:
                sys.stderr.write(text)
                failed = failed or f"hipcc failed on {os.path.basename(out)} ({proc.returncode})"
                pending.clear()
        if failed:
            raise RuntimeError(failed)
        tmp = LIB + ".tmp"
        cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"link failed with exit code {res.returncode}")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
