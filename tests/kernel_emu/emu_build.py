"""Host builds of the library's HIP sources for the CPU checks (test
infrastructure; the package never loads these libraries).

Two builds of the same sources (paper_2604_02130_amd/csrc) through the
header hip/hip_runtime.h of this folder:

  asan  AddressSanitizer + array-bounds checks on every translation unit:
        overflows of device buffers (each its own host allocation), of per-lane
        private arrays and of shared-memory objects, and indexes past a member
        array of the shared-memory struct.
  race  the kernels instrumented for emu_race.cpp: races between waves of a
        workgroup and between lanes of one wave (no barrier between two
        accesses, one a write), between workgroups of one launch, and reads of
        shared memory the workgroup never wrote.

Only the size classes asked for are compiled (32 and 512 by default: the
register/LDS code and the blocked code); the others are stubs that fail
loudly.  Libraries are cached under the system temporary folder by a digest
of every source they are built from.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2604_02130_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
ALL_CLASSES = (32, 64, 80, 96, 128, 512)

_COMMON = ["-std=c++17", "-fPIC", "-O1", "-g", "-Wno-unused-variable", "-Wno-unknown-pragmas",
           "-Wno-pass-failed", "-Wno-psabi", "-I", HERE, "-I", INCLUDE]
_ASAN = ["-fno-omit-frame-pointer", "-fsanitize=address,array-bounds", "-fstrict-flex-arrays=3",
         "-fno-sanitize-recover=all"]
MODES = {
    # (flags of kernel units, flags of host units, link flags, extra host sources)
    "asan": (_ASAN, _ASAN, ["-fsanitize=address,array-bounds", "-shared-libasan"], []),
    "race": (["-fsanitize=thread", "-DEMU_LDS_SECTION", "-DEMU_RACE"],
             ["-DEMU_LDS_SECTION", "-DEMU_RACE"], ["-ldl"], ["emu_race.cpp"]),
    # no checker: the fastest build, for counting work (MFMA instructions per launch)
    "plain": (["-O2"], ["-O2"], [], []),
}


def clang() -> str | None:
    for cand in (os.environ.get("FDET_EMU_CLANG"), "/opt/rocm/llvm/bin/clang++"):
        if cand and os.path.exists(cand):
            return cand
    return None


def asan_runtime() -> str | None:
    cc = clang()
    if not cc:
        return None
    path = subprocess.run([cc, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def digest(mode: str, classes) -> str:
    h = hashlib.sha256(f"{mode} {sorted(classes)}".encode())
    for d in (CSRC, INCLUDE, HERE, os.path.join(HERE, "hip")):
        for name in sorted(os.listdir(d)):
            path = os.path.join(d, name)
            if os.path.isfile(path) and name.endswith((".hip", ".hpp", ".h", ".cpp")):
                with open(path, "rb") as f:
                    h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def build(mode: str = "asan", classes=(32, 512), out_dir: str | None = None, jobs: int = 8) -> str:
    """Build (or take from the cache) the host library; returns its path."""
    cc = clang()
    if cc is None:
        raise RuntimeError("clang++ not found (set FDET_EMU_CLANG)")
    kflags, hflags, lflags, extra = MODES[mode]
    classes = tuple(sorted(classes))
    if 32 not in classes:
        raise ValueError("class 32 holds the status kernel and is always built")
    out_dir = out_dir or os.path.join(tempfile.gettempdir(), "fdet_kernel_emu")
    os.makedirs(out_dir, exist_ok=True)
    lib = os.path.join(out_dir, f"libfdet_{mode}_{'-'.join(map(str, classes))}_{digest(mode, classes)}.so")
    if os.path.exists(lib):
        return lib
    with tempfile.TemporaryDirectory(prefix="fdet_emu_") as tmp:
        units = []
        for c in classes:
            units.append((["-x", "c++", *kflags, f"-DFDET_NC={c}", f"-Dfdet=fdet_c{c}"],
                          os.path.join(CSRC, "fdet_kernels.hip"), f"k{c}.o"))
        for src, ns in (("fdet_obs.hip", "fdet_obs"), ("fdet_hmc.hip", "fdet_hmc"),
                        ("fdet_noalloc.hip", "fdet_na")):
            units.append((["-x", "c++", *kflags, f"-Dfdet={ns}"], os.path.join(CSRC, src), src + ".o"))
        units.append((["-x", "c++", *hflags, '-DFDET_SRC_DIGEST="host-emulation00"'],
                      os.path.join(CSRC, "fdet_abi.cpp"), "abi.o"))
        units.append((hflags, os.path.join(HERE, "emu_runtime.cpp"), "rt.o"))
        stubs = [f"-DEMU_STUB_{c}" for c in ALL_CLASSES if c not in classes and c != 32]
        units.append((hflags + stubs, os.path.join(HERE, "emu_stubs.cpp"), "stubs.o"))
        for src in extra:
            units.append((hflags, os.path.join(HERE, src), src + ".o"))
        objs, running, err = [], [], None
        pending = list(units)
        while pending or running:
            while pending and len(running) < jobs:
                flags, src, obj = pending.pop(0)
                out = os.path.join(tmp, obj)
                objs.append(out)
                running.append((subprocess.Popen([cc, *_COMMON, *flags, "-c", "-o", out, src],
                                                 stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                                 text=True), src))
            proc, src = running.pop(0)
            text, _ = proc.communicate()
            if proc.returncode != 0 and err is None:
                err = f"{os.path.basename(src)}: {text[-4000:]}"
                pending.clear()
        if err:
            raise RuntimeError("host build failed: " + err)
        tmp_lib = lib + f".{os.getpid()}.tmp"
        res = subprocess.run([cc, "-shared", *lflags, "-o", tmp_lib, *objs], capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("host link failed: " + res.stderr[-4000:])
        os.replace(tmp_lib, lib)
    return lib


def build_selftest(mode: str = "asan", out_dir: str | None = None) -> str:
    """The checkers' self-test program (emu_selftest.hip) for one build mode."""
    cc = clang()
    if cc is None:
        raise RuntimeError("clang++ not found (set FDET_EMU_CLANG)")
    kflags, hflags, lflags, extra = MODES[mode]
    out_dir = out_dir or os.path.join(tempfile.gettempdir(), "fdet_kernel_emu")
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, f"selftest_{mode}_{digest(mode, ('selftest',))}")
    if os.path.exists(exe):
        return exe
    with tempfile.TemporaryDirectory(prefix="fdet_emu_") as tmp:
        objs = []
        units = [(["-x", "c++", *kflags], os.path.join(HERE, "emu_selftest.hip"), "selftest.o"),
                 (hflags, os.path.join(HERE, "emu_runtime.cpp"), "rt.o")]
        units += [(hflags, os.path.join(HERE, src), src + ".o") for src in extra]
        for flags, src, obj in units:
            out = os.path.join(tmp, obj)
            res = subprocess.run([cc, *_COMMON, *flags, "-c", "-o", out, src], capture_output=True, text=True)
            if res.returncode != 0:
                raise RuntimeError(f"self-test build failed: {res.stdout[-2000:]}{res.stderr[-2000:]}")
            objs.append(out)
        link = [f for f in lflags if f != "-shared-libasan"]
        tmp_exe = exe + f".{os.getpid()}.tmp"
        res = subprocess.run([cc, *link, "-o", tmp_exe, *objs], capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("self-test link failed: " + res.stderr[-4000:])
        os.replace(tmp_exe, exe)
    return exe


if __name__ == "__main__":
    import sys
    mode = sys.argv[1] if len(sys.argv) > 1 else "asan"
    classes = tuple(int(c) for c in sys.argv[2:]) or (32, 512)
    print(build(mode, classes))
