"""One case of the host-built library against the oracle (test infrastructure).

    python emu_cases.py <library> <case>

Calls the library's C ABI through ctypes with host buffers (each input, output
and workspace its own allocation from the host build's hipMalloc, of exactly
the size the call needs, the workspace filled with NaN bytes), compares the
results with the oracle and prints one JSON line: the largest deviation
(relative to max(1, max |oracle value|); log det relative to max(1, |log det|)),
the status words and the run's counters (launches, workgroups, barriers,
wave-level operations, barrier-site mismatches and, for the race build, the
numbers of distinct races between waves or workgroups and between lanes of one
wave).  A sanitizer finding or an emulation error aborts
the process before that line is printed.  For the AddressSanitizer build the
caller preloads its runtime.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
from workload import Workload, honeycomb_hopping, sample_phi  # noqa: E402

FD_WHAT_GREENS, FD_WHAT_FORCE = 1, 2
FD_FORCE_SCANS = 0x2

lib = None


class Prob(C.Structure):
    _fields_ = [("N", C.c_int32), ("Nt", C.c_int32), ("dk", C.c_double), ("K", C.c_void_p),
                ("phi", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("s", C.c_int32), ("checkpoint", C.c_int32), ("segments", C.c_int32),
                ("flags", C.c_int32)]


class Ell(C.Structure):
    _fields_ = [("q", C.c_int32), ("col", C.c_void_p), ("val", C.c_void_p)]


def load(path):
    global lib
    lib = C.CDLL(path)
    for f in ("fd_workspace_bytes", "fd_displaced_workspace_bytes", "fd_sparse_workspace_bytes"):
        getattr(lib, f).restype = C.c_size_t
    lib.fd_last_error.restype = C.c_char_p
    lib.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    lib.hipFree.argtypes = [C.c_void_p]
    lib.emu_set_fill(0xFF)


class Buf:
    """Host-build device buffer of exactly `nbytes` (NaN bytes unless given)."""

    def __init__(self, nbytes, src=None):
        p = C.c_void_p()
        assert lib.hipMalloc(C.byref(p), nbytes) == 0
        self.p = p.value
        if src is not None:
            a = np.ascontiguousarray(src)
            assert a.nbytes == nbytes
            C.memmove(self.p, a.ctypes.data, nbytes)

    def get(self, dtype, shape):
        a = np.empty(shape, dtype)
        C.memmove(a.ctypes.data, self.p, a.nbytes)
        return a

    def __del__(self):
        lib.hipFree(self.p)


def check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what}: rc {rc}: {lib.fd_last_error().decode()}")


def problems(cfgs):
    keep, arr = [], (Prob * len(cfgs))()
    for i, (K, phi, dk) in enumerate(cfgs):
        bk, bp = Buf(K.nbytes, K), Buf(phi.nbytes, phi)
        keep += [bk, bp]
        arr[i] = Prob(K.shape[0], phi.shape[0], dk, bk.p, bp.p)
    return arr, keep


def cplx(a):
    return a[..., 0] + 1j * a[..., 1]


def rel(a, b):
    """Largest deviation of a from b relative to max(1, max |b|): rounding
    errors grow with the entries of G (and F, traces), not with 1."""
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max()) / max(1.0, float(np.abs(b).max()))


def dlog(a, b):
    d = a - b
    return abs(complex(d.real, math.remainder(d.imag, 2 * math.pi))) / max(1.0, abs(b))


def run_greens(cfgs, s, segments=0):
    P, keep = problems(cfgs)
    o = Opts(s, 0, segments, 0)
    n = len(cfgs)
    ws_n = lib.fd_workspace_bytes(P, n, C.byref(o), FD_WHAT_GREENS)
    assert ws_n > 0, lib.fd_last_error()
    ws, ld, st = Buf(ws_n), Buf(16 * n), Buf(4 * n)
    gsz = sum(2 * K.shape[0] ** 2 for K, _, _ in cfgs)
    G = Buf(8 * gsz)
    check(lib.fd_greens_batched(P, n, C.byref(o), C.c_void_p(ld.p), C.c_void_p(G.p), C.c_void_p(ws.p),
                                C.c_size_t(ws_n), C.c_void_p(st.p), None), "greens")
    Gall, out, off = G.get(np.float64, (gsz,)), [], 0
    for K, _, _ in cfgs:
        N = K.shape[0]
        out.append(cplx(Gall[off:off + 2 * N * N].reshape(N, N, 2)))
        off += 2 * N * N
    lds = ld.get(np.float64, (n, 2))
    return [complex(a, b) for a, b in lds], out, st.get(np.int32, (n,)).tolist()


def run_force(cfgs, s, c, flags=0, A=None):
    P, keep = problems(cfgs)
    o = Opts(s, c, 0, flags)
    n = len(cfgs)
    ws_n = lib.fd_workspace_bytes(P, n, C.byref(o), FD_WHAT_FORCE)
    assert ws_n > 0, lib.fd_last_error()
    ws, ld, st = Buf(ws_n), Buf(16 * n), Buf(4 * n)
    fsz = sum(K.shape[0] * phi.shape[0] for K, phi, _ in cfgs)
    F, Fi = Buf(8 * fsz), Buf(8 * fsz)
    tr = None
    if A is None:
        check(lib.fd_force_batched(P, n, C.byref(o), C.c_void_p(ld.p), C.c_void_p(F.p), C.c_void_p(Fi.p),
                                   C.c_void_p(ws.p), C.c_size_t(ws_n), C.c_void_p(st.p), None), "force")
    else:
        Aall = np.concatenate([np.stack([a.real, a.imag], -1).ravel() for a in A])
        bA = Buf(Aall.nbytes, Aall)
        tsz = sum(2 * phi.shape[0] for _, phi, _ in cfgs)
        bT = Buf(8 * tsz)
        check(lib.fd_force_response_batched(P, n, C.byref(o), C.c_void_p(bA.p), C.c_void_p(bT.p),
                                            C.c_void_p(ld.p), C.c_void_p(F.p), C.c_void_p(Fi.p),
                                            C.c_void_p(ws.p), C.c_size_t(ws_n), C.c_void_p(st.p), None),
              "force_response")
        tr = cplx(bT.get(np.float64, (tsz // 2, 2)))
    Fa, Fia = F.get(np.float64, (fsz,)), Fi.get(np.float64, (fsz,))
    outs, off = [], 0
    for K, phi, _ in cfgs:
        m = K.shape[0] * phi.shape[0]
        outs.append((Fa[off:off + m] + 1j * Fia[off:off + m]).reshape(phi.shape))
        off += m
    return outs, st.get(np.int32, (n,)).tolist(), tr


def honeycomb(L, Nt, beta, seed):
    w = Workload(L=L, Nt=Nt, beta=beta, U=3.0, seed=seed)
    return w.K(), w.phi(), w.dk


def ring_k(N, seed):
    """Symmetric hopping matrix of any size: a ring plus N/4 random chords
    (spectral radius about 3)."""
    rng = np.random.default_rng(seed)
    K = np.zeros((N, N))
    for i in range(N):
        K[i, (i + 1) % N] = K[(i + 1) % N, i] = 1.0
    for _ in range(N // 4):
        i, j = rng.integers(0, N, 2)
        if i != j:
            K[i, j] = K[j, i] = rng.uniform(0.5, 1.0)
    return K


def ring(N, Nt, beta, seed):
    return ring_k(N, seed), sample_phi(seed, Nt, N, beta / Nt, 3.0), beta / Nt


def batch_small(seed):
    """N = 8, 18 and 32: one class-32 launch per phase."""
    return [honeycomb(2, 8, 1.0, seed), honeycomb(3, 16, 2.0, seed + 1), honeycomb(4, 4, 0.5, seed + 2)]


def batch_512(seed):
    """N = 130 puts the launch in the blocked class; the N = 18 and 32 items
    then run the blocked code too."""
    return [ring(130, 4, 0.5, seed), honeycomb(3, 8, 1.0, seed + 1), honeycomb(4, 4, 0.5, seed + 2)]


def batch_mixed(seed):
    """N = 18, 50, 72, 98 and 128 in one class-128 launch: the items run the
    code of their own classes (32, 64, 80, 96, 128) on the class-128 layout
    of shared memory."""
    return [honeycomb(3, 8, 1.0, seed), honeycomb(5, 8, 1.0, seed + 1), honeycomb(6, 8, 1.0, seed + 2),
            honeycomb(7, 4, 0.5, seed + 3), honeycomb(8, 4, 0.5, seed + 4)]


def check_greens(cfgs, s):
    lds, Gs, st = run_greens(cfgs, s)
    worst = 0.0
    for (K, phi, dk), l, g in zip(cfgs, lds, Gs):
        lo, Go = O.stabilised_logdet_greens(K, dk, phi)
        worst = max(worst, dlog(l, lo), rel(g, Go))
    return worst, st


def check_force(cfgs, s, c, flags=0):
    Fs, st, _ = run_force(cfgs, s, c, flags)
    worst = 0.0
    for (K, phi, dk), f in zip(cfgs, Fs):
        worst = max(worst, rel(f, O.stabilised_force(K, dk, phi)))
    return worst, st


def case_response():
    K, phi, dk = honeycomb(3, 16, 2.0, 13)
    rng = np.random.default_rng(14)
    A = rng.normal(size=(18, 18)) + 1j * rng.normal(size=(18, 18))
    Fs, st, tr = run_force([(K, phi, dk)], 4, 4, A=[A])
    want = O.slice_response(K, dk, phi, A)
    worst = max(rel(tr, want), rel(Fs[0], O.stabilised_force(K, dk, phi)))
    return worst, st


def case_displaced(cfg):
    K, phi, dk = cfg
    N, Nt = K.shape[0], phi.shape[0]
    pairs = [(1, 1), (2, 4), (Nt, 1), (1, Nt), (Nt // 2 + 1, Nt // 3 + 1)]
    t = np.array([a for a, _ in pairs], np.int32)
    t0 = np.array([b for _, b in pairs], np.int32)
    P, keep = problems([cfg])
    o = Opts(4, 0, 0, 0)
    ws_n = lib.fd_displaced_workspace_bytes(P, C.byref(o), len(pairs))
    assert ws_n > 0, lib.fd_last_error()
    ws, G, st = Buf(ws_n), Buf(16 * N * N * len(pairs)), Buf(4)
    check(lib.fd_greens_displaced(P, C.byref(o), len(pairs), t.ctypes.data_as(C.c_void_p),
                                  t0.ctypes.data_as(C.c_void_p), C.c_void_p(G.p), C.c_void_p(ws.p),
                                  C.c_size_t(ws_n), C.c_void_p(st.p), None), "displaced")
    g = cplx(G.get(np.float64, (len(pairs), N, N, 2)))
    worst = max(rel(g[k], O.dsplit_displaced_greens(K, dk, phi, a, b)) for k, (a, b) in enumerate(pairs))
    return worst, st.get(np.int32, (1,)).tolist()


def case_sparse(cfg, n=4, s=4):
    K, phi, dk = cfg
    N = K.shape[0]
    q = int((K != 0).sum(1).max())
    col, val = np.zeros((N, q), np.int32), np.zeros((N, q))
    for i in range(N):
        nz = np.nonzero(K[i])[0]
        col[i, :len(nz)], val[i, :len(nz)] = nz, K[i, nz]
    bc, bv = Buf(col.nbytes, col), Buf(val.nbytes, val)
    P, keep = problems([cfg])
    hop = Ell(q, bc.p, bv.p)
    o = Opts(s, 0, 0, 0)
    ws_n = lib.fd_sparse_workspace_bytes(P, 1, C.byref(o), FD_WHAT_GREENS)
    assert ws_n > 0, lib.fd_last_error()
    ws, G, ld, st = Buf(ws_n), Buf(16 * N * N), Buf(16), Buf(4)
    check(lib.fd_sparse_greens(P, C.byref(hop), n, C.byref(o), C.c_void_p(ld.p), C.c_void_p(G.p),
                               C.c_void_p(ws.p), C.c_size_t(ws_n), C.c_void_p(st.p), None), "sparse")
    l = ld.get(np.float64, (2,))
    lo, Go = O.sparse_logdet_greens(K, dk, phi, n, s)
    worst = max(dlog(complex(l[0], l[1]), lo), rel(cplx(G.get(np.float64, (N, N, 2))), Go))
    return worst, st.get(np.int32, (1,)).tolist()


CASES = {
    # class 32 (register QR)
    "greens": lambda: check_greens([honeycomb(3, 16, 2.0, 11)], 4),
    "force_windows": lambda: check_force([honeycomb(3, 16, 2.0, 12)], 4, 4),
    "force_scans": lambda: check_force([honeycomb(3, 32, 4.0, 12)], 4, 4, FD_FORCE_SCANS),
    "response": case_response,
    "displaced": lambda: case_displaced(honeycomb(3, 12, 1.5, 31)),
    "sparse": lambda: case_sparse(honeycomb(3, 16, 2.0, 41)),
    "batch_greens": lambda: check_greens(batch_small(21), 4),
    "batch_force": lambda: check_force(batch_small(22), 4, 4),
    # class 512 (blocked QR, MFMA products from device memory)
    "b512_greens": lambda: check_greens(batch_512(51), 4),
    "b512_force": lambda: check_force(batch_512(52), 4, 2),
    "b512_force_scans": lambda: check_force(batch_512(53), 4, 2, FD_FORCE_SCANS),
    "b512_displaced": lambda: case_displaced(ring(130, 4, 0.5, 54)),
    "b512_sparse": lambda: case_sparse(ring(130, 4, 0.5, 55)),
    # every class (host builds with all classes only)
    "mixed_greens": lambda: check_greens(batch_mixed(61), 4),
    "mixed_force": lambda: check_force(batch_mixed(62), 4, 4),
    "class80_force": lambda: check_force([honeycomb(6, 32, 4.0, 63)], 8, 16),
}


def main():
    load(sys.argv[1])
    name = sys.argv[2]
    t = time.time()
    worst, status = CASES[name]()
    st = (C.c_uint64 * 6)()
    lib.emu_stats(st)
    out = {"case": name, "worst": worst, "status": status, "seconds": round(time.time() - t, 2),
           "launches": st[0], "groups": st[1], "barriers": st[2], "wave_ops": st[3], "mfma": st[4],
           "barrier_site_mismatch": st[5]}
    if hasattr(lib, "emu_race_stats"):
        rs = (C.c_uint64 * 3)()
        lib.emu_race_stats(rs)
        out["races"], out["checked_accesses"], out["lane_races"] = rs[0], rs[1], rs[2]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
