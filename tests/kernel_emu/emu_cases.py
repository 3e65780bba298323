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
wave), and per launch its workgroups, MFMA instructions (per wave) and barrier
arrivals (and, for the race build, the device bytes read and written).  A sanitizer finding or an emulation error aborts the process before
that line is printed.  For the AddressSanitizer build the caller preloads its
runtime.
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


FD_WHAT_LOGDET, FD_WHAT_UDV, FD_WHAT_HMC = 0, 3, 4
FD_REUSE_E, FD_KEEP_CHECKPOINTS = 0x1, 0x8


def bits_equal(a, b):
    return np.array_equal(np.atleast_1d(np.asarray(a)).view(np.uint8), np.atleast_1d(np.asarray(b)).view(np.uint8))


def case_plans():
    """Prepared force and G plans, each launched twice, against the eager
    calls bit for bit; a plan with FD_REUSE_E on the eager call's workspace."""
    cfgs = [honeycomb(3, 16, 2.0, 71), honeycomb(2, 8, 1.0, 72)]
    n = len(cfgs)
    P, keep = problems(cfgs)
    worst = 0.0
    fsz = sum(K.shape[0] * phi.shape[0] for K, phi, _ in cfgs)
    gsz = sum(2 * K.shape[0] ** 2 for K, _, _ in cfgs)
    for what in (FD_WHAT_GREENS, FD_WHAT_FORCE):
        o = Opts(4, 4, 0, 0)
        ws_n = lib.fd_workspace_bytes(P, n, C.byref(o), what)
        outs = []
        for mode in ("eager", "plan", "reuse"):
            ws, ld, st, G = Buf(ws_n), Buf(16 * n), Buf(4 * n), Buf(8 * gsz)
            F, Fi = Buf(8 * fsz), Buf(8 * fsz)
            args = (C.c_void_p(ld.p), C.c_void_p(G.p))
            fargs = (C.c_void_p(F.p), C.c_void_p(Fi.p))
            if mode in ("eager", "reuse"):
                if what == FD_WHAT_GREENS:
                    check(lib.fd_greens_batched(P, n, C.byref(o), *args, C.c_void_p(ws.p), C.c_size_t(ws_n),
                                                C.c_void_p(st.p), None), "greens")
                else:
                    check(lib.fd_force_batched(P, n, C.byref(o), C.c_void_p(ld.p), *fargs, C.c_void_p(ws.p),
                                               C.c_size_t(ws_n), C.c_void_p(st.p), None), "force")
            if mode in ("plan", "reuse"):
                o2 = Opts(4, 4, 0, FD_REUSE_E if mode == "reuse" else 0)
                plan = C.c_void_p()
                check(lib.fd_plan_create(what, P, n, C.byref(o2), *args, *(fargs if what == FD_WHAT_FORCE else
                                                                            (None, None)),
                                         C.c_void_p(ws.p), C.c_size_t(ws_n), C.c_void_p(st.p), None,
                                         C.byref(plan)), "plan_create")
                for _ in range(2):
                    check(lib.fd_plan_launch(plan, None), "plan_launch")
                lib.fd_plan_destroy(plan)
            res = [ld.get(np.float64, (n, 2))]
            res.append(G.get(np.float64, (gsz,)) if what == FD_WHAT_GREENS else F.get(np.float64, (fsz,)))
            assert st.get(np.int32, (n,)).tolist() == [0] * n
            outs.append(res)
        for o_ in outs[1:]:
            for a, b in zip(outs[0], o_):
                if not bits_equal(a, b):
                    worst = max(worst, 1.0)
    # the eager results against the oracle
    w2, st = check_force(cfgs, 4, 4)
    return max(worst, w2), st


def case_keep_checkpoints():
    """G with FD_KEEP_CHECKPOINTS, then the force from its checkpoints, against
    the full force (and the oracle)."""
    cfg = honeycomb(3, 16, 2.0, 73)
    K, phi, dk = cfg
    P, keep = problems([cfg])
    o = Opts(4, 4, 0, FD_KEEP_CHECKPOINTS)
    ws_n = lib.fd_workspace_bytes(P, 1, C.byref(o), FD_WHAT_FORCE)
    ws, ld, st, G = Buf(ws_n), Buf(16), Buf(4), Buf(16 * 18 * 18)
    F, Fi = Buf(8 * 16 * 18), Buf(8 * 16 * 18)
    check(lib.fd_greens(P, C.byref(o), C.c_void_p(ld.p), C.c_void_p(G.p), C.c_void_p(ws.p), C.c_size_t(ws_n),
                        C.c_void_p(st.p), None), "greens keep")
    check(lib.fd_force(P, C.byref(o), None, C.c_void_p(F.p), C.c_void_p(Fi.p), C.c_void_p(ws.p),
                       C.c_size_t(ws_n), C.c_void_p(st.p), None), "force keep")
    f = (F.get(np.float64, (16, 18)) + 1j * Fi.get(np.float64, (16, 18)))
    full, _, _ = run_force([cfg], 4, 4)
    lo, Go = O.stabilised_logdet_greens(K, dk, phi)
    l = ld.get(np.float64, (2,))
    worst = max(rel(f, full[0]), rel(f, O.stabilised_force(K, dk, phi)), dlog(complex(l[0], l[1]), lo),
                rel(cplx(G.get(np.float64, (18, 18, 2))), Go))
    return worst, st.get(np.int32, (1,)).tolist()


def case_udv_exp():
    """fd_udv: X unitary, X diag(D) T = B_{N_t} ... B_1; fd_slice_exponential
    against exp(dk K)."""
    cfg = honeycomb(3, 8, 0.5, 74)
    K, phi, dk = cfg
    N = 18
    P, keep = problems([cfg])
    o = Opts(4, 0, 0, 0)
    ws_n = lib.fd_workspace_bytes(P, 1, C.byref(o), FD_WHAT_UDV)
    ws, st = Buf(ws_n), Buf(4)
    X, D, T = Buf(16 * N * N), Buf(8 * N), Buf(16 * N * N)
    check(lib.fd_udv(P, C.byref(o), C.c_void_p(X.p), C.c_void_p(D.p), C.c_void_p(T.p), C.c_void_p(ws.p),
                     C.c_size_t(ws_n), C.c_void_p(st.p), None), "udv")
    x, d, t = cplx(X.get(np.float64, (N, N, 2))), D.get(np.float64, (N,)), cplx(T.get(np.float64, (N, N, 2)))
    prod = np.eye(N, dtype=complex)
    for B in O.slice_matrices(K, dk, phi):
        prod = B @ prod
    worst = max(rel((x * d) @ t, prod), float(np.abs(x.conj().T @ x - np.eye(N)).max()))
    ws_e = lib.fd_workspace_bytes(P, 1, C.byref(o), FD_WHAT_LOGDET)
    wse, E = Buf(ws_e), Buf(8 * N * N)
    check(lib.fd_slice_exponential(P, C.c_void_p(E.p), C.c_void_p(wse.p), C.c_size_t(ws_e), None), "exp")
    worst = max(worst, rel(E.get(np.float64, (N, N)), O.slice_exponential(K, dk)))
    return worst, st.get(np.int32, (1,)).tolist()


def case_observables():
    """fd_response_trace (A and the fermion number) and fd_diag_response
    against the oracle, on the library's own G and force."""
    cfg = honeycomb(3, 16, 2.0, 75)
    K, phi, dk = cfg
    N, Nt = 18, 16
    lds, Gs, st = run_greens([cfg], 4)
    Fs, st2, _ = run_force([cfg], 4, 4)
    rng = np.random.default_rng(76)
    A = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    a = rng.normal(size=N)
    g_il = np.stack([Gs[0].real, Gs[0].imag], -1)
    bG = Buf(g_il.nbytes, g_il)
    a_il = np.stack([A.real, A.imag], -1)
    bA = Buf(a_il.nbytes, a_il)
    lib.fd_response_trace_workspace_bytes.restype = C.c_size_t
    wn = lib.fd_response_trace_workspace_bytes(N)
    ws, out = Buf(wn), Buf(16)
    worst = 0.0
    for Aop, ref in ((bA, O.response_trace(Gs[0], A)), (None, O.response_trace(Gs[0]))):
        check(lib.fd_response_trace(N, C.c_void_p(bG.p), C.c_void_p(Aop.p if Aop else None), C.c_void_p(out.p),
                                    C.c_void_p(ws.p), C.c_size_t(wn), None), "trace")
        r = out.get(np.float64, (2,))
        worst = max(worst, abs(complex(r[0], r[1]) - ref) / max(1.0, abs(ref)))
    f = Fs[0]
    bF, bFi, ba = Buf(8 * N * Nt, np.ascontiguousarray(f.real)), Buf(8 * N * Nt, np.ascontiguousarray(f.imag)), Buf(8 * N, a)
    check(lib.fd_diag_response(Nt, N, C.c_void_p(bF.p), C.c_void_p(bFi.p), C.c_void_p(ba.p), C.c_void_p(out.p),
                               None), "diag")
    r = out.get(np.float64, (2,))
    ref = O.diag_response(f, a)
    worst = max(worst, abs(complex(r[0], r[1]) - ref) / max(1.0, abs(ref)))
    return worst, st + st2


def case_leapfrog():
    """fd_hmc_leapfrog against the oracle's leapfrog, and the prepared
    trajectory (fd_hmc_plan_*) against fd_hmc_leapfrog bit for bit."""
    K, phi0, dk = honeycomb(2, 8, 1.0, 77)
    N, Nt = 8, 8
    dU, eps, nsteps = dk * 3.0, 0.05, 2
    pi0 = np.random.default_rng(78).normal(size=(Nt, N))
    ph_o, pi_o, dH_o = O.hmc_leapfrog(K, dk, phi0, pi0, dU, eps, nsteps)
    res = []
    for mode in ("call", "plan"):
        bK, bphi, bpi = Buf(K.nbytes, K), Buf(phi0.nbytes, phi0), Buf(pi0.nbytes, pi0)
        P = (Prob * 1)(Prob(N, Nt, dk, bK.p, bphi.p))
        o = Opts(4, 4, 0, 0)
        ws_n = lib.fd_workspace_bytes(P, 1, C.byref(o), FD_WHAT_HMC)
        ws, dH, st = Buf(ws_n), Buf(8), Buf(4)
        if mode == "call":
            check(lib.fd_hmc_leapfrog(P, 1, C.byref(o), C.c_double(dU), C.c_double(eps), nsteps, C.c_void_p(bpi.p),
                                      C.c_void_p(dH.p), C.c_void_p(ws.p), C.c_size_t(ws_n), C.c_void_p(st.p), None),
                  "leapfrog")
        else:
            plan = C.c_void_p()
            check(lib.fd_hmc_plan_create(P, 1, C.byref(o), C.c_double(dU), C.c_double(eps), nsteps,
                                         C.c_void_p(bpi.p), C.c_void_p(dH.p), C.c_void_p(ws.p), C.c_size_t(ws_n),
                                         C.c_void_p(st.p), None, C.byref(plan)), "hmc plan")
            check(lib.fd_hmc_plan_launch(plan, None), "hmc plan launch")
            lib.fd_hmc_plan_destroy(plan)
        res.append((bphi.get(np.float64, (Nt, N)), bpi.get(np.float64, (Nt, N)), dH.get(np.float64, (1,))[0],
                    st.get(np.int32, (1,)).tolist()))
    worst = max(rel(res[0][0], ph_o), rel(res[0][1], pi_o), abs(res[0][2] - dH_o) / max(1.0, abs(dH_o)))
    if not (bits_equal(res[0][0], res[1][0]) and bits_equal(res[0][1], res[1][1])
            and bits_equal(np.float64(res[0][2]), np.float64(res[1][2]))):
        worst = max(worst, 1.0)
    return worst, res[0][3] + res[1][3]


def case_noalloc():
    """fd_greens_noalloc against fd_greens bit for bit, two calls in a row,
    the second smaller."""
    worst, sts = 0.0, []
    for cfg in (honeycomb(3, 16, 2.0, 79), honeycomb(2, 8, 1.0, 80)):
        N = cfg[0].shape[0]
        P, keep = problems([cfg])
        o = Opts(4, 0, 0, 0)
        ld, G, st = Buf(16), Buf(16 * N * N), Buf(4)
        check(lib.fd_greens_noalloc(P, C.byref(o), C.c_void_p(ld.p), C.c_void_p(G.p), C.c_void_p(st.p), None),
              "noalloc")
        lds, Gs, st2 = run_greens([cfg], 4)
        g = cplx(G.get(np.float64, (N, N, 2)))
        l = ld.get(np.float64, (2,))
        if not (bits_equal(g, Gs[0]) and bits_equal(l, np.array([lds[0].real, lds[0].imag]))):
            worst = 1.0
        sts += st.get(np.int32, (1,)).tolist() + st2
    return worst, sts


def case_full_lowT():
    """lowT_L6 at full size (N = 72, N_t = 256, beta = 32, s = 8) with 32
    segments, det + G."""
    from workload import WORKLOADS
    w = WORKLOADS["lowT_L6"]
    return check_greens_seg([(w.K(), w.phi(), w.dk)], w.s, 32)


def case_full_force_L8():
    """force_L8 at full size (N = 128, N_t = 256, beta = 32, s = 8, c = 16)."""
    from workload import WORKLOADS
    w = WORKLOADS["force_L8"]
    return check_force([(w.K(), w.phi(), w.dk)], w.s, w.c)


def case_n512_force():
    """The HMC step's shape per field (L = 16, N = 512, delta kappa = 0.125,
    s = c = 16) on the first 32 slices of field 0: two checkpoint intervals."""
    from workload import hmc_batch
    w = hmc_batch(1)[0]
    phi = np.ascontiguousarray(w.phi()[:32])
    return check_force([(w.K(), phi, w.dk)], w.s, w.c)


def check_greens_seg(cfgs, s, segments):
    lds, Gs, st = run_greens(cfgs, s, segments)
    worst = 0.0
    for (K, phi, dk), l, g in zip(cfgs, lds, Gs):
        lo, Go = O.stabilised_logdet_greens(K, dk, phi)
        worst = max(worst, dlog(l, lo), rel(g, Go))
    return worst, st


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
    # further entry points (class 32)
    "plans": case_plans,
    "keep_checkpoints": case_keep_checkpoints,
    "udv_exp": case_udv_exp,
    "observables": case_observables,
    "leapfrog": case_leapfrog,
    "noalloc": case_noalloc,
    # every class (host builds with all classes only)
    "mixed_greens": lambda: check_greens(batch_mixed(61), 4),
    "mixed_force": lambda: check_force(batch_mixed(62), 4, 4),
    "class80_force": lambda: check_force([honeycomb(6, 32, 4.0, 63)], 8, 16),
    # named workloads at full size, and the HMC step's N = 512 shape (long)
    "full_lowT_L6": case_full_lowT,
    "full_force_L8": case_full_force_L8,
    "full_n512_force": case_n512_force,
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
    log = (C.c_uint64 * (3 * 4096))()
    nl = lib.emu_launch_log(log, 4096)
    out["launch_log"] = [[log[3 * i], log[3 * i + 1], log[3 * i + 2]] for i in range(min(nl, 4096))]
    if hasattr(lib, "emu_race_launch_bytes"):
        b = (C.c_uint64 * (2 * 4096))()
        nb = lib.emu_race_launch_bytes(b, 4096)
        out["launch_bytes"] = [[b[2 * i], b[2 * i + 1]] for i in range(min(nb, 4096))]
    if hasattr(lib, "emu_race_stats"):
        rs = (C.c_uint64 * 3)()
        lib.emu_race_stats(rs)
        out["races"], out["checked_accesses"], out["lane_races"] = rs[0], rs[1], rs[2]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
