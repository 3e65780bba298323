"""Python binding of libfdet: the stabilised fermion determinant on gfx950.

Argument marshalling only.  Every step of the computation runs in the HIP
kernels of libfdet.so; PyTorch supplies device memory and the stream.  There
is no CPU fallback: without the built library or a GPU the calls raise.

    import paper_2604_02130_amd as fd
    ld, G = fd.greens(K, phi, dk, s=8)        # K, phi: float64 CUDA tensors
    F = fd.force(K, phi, dk, s=8, checkpoint=16).real
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdet.so")

FD_OK = 0
FD_WARN_ILLCOND = 1
FD_ERR_INVALID_ARG = -1
FD_ERR_WORKSPACE = -2
FD_ERR_SINGULAR = -3
FD_ERR_NONFINITE = -4
FD_ERR_HIP = -5
FD_ERR_UNSUPPORTED = -6

FD_WHAT_LOGDET, FD_WHAT_GREENS, FD_WHAT_FORCE, FD_WHAT_UDV, FD_WHAT_HMC = 0, 1, 2, 3, 4
FD_REUSE_E = 0x1
FD_FORCE_SCANS = 0x2
FD_SINGLE_LAUNCH = 0x4   # switched off in the library (returns FD_ERR_UNSUPPORTED)
FD_KEEP_CHECKPOINTS = 0x8
MAX_N = 512

# exported names (each declared in include/fdet.h)
SYMBOLS = (
    "fd_workspace_bytes", "fd_slice_exponential", "fd_logdet", "fd_greens", "fd_force",
    "fd_udv", "fd_logdet_batched", "fd_greens_batched", "fd_force_batched",
    "fd_strerror", "fd_last_error", "fd_version", "fd_profile_start", "fd_profile_stop",
    "fd_plan_create", "fd_plan_launch", "fd_plan_destroy", "fd_autotune", "fd_tune_save",
    "fd_tune_load", "fd_tune_clear", "fd_response_trace_workspace_bytes", "fd_response_trace",
    "fd_hmc_leapfrog", "fd_diag_response", "fd_hmc_plan_create", "fd_hmc_plan_launch",
    "fd_hmc_plan_destroy", "fd_plan_segments", "fd_greens_noalloc",
    "fd_displaced_workspace_bytes", "fd_greens_displaced", "fd_force_response",
    "fd_force_response_batched", "fd_sparse_workspace_bytes", "fd_sparse_greens",
    "fd_sparse_greens_batched",
)

PHASE_NAMES = {0: "expm", 1: "chain", 2: "combine", 3: "close", 4: "force", 5: "export",
               -1: "single"}


class FdProblem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("Nt", ctypes.c_int32), ("dk", ctypes.c_double),
                ("K", ctypes.c_void_p), ("phi", ctypes.c_void_p)]


class FdEll(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class FdOptions(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int32), ("checkpoint", ctypes.c_int32),
                ("segments", ctypes.c_int32), ("flags", ctypes.c_int32)]


class FdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfdet error {code}: {msg}")
        self.code = code


_lib = None


def _check_sources(ver: str, path: str):
    """The library carries a digest of the sources it was built from; refuse
    one built from other sources than those next to this file."""
    from . import build as _build
    if not os.path.isdir(_build.CSRC):
        return
    want = _build.source_digest()
    got = ver.rsplit(" ", 1)[-1] if " src " in ver else "none"
    if got != want:
        raise FdError(FD_ERR_UNSUPPORTED,
                      f"{path} was built from other sources (src {got}, this tree {want}); "
                      "rebuild with `python -m paper_2604_02130_amd.build`")


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfdet.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FdError(FD_ERR_UNSUPPORTED,
                      f"{path} is not built; run `python -m paper_2604_02130_amd.build`")
    from . import build as _build
    if os.path.isdir(_build.CSRC):
        _check_sources(f"libfdet src {_build.library_digest(path)}", path)
    lib = ctypes.CDLL(path)
    lib.fd_version.argtypes = []
    lib.fd_version.restype = ctypes.c_char_p
    _check_sources(lib.fd_version().decode(), path)
    P = ctypes.POINTER(FdProblem)
    O = ctypes.POINTER(FdOptions)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.fd_workspace_bytes.argtypes = [P, i32, O, i32]
    lib.fd_workspace_bytes.restype = sz
    lib.fd_slice_exponential.argtypes = [P, vp, vp, sz, vp]
    lib.fd_logdet.argtypes = [P, O, vp, vp, sz, vp, vp]
    lib.fd_greens.argtypes = [P, O, vp, vp, vp, sz, vp, vp]
    lib.fd_force.argtypes = [P, O, vp, vp, vp, vp, sz, vp, vp]
    lib.fd_udv.argtypes = [P, O, vp, vp, vp, vp, sz, vp, vp]
    lib.fd_logdet_batched.argtypes = [P, i32, O, vp, vp, sz, vp, vp]
    lib.fd_greens_batched.argtypes = [P, i32, O, vp, vp, vp, sz, vp, vp]
    lib.fd_force_batched.argtypes = [P, i32, O, vp, vp, vp, vp, sz, vp, vp]
    lib.fd_force_response.argtypes = [P, O, vp, vp, vp, vp, vp, vp, sz, vp, vp]
    EL = ctypes.POINTER(FdEll)
    lib.fd_sparse_workspace_bytes.argtypes = [P, i32, O, i32]
    lib.fd_sparse_workspace_bytes.restype = sz
    lib.fd_sparse_greens.argtypes = [P, EL, i32, O, vp, vp, vp, sz, vp, vp]
    lib.fd_sparse_greens.restype = ctypes.c_int
    lib.fd_sparse_greens_batched.argtypes = [P, i32, EL, i32, O, vp, vp, vp, sz, vp, vp]
    lib.fd_sparse_greens_batched.restype = ctypes.c_int
    lib.fd_force_response_batched.argtypes = [P, i32, O, vp, vp, vp, vp, vp, vp, sz, vp, vp]
    for name in ("fd_slice_exponential", "fd_logdet", "fd_greens", "fd_force", "fd_udv",
                 "fd_logdet_batched", "fd_greens_batched", "fd_force_batched",
                 "fd_force_response", "fd_force_response_batched"):
        getattr(lib, name).restype = ctypes.c_int
    lib.fd_strerror.argtypes = [ctypes.c_int]
    lib.fd_strerror.restype = ctypes.c_char_p
    lib.fd_last_error.argtypes = []
    lib.fd_last_error.restype = ctypes.c_char_p
    lib.fd_version.argtypes = []
    lib.fd_version.restype = ctypes.c_char_p
    lib.fd_profile_start.argtypes = []
    lib.fd_profile_start.restype = ctypes.c_int
    lib.fd_profile_stop.argtypes = [i32, vp, vp, vp]
    lib.fd_profile_stop.restype = ctypes.c_int
    lib.fd_plan_create.argtypes = [i32, P, i32, O, vp, vp, vp, vp, vp, sz, vp, vp,
                                   ctypes.POINTER(vp)]
    lib.fd_plan_create.restype = ctypes.c_int
    lib.fd_plan_launch.argtypes = [vp, vp]
    lib.fd_plan_launch.restype = ctypes.c_int
    lib.fd_plan_destroy.argtypes = [vp]
    lib.fd_plan_destroy.restype = None
    lib.fd_plan_segments.argtypes = [vp, vp, i32]
    lib.fd_plan_segments.restype = ctypes.c_int
    lib.fd_greens_noalloc.argtypes = [P, O, vp, vp, vp, vp]
    lib.fd_greens_noalloc.restype = ctypes.c_int
    lib.fd_displaced_workspace_bytes.argtypes = [P, O, i32]
    lib.fd_displaced_workspace_bytes.restype = sz
    lib.fd_greens_displaced.argtypes = [P, O, i32, vp, vp, vp, vp, sz, vp, vp]
    lib.fd_greens_displaced.restype = ctypes.c_int
    lib.fd_autotune.argtypes = [i32, P, i32, O, vp, O, ctypes.POINTER(ctypes.c_float)]
    lib.fd_autotune.restype = ctypes.c_int
    lib.fd_tune_save.argtypes = [ctypes.c_char_p]
    lib.fd_tune_save.restype = ctypes.c_int
    lib.fd_tune_load.argtypes = [ctypes.c_char_p]
    lib.fd_tune_load.restype = ctypes.c_int
    lib.fd_tune_clear.argtypes = []
    lib.fd_tune_clear.restype = ctypes.c_int
    lib.fd_hmc_leapfrog.argtypes = [P, i32, O, ctypes.c_double, ctypes.c_double, i32, vp, vp, vp,
                                    sz, vp, vp]
    lib.fd_hmc_leapfrog.restype = ctypes.c_int
    lib.fd_hmc_plan_create.argtypes = [P, i32, O, ctypes.c_double, ctypes.c_double, i32, vp, vp,
                                       vp, sz, vp, vp, ctypes.POINTER(vp)]
    lib.fd_hmc_plan_create.restype = ctypes.c_int
    lib.fd_hmc_plan_launch.argtypes = [vp, vp]
    lib.fd_hmc_plan_launch.restype = ctypes.c_int
    lib.fd_hmc_plan_destroy.argtypes = [vp]
    lib.fd_hmc_plan_destroy.restype = None
    lib.fd_diag_response.argtypes = [i32, i32, vp, vp, vp, vp, vp]
    lib.fd_diag_response.restype = ctypes.c_int
    lib.fd_response_trace_workspace_bytes.argtypes = [i32]
    lib.fd_response_trace_workspace_bytes.restype = sz
    lib.fd_response_trace.argtypes = [i32, vp, vp, vp, vp, sz, vp]
    lib.fd_response_trace.restype = ctypes.c_int
    _lib = lib
    return lib


def profile_start():
    """Start timing every kernel phase of this thread's calls with HIP events."""
    _check(load_library().fd_profile_start())


def profile_stop(max_records: int = 65536):
    """Stop timing; returns a list of (phase name, work items, milliseconds)."""
    lib = load_library()
    kinds = (ctypes.c_int32 * max_records)()
    nitems = (ctypes.c_int32 * max_records)()
    ms = (ctypes.c_float * max_records)()
    n = lib.fd_profile_stop(max_records, kinds, nitems, ms)
    n = min(n, max_records)
    return [(PHASE_NAMES.get(kinds[i], str(kinds[i])), nitems[i], float(ms[i])) for i in range(n)]


def version() -> str:
    return load_library().fd_version().decode()


def strerror(code: int) -> str:
    return load_library().fd_strerror(int(code)).decode()


def _check(rc: int):
    if rc != FD_OK:
        lib = load_library()
        raise FdError(rc, f"{lib.fd_strerror(rc).decode()}: {lib.fd_last_error().decode()}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise FdError(FD_ERR_UNSUPPORTED, "libfdet needs a ROCm GPU; none is visible")
    return torch


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else 0


def _prob(K, phi, dk) -> FdProblem:
    torch = _torch()
    for name, t in (("K", K), ("phi", phi)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise FdError(FD_ERR_INVALID_ARG, f"{name} must be a CUDA tensor")
        if t.dtype != torch.float64 or not t.is_contiguous():
            raise FdError(FD_ERR_INVALID_ARG, f"{name} must be contiguous float64")
    if K.dim() != 2 or K.shape[0] != K.shape[1]:
        raise FdError(FD_ERR_INVALID_ARG, "K must be square")
    if phi.dim() != 2 or phi.shape[1] != K.shape[0]:
        raise FdError(FD_ERR_INVALID_ARG, "phi must have shape (Nt, N)")
    return FdProblem(int(K.shape[0]), int(phi.shape[0]), float(dk), K.data_ptr(), phi.data_ptr())


def _opts(s=0, checkpoint=0, segments=0, flags=0) -> FdOptions:
    return FdOptions(int(s), int(checkpoint), int(segments), int(flags))


class Workspace:
    """A growable device byte buffer reused across calls on one device."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device):
        torch = _torch()
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        off = (-base) % 256
        return base + off, self.buf.numel() - off


_default_ws = Workspace()


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _status_check(status, check: bool):
    if not check:
        return
    vals = status.cpu().tolist()
    for i, v in enumerate(vals):
        if v < 0:
            raise FdError(v, f"problem {i}: {strerror(v)}")


def workspace_bytes(probs: Sequence[FdProblem], what: int, **opts) -> int:
    lib = load_library()
    arr = (FdProblem * len(probs))(*probs)
    o = _opts(**opts)
    n = lib.fd_workspace_bytes(arr, len(probs), ctypes.byref(o), what)
    if n == 0:
        raise FdError(FD_ERR_INVALID_ARG, lib.fd_last_error().decode())
    return int(n)


def slice_exponential(K, dk, ws: Workspace | None = None):
    """E = exp(dk K) computed on the GPU (N x N float64)."""
    torch = _torch()
    lib = load_library()
    phi = torch.zeros((1, K.shape[0]), dtype=torch.float64, device=K.device)
    p = _prob(K, phi, dk)
    E = torch.empty_like(K)
    need = workspace_bytes([p], FD_WHAT_LOGDET)
    wsp, wsn = (ws or _default_ws).get(need, K.device)
    _check(lib.fd_slice_exponential(ctypes.byref(p), E.data_ptr(), wsp, wsn, _stream()))
    return E


def logdet(K, phi, dk, s=0, segments=0, flags=0, check=True, ws: Workspace | None = None,
           checkpoint=0):
    """log det(1 + B_{N_t}...B_1) as a complex128 scalar tensor on the device.
    checkpoint: the checkpoint interval when flags has FD_KEEP_CHECKPOINTS."""
    torch = _torch()
    lib = load_library()
    p = _prob(K, phi, dk)
    o = _opts(s=s, checkpoint=checkpoint, segments=segments, flags=flags)
    out = torch.empty(2, dtype=torch.float64, device=K.device)
    status = torch.empty(1, dtype=torch.int32, device=K.device)
    need = workspace_bytes([p], FD_WHAT_LOGDET, s=s, checkpoint=checkpoint, segments=segments,
                           flags=flags)
    wsp, wsn = (ws or _default_ws).get(need, K.device)
    _check(lib.fd_logdet(ctypes.byref(p), ctypes.byref(o), out.data_ptr(), wsp, wsn,
                         status.data_ptr(), _stream()))
    _status_check(status, check)
    return torch.view_as_complex(out)


def greens(K, phi, dk, s=0, segments=0, flags=0, check=True, ws: Workspace | None = None,
           out=None, status=None, checkpoint=0):
    """(log det M, G = M^{-1}); G is an N x N complex128 tensor.
    checkpoint: the checkpoint interval when flags has FD_KEEP_CHECKPOINTS."""
    torch = _torch()
    lib = load_library()
    p = _prob(K, phi, dk)
    N = p.N
    o = _opts(s=s, checkpoint=checkpoint, segments=segments, flags=flags)
    ld = torch.empty(2, dtype=torch.float64, device=K.device) if out is None else out[0]
    G = torch.empty((N, N, 2), dtype=torch.float64, device=K.device) if out is None else out[1]
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=K.device)
    need = workspace_bytes([p], FD_WHAT_GREENS, s=s, checkpoint=checkpoint, segments=segments,
                           flags=flags)
    wsp, wsn = (ws or _default_ws).get(need, K.device)
    _check(lib.fd_greens(ctypes.byref(p), ctypes.byref(o), ld.data_ptr(), G.data_ptr(), wsp, wsn,
                         status.data_ptr(), _stream()))
    _status_check(status, check)
    return torch.view_as_complex(ld), torch.view_as_complex(G)


def ell(K, device=None):
    """(col, val): the nonzeros of a hopping matrix in the ELL layout of
    fd_ell (q = the most nonzeros of any row; short rows padded with their
    own index and weight 0), as int32 / float64 tensors of shape (N, q) on
    `device` (default: K's).  Layout conversion only."""
    torch = _torch()
    Kh = K.detach().to("cpu", torch.float64)
    N = Kh.shape[0]
    nz = [torch.nonzero(Kh[i]).flatten().tolist() for i in range(N)]
    q = max(1, max(len(r) for r in nz))
    col = torch.empty((N, q), dtype=torch.int32)
    val = torch.zeros((N, q), dtype=torch.float64)
    for i, r in enumerate(nz):
        col[i] = i
        for j, c in enumerate(r):
            col[i, j] = c
            val[i, j] = Kh[i, c]
    dev = device if device is not None else K.device
    return col.to(dev), val.to(dev)


def sparse_greens(col, val, phi, dk, n=4, s=0, segments=0, want_g=True, check=True,
                  ws: Workspace | None = None):
    """fd_sparse_greens: log det and (if want_g) G of the sausage whose slices
    are [prod_k (1 + gamma_k dk K)] diag(e^{i phi_t}) (degree-n product-form
    Taylor polynomial, applied matrix-free from the ELL arrays col / val of
    shape (N, q)), QR every s slices.  Returns (logdet, G or None)."""
    torch = _torch()
    lib = load_library()
    for name, t, dt in (("col", col, torch.int32), ("val", val, torch.float64),
                        ("phi", phi, torch.float64)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise FdError(FD_ERR_INVALID_ARG, f"{name} must be a contiguous CUDA {dt} tensor")
    if col.dim() != 2 or tuple(col.shape) != tuple(val.shape) or phi.dim() != 2 \
            or phi.shape[1] != col.shape[0]:
        raise FdError(FD_ERR_INVALID_ARG, "col, val must be (N, q) and phi (Nt, N)")
    N, q = int(col.shape[0]), int(col.shape[1])
    p = FdProblem(N, int(phi.shape[0]), float(dk), None, phi.data_ptr())
    h = FdEll(q, col.data_ptr(), val.data_ptr())
    o = _opts(s=s, segments=segments)
    what = FD_WHAT_GREENS if want_g else FD_WHAT_LOGDET
    ld = torch.empty(2, dtype=torch.float64, device=phi.device)
    G = torch.empty((N, N, 2), dtype=torch.float64, device=phi.device) if want_g else None
    status = torch.empty(1, dtype=torch.int32, device=phi.device)
    need = lib.fd_sparse_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), what)
    if need == 0:
        raise FdError(FD_ERR_INVALID_ARG, "fd_sparse_workspace_bytes: " + lib.fd_last_error().decode())
    wsp, wsn = (ws or _default_ws).get(need, phi.device)
    _check(lib.fd_sparse_greens(ctypes.byref(p), ctypes.byref(h), int(n), ctypes.byref(o),
                                ld.data_ptr(), G.data_ptr() if want_g else None, wsp, wsn,
                                status.data_ptr(), _stream()))
    _status_check(status, check)
    return torch.view_as_complex(ld), (torch.view_as_complex(G) if want_g else None)


def greens_noalloc(K, phi, dk, logdet, G, status, s=0, segments=0, flags=0):
    """fd_greens_noalloc: log det and G into caller tensors (logdet: 2 float64,
    G: N*N*2 float64, status: 1 int32, all on the device) with the library's
    fixed workspace; nothing is allocated.  The caller reads status after
    synchronising."""
    lib = load_library()
    p = _prob(K, phi, dk)
    o = _opts(s=s, segments=segments, flags=flags)
    _check(lib.fd_greens_noalloc(ctypes.byref(p), ctypes.byref(o), logdet.data_ptr(),
                                 G.data_ptr(), status.data_ptr(), _stream()))


def greens_displaced(K, phi, dk, pairs, s=0, flags=0, check=True, ws: Workspace | None = None):
    """Time-displaced Green's functions G(t, t0) (block (t, t0) of the inverse
    block fermion matrix, 1-based slices, G(1, 1) = G) for the (t, t0) in
    `pairs`; returns an (npairs, N, N) complex128 tensor."""
    torch = _torch()
    lib = load_library()
    p = _prob(K, phi, dk)
    o = _opts(s=s, flags=flags)
    n = len(pairs)
    th = (ctypes.c_int32 * n)(*[int(a) for a, _ in pairs])
    t0h = (ctypes.c_int32 * n)(*[int(b) for _, b in pairs])
    G = torch.empty((n, p.N, p.N, 2), dtype=torch.float64, device=K.device)
    status = torch.empty(1, dtype=torch.int32, device=K.device)
    need = lib.fd_displaced_workspace_bytes(ctypes.byref(p), ctypes.byref(o), n)
    if need == 0:
        raise FdError(FD_ERR_INVALID_ARG, lib.fd_last_error().decode())
    wsp, wsn = (ws or _default_ws).get(need, K.device)
    _check(lib.fd_greens_displaced(ctypes.byref(p), ctypes.byref(o), n, th, t0h, G.data_ptr(),
                                   wsp, wsn, status.data_ptr(), _stream()))
    _status_check(status, check)
    return torch.view_as_complex(G)


def force(K, phi, dk, s=0, checkpoint=0, flags=0, check=True, ws: Workspace | None = None,
          with_logdet=False):
    """Complex force F[t-1, x] = d log det M / d phi_{t,x} as an (N_t, N) tensor."""
    torch = _torch()
    lib = load_library()
    p = _prob(K, phi, dk)
    o = _opts(s=s, checkpoint=checkpoint, flags=flags)
    Fr = torch.empty((p.Nt, p.N), dtype=torch.float64, device=K.device)
    Fi = torch.empty((p.Nt, p.N), dtype=torch.float64, device=K.device)
    ld = torch.empty(2, dtype=torch.float64, device=K.device)
    status = torch.empty(1, dtype=torch.int32, device=K.device)
    need = workspace_bytes([p], FD_WHAT_FORCE, s=s, checkpoint=checkpoint, flags=flags)
    wsp, wsn = (ws or _default_ws).get(need, K.device)
    _check(lib.fd_force(ctypes.byref(p), ctypes.byref(o), ld.data_ptr(), Fr.data_ptr(),
                        Fi.data_ptr(), wsp, wsn, status.data_ptr(), _stream()))
    _status_check(status, check)
    F = torch.complex(Fr, Fi)
    return (F, torch.view_as_complex(ld)) if with_logdet else F


def force_response(K, phi, dk, A, s=0, checkpoint=0, flags=0, check=True,
                   ws: Workspace | None = None):
    """(F, traces): the complex force as force() returns it and the per-slice
    responses traces[t-1] = tr((1 - G~_t) A) to the (N, N) complex operator A
    (fd_force_response); traces.mean() is the slice-averaged response."""
    torch = _torch()
    lib = load_library()
    p = _prob(K, phi, dk)
    o = _opts(s=s, checkpoint=checkpoint, flags=flags)
    Ac = torch.view_as_real(A.to(device=K.device, dtype=torch.complex128).contiguous()).contiguous()
    if tuple(Ac.shape) != (p.N, p.N, 2):
        raise ValueError(f"A must be ({p.N}, {p.N}), got {tuple(A.shape)}")
    Fr = torch.empty((p.Nt, p.N), dtype=torch.float64, device=K.device)
    Fi = torch.empty((p.Nt, p.N), dtype=torch.float64, device=K.device)
    tr = torch.empty((p.Nt, 2), dtype=torch.float64, device=K.device)
    status = torch.empty(1, dtype=torch.int32, device=K.device)
    need = workspace_bytes([p], FD_WHAT_FORCE, s=s, checkpoint=checkpoint, flags=flags)
    wsp, wsn = (ws or _default_ws).get(need, K.device)
    _check(lib.fd_force_response(ctypes.byref(p), ctypes.byref(o), Ac.data_ptr(), tr.data_ptr(),
                                 None, Fr.data_ptr(), Fi.data_ptr(), wsp, wsn, status.data_ptr(),
                                 _stream()))
    _status_check(status, check)
    return torch.complex(Fr, Fi), torch.view_as_complex(tr)


def udv(K, phi, dk, s=0, segments=0, check=True, ws: Workspace | None = None):
    """(X, D, T) with B_{N_t}...B_1 = X diag(D) T."""
    torch = _torch()
    lib = load_library()
    p = _prob(K, phi, dk)
    N = p.N
    o = _opts(s=s, segments=segments)
    X = torch.empty((N, N, 2), dtype=torch.float64, device=K.device)
    T = torch.empty((N, N, 2), dtype=torch.float64, device=K.device)
    D = torch.empty(N, dtype=torch.float64, device=K.device)
    status = torch.empty(1, dtype=torch.int32, device=K.device)
    need = workspace_bytes([p], FD_WHAT_UDV, s=s, segments=segments)
    wsp, wsn = (ws or _default_ws).get(need, K.device)
    _check(lib.fd_udv(ctypes.byref(p), ctypes.byref(o), X.data_ptr(), D.data_ptr(), T.data_ptr(),
                      wsp, wsn, status.data_ptr(), _stream()))
    _status_check(status, check)
    return torch.view_as_complex(X), D, torch.view_as_complex(T)


def hmc_leapfrog(problems, pi, dU, eps, nsteps, s=0, checkpoint=0, flags=0, check=True,
                 ws: Workspace | None = None):
    """One leapfrog trajectory (Sec. 3.1) of `nsteps` steps of size `eps` for
    every (K, phi, dk) in `problems`, with
        H = 1/2 sum pi^2 + sum phi^2 / (2 dU) - 2 Re log det M(phi).
    Each phi and the momenta are advanced in place: `pi` is one flat float64
    device tensor in the layout of force_batched (the fields' (N_t, N) blocks
    one after another) or a list of (N_t, N) tensors.  Returns dH = H_end -
    H_start per problem (float64 device tensor)."""
    torch = _torch()
    lib = load_library()
    probs = _batch(problems)
    dev = problems[0][1].device
    n = len(probs)
    flat = pi if isinstance(pi, torch.Tensor) else torch.cat([t.reshape(-1) for t in pi])
    total = sum(p.Nt * p.N for p in probs)
    if (not flat.is_cuda or flat.dtype != torch.float64 or not flat.is_contiguous()
            or flat.numel() != total):
        raise FdError(FD_ERR_INVALID_ARG, f"pi must hold {total} contiguous float64 values on the GPU")
    arr = (FdProblem * n)(*probs)
    o = _opts(s=s, checkpoint=checkpoint, flags=flags)
    need = lib.fd_workspace_bytes(arr, n, ctypes.byref(o), FD_WHAT_HMC)
    if need == 0:
        raise FdError(FD_ERR_INVALID_ARG, lib.fd_last_error().decode())
    wsp, wsn = (ws or _default_ws).get(need, dev)
    dH = torch.empty(n, dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    _check(lib.fd_hmc_leapfrog(arr, n, ctypes.byref(o), float(dU), float(eps), int(nsteps),
                               flat.data_ptr(), dH.data_ptr(), wsp, wsn, status.data_ptr(),
                               _stream()))
    _status_check(status, check)
    if not isinstance(pi, torch.Tensor):
        off = 0
        for t in pi:
            t.copy_(flat[off:off + t.numel()].view_as(t))
            off += t.numel()
    return dH


def hmc_trajectory(problems, dU, eps, nsteps, rng, **kw):
    """Momenta drawn from N(0, 1) with the numpy Generator `rng` (one draw of
    all fields' momenta, then one uniform per field: the same sequence as
    HmcPlan.trajectory), one leapfrog trajectory, and the Metropolis step:
    field i keeps its new value with probability min(1, exp(-dH_i)), else
    gets its old one back.  Returns (dH as numpy array, accepted flags)."""
    torch = _torch()
    old = [phi.clone() for _, phi, _ in problems]
    # one flat draw in the layout of force_batched, as HmcPlan.trajectory draws
    total = sum(phi.numel() for _, phi, _ in problems)
    pi = torch.from_numpy(rng.standard_normal(total)).to(problems[0][1].device)
    dH = hmc_leapfrog(problems, pi, dU, eps, nsteps, **kw).cpu().numpy()
    return dH, _metropolis(problems, old, dH, rng)


def _metropolis(problems, old, dH, rng):
    """Accept field i with probability min(1, exp(-dH_i)) (one uniform draw
    per field from `rng`); a rejected field gets its old value back."""
    import numpy as np
    u = rng.random(len(problems))
    acc = u < np.exp(-np.minimum(dH, 700.0))
    for (_, phi, _), o, a in zip(problems, old, acc):
        if not a:
            phi.copy_(o)
    return acc


def diag_response(F, a=None):
    """(1 / N_t) sum_t sum_x a_x (1 - G~_t)_xx from the complex force F
    ((N_t, N) device tensor as fd.force returns it), as a complex128 scalar
    tensor on the device; a = None gives the fermion number averaged over the
    slices."""
    torch = _torch()
    lib = load_library()
    if not isinstance(F, torch.Tensor) or not F.is_cuda or F.dim() != 2:
        raise FdError(FD_ERR_INVALID_ARG, "F must be an (N_t, N) CUDA tensor")
    Nt, N = int(F.shape[0]), int(F.shape[1])
    Fc = F.to(torch.complex128)
    fre, fim = Fc.real.contiguous(), Fc.imag.contiguous()
    ad = None
    if a is not None:
        ad = a.to(device=F.device, dtype=torch.float64).contiguous()
        if ad.numel() != N:
            raise FdError(FD_ERR_INVALID_ARG, f"a must hold {N} values")
    out = torch.empty(2, dtype=torch.float64, device=F.device)
    _check(lib.fd_diag_response(Nt, N, fre.data_ptr(), fim.data_ptr(), _ptr(ad), out.data_ptr(),
                                _stream()))
    return torch.view_as_complex(out)


class HmcPlan:
    """A prepared leapfrog trajectory (fd_hmc_plan_create) on fixed fields,
    momenta and step parameters, with a workspace of its own.  launch() only
    enqueues kernels, so capture() records it in a graph that replay()
    reruns; the fields (the phi tensors of `problems`) and the momenta
    (`self.pi`, flat, in the layout of force_batched) are read at launch time
    and advanced in place.  exp(+-dk K) is computed once here.

        plan = HmcPlan(problems, dU, eps, nsteps, s=8, checkpoint=16)
        dH, acc = plan.trajectory(np.random.default_rng(1))   # draw, run, accept
    """

    def __init__(self, problems, dU, eps, nsteps, s=0, checkpoint=0, flags=0):
        torch = _torch()
        self.lib = load_library()
        self.problems = list(problems)
        self.probs = _batch(self.problems)
        n = len(self.probs)
        dev = self.problems[0][1].device
        self.n = n
        self.shapes = [(p.Nt, p.N) for p in self.probs]
        self.arr = (FdProblem * n)(*self.probs)
        self.pi = torch.zeros(sum(p.Nt * p.N for p in self.probs), dtype=torch.float64, device=dev)
        self.dH = torch.empty(n, dtype=torch.float64, device=dev)
        self.status = torch.empty(n, dtype=torch.int32, device=dev)
        o = _opts(s=s, checkpoint=checkpoint, flags=flags)
        need = self.lib.fd_workspace_bytes(self.arr, n, ctypes.byref(o), FD_WHAT_HMC)
        if need == 0:
            raise FdError(FD_ERR_INVALID_ARG, self.lib.fd_last_error().decode())
        self.ws = Workspace()
        self.wsp, self.wsn = self.ws.get(need, dev)
        self.handle = ctypes.c_void_p(0)
        _check(self.lib.fd_hmc_plan_create(self.arr, n, ctypes.byref(o), float(dU), float(eps),
                                           int(nsteps), self.pi.data_ptr(), self.dH.data_ptr(),
                                           self.wsp, self.wsn, self.status.data_ptr(), _stream(),
                                           ctypes.byref(self.handle)))
        self.graph = None

    def launch(self):
        """Enqueue one trajectory on the current stream."""
        _check(self.lib.fd_hmc_plan_launch(self.handle, _stream()))

    def capture(self):
        """Record launch() in a CUDA/HIP graph (after one warm-up launch on
        a side stream, which advances the fields and momenta once)."""
        torch = _torch()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.launch()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.launch()
        torch.cuda.synchronize()

    def replay(self):
        if self.graph is None:
            self.launch()
        else:
            self.graph.replay()

    def momenta(self):
        """Views of self.pi per field, shaped (N_t, N)."""
        out, off = [], 0
        for Nt, N in self.shapes:
            out.append(self.pi[off:off + Nt * N].view(Nt, N))
            off += Nt * N
        return out

    def trajectory(self, rng, check=True):
        """Momenta from N(0, 1) drawn with the numpy Generator `rng`, one
        trajectory (the graph if captured), and the Metropolis step.  Returns
        (dH as numpy array, accepted flags)."""
        torch = _torch()
        old = [phi.clone() for _, phi, _ in self.problems]
        self.pi.copy_(torch.from_numpy(rng.standard_normal(self.pi.numel())))
        self.replay()
        _status_check(self.status, check)
        dH = self.dH.cpu().numpy()
        return dH, _metropolis(self.problems, old, dH, rng)

    def close(self):
        if self.handle:
            self.lib.fd_hmc_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _c128_matrix(name, t, N=None):
    """Device complex128 (N, N) tensor as a contiguous interleaved buffer."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise FdError(FD_ERR_INVALID_ARG, f"{name} must be a CUDA tensor")
    if t.dim() != 2 or t.shape[0] != t.shape[1] or (N is not None and t.shape[0] != N):
        raise FdError(FD_ERR_INVALID_ARG, f"{name} must be square" +
                      (f" with {N} rows" if N is not None else ""))
    return t.to(torch.complex128).contiguous()


def response_trace(G, A=None, ws: Workspace | None = None):
    """tr((1 - G) A) for one Green's function G (Sec. 4 shortcut) as a
    complex128 scalar tensor on the device; A = None gives the fermion number
    n = 1 - tr G / N (eq. fermion_number).  G and A are (N, N) device tensors
    (A may be real)."""
    torch = _torch()
    lib = load_library()
    Gc = _c128_matrix("G", G)
    N = int(Gc.shape[0])
    Ac = _c128_matrix("A", A, N) if A is not None else None
    out = torch.empty(2, dtype=torch.float64, device=Gc.device)
    need = lib.fd_response_trace_workspace_bytes(N)
    if need == 0:
        raise FdError(FD_ERR_INVALID_ARG, lib.fd_last_error().decode())
    wsp, wsn = (ws or _default_ws).get(need, Gc.device)
    _check(lib.fd_response_trace(N, Gc.data_ptr(), _ptr(Ac), out.data_ptr(), wsp, wsn, _stream()))
    return torch.view_as_complex(out)


def _batch(problems):
    return [_prob(K, phi, dk) for (K, phi, dk) in problems]


def greens_batched(problems, s=0, segments=0, flags=0, check=True, ws: Workspace | None = None,
                   want_g=True):
    """Batched log det (and G) of a list of (K, phi, dk); all problems share the
    kernel launches.  Returns (logdet complex (nprob,), [G_i])."""
    torch = _torch()
    lib = load_library()
    probs = _batch(problems)
    n = len(probs)
    dev = problems[0][0].device
    arr = (FdProblem * n)(*probs)
    o = _opts(s=s, segments=segments, flags=flags)
    ld = torch.empty((n, 2), dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    if want_g:
        total = sum(2 * p.N * p.N for p in probs)
        G = torch.empty(total, dtype=torch.float64, device=dev)
        need = workspace_bytes(probs, FD_WHAT_GREENS, s=s, segments=segments, flags=flags)
        wsp, wsn = (ws or _default_ws).get(need, dev)
        _check(lib.fd_greens_batched(arr, n, ctypes.byref(o), ld.data_ptr(), G.data_ptr(), wsp,
                                     wsn, status.data_ptr(), _stream()))
    else:
        need = workspace_bytes(probs, FD_WHAT_LOGDET, s=s, segments=segments, flags=flags)
        wsp, wsn = (ws or _default_ws).get(need, dev)
        _check(lib.fd_logdet_batched(arr, n, ctypes.byref(o), ld.data_ptr(), wsp, wsn,
                                     status.data_ptr(), _stream()))
    _status_check(status, check)
    Gs = []
    if want_g:
        off = 0
        for p in probs:
            m = 2 * p.N * p.N
            Gs.append(torch.view_as_complex(G[off:off + m].view(p.N, p.N, 2)))
            off += m
    return torch.view_as_complex(ld), Gs


def force_batched(problems, s=0, checkpoint=0, flags=0, check=True, ws: Workspace | None = None):
    """Batched complex force of a list of (K, phi, dk) -> ([F_i], logdet (nprob,))."""
    torch = _torch()
    lib = load_library()
    probs = _batch(problems)
    n = len(probs)
    dev = problems[0][0].device
    arr = (FdProblem * n)(*probs)
    o = _opts(s=s, checkpoint=checkpoint, flags=flags)
    total = sum(p.N * p.Nt for p in probs)
    Fr = torch.empty(total, dtype=torch.float64, device=dev)
    Fi = torch.empty(total, dtype=torch.float64, device=dev)
    ld = torch.empty((n, 2), dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    need = workspace_bytes(probs, FD_WHAT_FORCE, s=s, checkpoint=checkpoint, flags=flags)
    wsp, wsn = (ws or _default_ws).get(need, dev)
    _check(lib.fd_force_batched(arr, n, ctypes.byref(o), ld.data_ptr(), Fr.data_ptr(),
                                Fi.data_ptr(), wsp, wsn, status.data_ptr(), _stream()))
    _status_check(status, check)
    Fs, off = [], 0
    for p in probs:
        m = p.N * p.Nt
        Fs.append(torch.complex(Fr[off:off + m], Fi[off:off + m]).view(p.Nt, p.N))
        off += m
    return Fs, torch.view_as_complex(ld)


# ---------------------------------------------------------------------------
# Prepared calls, graph replay, autograd and autotuning
# ---------------------------------------------------------------------------
_WHAT = {"logdet": FD_WHAT_LOGDET, "greens": FD_WHAT_GREENS, "force": FD_WHAT_FORCE}


class Plan:
    """One prepared call (fd_plan_create) on fixed problems, outputs and a
    workspace of its own.  launch() only enqueues kernels, so it can be
    captured in a graph; phi tensors are read at launch time and may be
    updated in place between launches.

    what: "logdet", "greens" or "force"; problems: list of (K, phi, dk).
    reuse_e: compute exp(+-dk K) once now and skip it in every launch (K and
    dk must then stay fixed).
    want_g: with "force", also return G = M^{-1} (the force's checkpoint at
    row 0 already holds it).
    """

    def __init__(self, what, problems, s=0, checkpoint=0, segments=0, reuse_e=False,
                 want_g=False, flags=0):
        torch = _torch()
        self.lib = load_library()
        self.what = _WHAT[what]
        self.problems = list(problems)
        self.probs = _batch(self.problems)
        n = len(self.probs)
        dev = self.problems[0][0].device
        self.n = n
        self.arr = (FdProblem * n)(*self.probs)
        self.ld = torch.empty((n, 2), dtype=torch.float64, device=dev)
        self.status = torch.empty(n, dtype=torch.int32, device=dev)
        self.G = self.Fr = self.Fi = None
        if self.what == FD_WHAT_GREENS or (self.what == FD_WHAT_FORCE and want_g):
            self.G = torch.empty(sum(2 * p.N * p.N for p in self.probs), dtype=torch.float64,
                                 device=dev)
        if self.what == FD_WHAT_FORCE:
            tot = sum(p.N * p.Nt for p in self.probs)
            self.Fr = torch.empty(tot, dtype=torch.float64, device=dev)
            self.Fi = torch.empty(tot, dtype=torch.float64, device=dev)
        self.ws = Workspace()
        flags &= ~FD_REUSE_E
        need = workspace_bytes(self.probs, self.what, s=s, checkpoint=checkpoint,
                               segments=segments, flags=flags)
        self.wsp, self.wsn = self.ws.get(need, dev)
        self.handle = ctypes.c_void_p(0)
        if reuse_e:
            # one full call fills exp(+-dk K) into this workspace
            self._create(_opts(s=s, checkpoint=checkpoint, segments=segments, flags=flags))
            self.launch()
            torch.cuda.current_stream().synchronize()
            _status_check(self.status, True)
            self.lib.fd_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)
        self._create(_opts(s=s, checkpoint=checkpoint, segments=segments,
                           flags=flags | (FD_REUSE_E if reuse_e else 0)))

    def _create(self, o):
        _check(self.lib.fd_plan_create(
            self.what, self.arr, self.n, ctypes.byref(o), _ptr(self.ld), _ptr(self.G),
            _ptr(self.Fr), _ptr(self.Fi), self.wsp, self.wsn, _ptr(self.status), _stream(),
            ctypes.byref(self.handle)))

    def launch(self):
        """Enqueue the plan's kernels on the current stream."""
        _check(self.lib.fd_plan_launch(self.handle, _stream()))

    def segments(self):
        """Per problem: time segments (logdet / greens) or checkpoint
        intervals (force) of this plan."""
        buf = (ctypes.c_int32 * self.n)()
        _check(min(0, self.lib.fd_plan_segments(self.handle, buf, self.n)))
        return [int(v) for v in buf]

    def greens(self):
        """[G_i] views (greens, or force with want_g); [] otherwise."""
        torch = _torch()
        if self.G is None:
            return []
        out, off = [], 0
        for p in self.probs:
            m = 2 * p.N * p.N
            out.append(torch.view_as_complex(self.G[off:off + m].view(p.N, p.N, 2)))
            off += m
        return out

    def results(self, check=False):
        """Outputs: logdet (n,) complex, plus [G_i] (greens) or [F_i] (force;
        complex (Nt, N), built from the real and imaginary parts)."""
        torch = _torch()
        _status_check(self.status, check)
        ld = torch.view_as_complex(self.ld)
        if self.what == FD_WHAT_GREENS:
            return ld, self.greens()
        if self.what == FD_WHAT_FORCE:
            out, off = [], 0
            for p in self.probs:
                m = p.N * p.Nt
                out.append(torch.complex(self.Fr[off:off + m], self.Fi[off:off + m])
                           .view(p.Nt, p.N))
                off += m
            return ld, out
        return ld, []

    def close(self):
        if self.handle:
            self.lib.fd_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trajectory:
    """The force and log det of fixed K captured once as a graph and replayed
    for each molecular-dynamics step of HMC (Sec. 3.1: every leapfrog step
    needs dH/dphi at the current field).

        traj = Trajectory(K, phi0, dk, s=8, checkpoint=16)
        logdet, F = traj.step(phi)      # F: (Nt, N) complex

        traj = Trajectory(problems=[(K, phi_j, dk), ...], want_g=True)
        logdets, Fs, Gs = traj.step([phi_j, ...])   # a batch in one graph

    exp(+-dk K) is computed once at construction; every replay runs the
    interval chains, the prefix / suffix scans, the checkpoint closes and the
    force sweep on static copies of the fields (step() copies its arguments
    in first).  Outputs are overwritten by the next step(); clone to keep.
    """

    def __init__(self, K=None, phi=None, dk=None, s=0, checkpoint=0, what="force", want_g=False,
                 problems=None):
        torch = _torch()
        self.single = problems is None
        if self.single:
            problems = [(K, phi, dk)]
        self.phis = [p.clone() for (_, p, _) in problems]
        probs = [(Kj, ph, dkj) for (Kj, _, dkj), ph in zip(problems, self.phis)]
        self.plan = Plan(what, probs, s=s, checkpoint=checkpoint, reuse_e=True, want_g=want_g)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.plan.launch()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.plan.launch()
        torch.cuda.synchronize()

    def replay(self):
        """Replay the captured step on the current static fields."""
        self.graph.replay()

    def step(self, phi=None, check=True):
        if phi is not None:
            if self.single:
                self.phis[0].copy_(phi)
            else:
                for dst, src in zip(self.phis, phi):
                    dst.copy_(src)
        self.graph.replay()
        ld, outs = self.plan.results(check=check)
        if self.single:
            return ld[0], (outs[0] if outs else None)
        return ld, outs, self.plan.greens()


def _logdet_function():
    torch = _torch()

    class LogDet(torch.autograd.Function):
        """log det M as a differentiable function of phi (K, dk fixed).

        Forward computes log det M with FD_KEEP_CHECKPOINTS when phi needs a
        gradient: the UDV products of the checkpoint intervals (and the
        prefix / suffix or window products built from them) stay in a
        workspace owned by the autograd context.  Backward runs only the
        force's checkpoint items on that workspace: G~ at every checkpoint
        from its two stored factors, then the slices in between carried from
        it (recomputed, not stored), F = d log det M / d phi.  For a real
        loss with upstream gradient g = dL/dRe + i dL/dIm the backward
        returns g.real * Re F + g.imag * Im F.
        """

        @staticmethod
        def forward(ctx, phi, K, dk, s, checkpoint):
            if ctx.needs_input_grad[0]:
                ws = Workspace()
                ld = logdet(K, phi.detach(), dk, s=s, checkpoint=checkpoint,
                            flags=FD_KEEP_CHECKPOINTS, ws=ws)
                ctx.save_for_backward(phi)
                ctx.fd_args = (K, dk, s, checkpoint, ws)
            else:
                ld = logdet(K, phi.detach(), dk, s=s)
            return ld.clone()

        @staticmethod
        def backward(ctx, g):
            (phi,) = ctx.saved_tensors
            K, dk, s, checkpoint, ws = ctx.fd_args
            F = force(K, phi.detach(), dk, s=s, checkpoint=checkpoint,
                      flags=FD_KEEP_CHECKPOINTS, ws=ws)
            g = g.to(torch.complex128)
            return g.real * F.real + g.imag * F.imag, None, None, None, None

    return LogDet


_LogDet = None


def log_det(phi, K, dk, s=0, checkpoint=0):
    """Differentiable log det M (complex scalar); see LogDet."""
    global _LogDet
    if _LogDet is None:
        _LogDet = _logdet_function()
    return _LogDet.apply(phi, K, dk, int(s), int(checkpoint))


def autotune(problems, what="greens", s=0, checkpoint=0, segments=0):
    """Time candidate (s, segments) for these (K, phi, dk) problems on the GPU and
    store the winner for later calls with those options left at 0.
    Returns {"s", "segments", "checkpoint", "ms"}."""
    _torch()
    lib = load_library()
    probs = _batch(problems)
    arr = (FdProblem * len(probs))(*probs)
    o = _opts(s=s, checkpoint=checkpoint, segments=segments)
    best = FdOptions()
    ms = ctypes.c_float(0.0)
    _check(lib.fd_autotune(_WHAT[what], arr, len(probs), ctypes.byref(o), _stream(),
                           ctypes.byref(best), ctypes.byref(ms)))
    return {"s": best.s, "segments": best.segments, "checkpoint": best.checkpoint,
            "ms": float(ms.value)}


def tune_save(path: str):
    _check(load_library().fd_tune_save(os.fsencode(path)))


def tune_load(path: str) -> int:
    n = load_library().fd_tune_load(os.fsencode(path))
    if n < 0:
        _check(n)
    return n


def tune_clear():
    _check(load_library().fd_tune_clear())
