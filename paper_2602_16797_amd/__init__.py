"""Python binding of the gfx950 RLOBPCG library (argument marshalling only).

Every computation runs in the HIP kernels of ``libpaper_2602_16797_amd.so``;
this module only checks shapes, allocates the output tensors with torch on the
caller's device and passes raw pointers and the current HIP stream through the
C-ABI declared in ``include/rlobpcg.h``.  There is no CPU fallback: if the
library is missing or no GPU is visible, every call raises.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpaper_2602_16797_amd.so")

RL_OK = 0
RL_NOT_CONVERGED = 1
RL_ERR_ARG = -1
RL_ERR_DEVICE = -2
RL_ERR_NOMEM = -3
RL_ERR_NONFINITE = -4
RL_ERR_UNSUPPORTED = -7
RL_PENDING = 2
RL_ERR_ADMISSION = -5
RL_ERR_CANCELLED = -6
RL_ERR_SCRATCH = -8

RL_SKETCH_F64 = 0
RL_SKETCH_F32 = 1
RL_SKETCH_BF16 = 2
SKETCH_PRECS = {"f64": RL_SKETCH_F64, "f32": RL_SKETCH_F32, "bf16": RL_SKETCH_BF16}
LOOP_PRECONDS = {"sketch": 0, "diag": 1, "none": 2}  # RL_PREC_*
ORTHS = {"cgs2": 0, "svqb": 1}  # RL_ORTH_*
STOP_RULES = {"paper": 0, "tol": 1, "none": 2}

EXPORTED = (
    "rl_create", "rl_destroy", "rl_set_stream", "rl_default_opts",
    "rl_svds_smallest_d", "rl_svds_smallest_z",
    "rl_step_sketch", "rl_step_qr", "rl_step_astream", "rl_step_astream_iter", "rl_step_astream_iter_noalloc",
    "rl_step_tall_svd", "rl_step_orth",
    "rl_step_sketch_f32", "rl_step_qr_lowp", "rl_status_string",
    "rl_server_create", "rl_server_submit", "rl_server_poll", "rl_server_wait", "rl_server_destroy",
)


class RlOpts(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int64),
        ("zeta", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("tau", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("stop_rule", ctypes.c_int32),
        ("dot2", ctypes.c_int32),
        ("init_iters", ctypes.c_int32),
        ("lanczos_steps", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("sketch_prec", ctypes.c_int32),
        ("loop_precond", ctypes.c_int32),
        ("orth", ctypes.c_int32),
        ("refresh", ctypes.c_int32),
        ("prec_guard", ctypes.c_int32),
        ("lock", ctypes.c_int32),
    ]


class RlInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("a_passes", ctypes.c_int32),
        ("degenerate", ctypes.c_int32),
        ("zero_theta", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("sigma1", ctypes.c_double),
        ("t_setup_us", ctypes.c_double),
        ("t_iter_us", ctypes.c_double),
        ("t_final_us", ctypes.c_double),
        ("bytes_a", ctypes.c_int64),
        ("hist_cap", ctypes.c_int32),
        ("n_astream", ctypes.c_int32),
        ("t_astream_us", ctypes.c_double),
        ("theta_hist", ctypes.POINTER(ctypes.c_double)),
        ("rnorm_hist", ctypes.POINTER(ctypes.c_double)),
        ("n_pass_g", ctypes.c_int32),
        ("sketch_prec_used", ctypes.c_int32),
        ("t_pass_g_us", ctypes.c_double),
        ("kappa_est", ctypes.c_double),
        ("n_locked", ctypes.c_int32),
        ("act_mask", ctypes.c_int32),
    ]


class RlRequest(ctypes.Structure):
    """Mirror of rl_request (include/rlobpcg.h)."""
    _fields_ = [
        ("is_complex", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("A", ctypes.c_void_p),
        ("lda", ctypes.c_int64),
        ("opts", ctypes.POINTER(RlOpts)),
        ("sigma", ctypes.c_void_p),
        ("V", ctypes.c_void_p),
        ("ldv", ctypes.c_int64),
        ("U", ctypes.c_void_p),
        ("ldu", ctypes.c_int64),
    ]


class RlJobTimes(ctypes.Structure):
    """Mirror of rl_job_times (include/rlobpcg.h)."""
    _fields_ = [
        ("queued_us", ctypes.c_double),
        ("run_us", ctypes.c_double),
        ("latency_us", ctypes.c_double),
        ("workspace_bytes", ctypes.c_int64),
    ]


class RlError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {status_string(code)} ({code})")


_lib = None


def load_library() -> ctypes.CDLL:
    """Load the built library (no GPU is touched)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run python -m paper_2602_16797_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32, U64, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    lib.rl_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P]
    lib.rl_destroy.argtypes = [P]
    lib.rl_set_stream.argtypes = [P, P]
    lib.rl_default_opts.argtypes = [ctypes.POINTER(RlOpts), I64, I64, I32]
    for name in ("rl_svds_smallest_d", "rl_svds_smallest_z"):
        getattr(lib, name).argtypes = [P, I64, I64, P, I64, I32, ctypes.POINTER(RlOpts), P, P, I64, P, I64,
                                       ctypes.POINTER(RlInfo)]
    lib.rl_step_sketch.argtypes = [P, ctypes.c_int, I64, I64, P, I64, I64, I32, U64, P, I64]
    lib.rl_step_qr.argtypes = [P, ctypes.c_int, I64, I64, P, I64, P, P]
    lib.rl_step_sketch_f32.argtypes = [P, I64, I64, P, I64, I64, I32, U64, P, I64]
    lib.rl_step_qr_lowp.argtypes = [P, I64, I64, P, I64, I32, P, P]
    lib.rl_step_astream.argtypes = [P, ctypes.c_int, I64, I64, P, I64, I32, P, P, P, I32]
    lib.rl_step_astream_iter.argtypes = [P, ctypes.c_int, I64, I64, P, I64, I32, P, P, P, P, P, I32]
    lib.rl_step_astream_iter_noalloc.argtypes = [P, ctypes.c_int, I64, I64, P, I64, I32, P, P, P, P, P, I32]
    lib.rl_step_tall_svd.argtypes = [P, ctypes.c_int, I64, I32, P, P, P]
    lib.rl_step_orth.argtypes = [P, ctypes.c_int, I64, I32, P, P, I32, I32, P, ctypes.POINTER(I32)]
    lib.rl_status_string.argtypes = [ctypes.c_int]
    lib.rl_server_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.c_size_t, I32]
    lib.rl_server_submit.argtypes = [P, ctypes.POINTER(RlRequest), ctypes.POINTER(U64)]
    lib.rl_server_poll.argtypes = [P, U64, ctypes.POINTER(I32), ctypes.POINTER(RlInfo), ctypes.POINTER(RlJobTimes)]
    lib.rl_server_wait.argtypes = [P, U64, I64, ctypes.POINTER(RlInfo), ctypes.POINTER(RlJobTimes)]
    lib.rl_server_destroy.argtypes = [P]
    lib.rl_status_string.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name != "rl_status_string":
            getattr(lib, name).restype = ctypes.c_int
    _ = D
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load_library().rl_status_string(int(code)).decode()


def default_opts(m: int, n: int, k: int) -> RlOpts:
    o = RlOpts()
    rc = load_library().rl_default_opts(ctypes.byref(o), m, n, k)
    if rc != RL_OK:
        raise RlError(rc, "rl_default_opts")
    return o


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2602_16797_amd needs a ROCm GPU: torch.cuda.is_available() is False")
    return torch


class Handle:
    """One library handle on one device, bound to the current torch stream."""

    def __init__(self, device: int = 0):
        torch = _torch()
        self.lib = load_library()
        self.device = device
        with torch.cuda.device(device):
            stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        rc = self.lib.rl_create(ctypes.byref(h), device, ctypes.c_void_p(stream))
        if rc != RL_OK:
            raise RlError(rc, "rl_create")
        self.h = h

    def sync_stream(self):
        torch = _torch()
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.lib.rl_set_stream(self.h, ctypes.c_void_p(s))

    def close(self):
        if getattr(self, "h", None):
            self.lib.rl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles: dict[int, Handle] = {}


def handle(device: int = 0) -> Handle:
    h = _handles.get(device)
    if h is None or h.h is None:
        h = Handle(device)
        _handles[device] = h
    h.sync_stream()
    return h


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _check_matrix(A, torch):
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    if A.dim() != 2:
        raise ValueError("A must be 2-D")
    if A.dtype not in (torch.float64, torch.complex128):
        raise ValueError("A must be float64 or complex128")
    if A.stride(1) != 1:
        raise ValueError("A must be row-major with unit column stride")


@dataclass
class SolveResult:
    sigma: object
    V: object
    U: object
    status: int
    iters: int
    a_passes: int
    sigma1: float
    degenerate: bool
    zero_theta: bool
    t_setup_us: float
    t_iter_us: float
    t_final_us: float
    bytes_a: int
    n_astream: int = 0
    t_astream_us: float = 0.0
    n_pass_g: int = 0
    t_pass_g_us: float = 0.0
    sketch_prec_used: int = 0
    kappa_est: float = 0.0
    n_locked: int = 0
    act_mask: int = 0
    block: int = 0
    theta_hist: np.ndarray = field(default=None)
    rnorm_hist: np.ndarray = field(default=None)


def make_opts(m: int, n: int, k: int, *, block=None, d=None, zeta=None, seed=0, tau=None, max_iter=None,
              check_every=None, rule="paper", dot2=None, init_iters=None, lanczos_steps=None,
              profile=False, sketch_prec="f64", loop_precond="sketch", orth="cgs2", refresh=None,
              prec_guard=None, lock=None) -> RlOpts:
    o = default_opts(m, n, k if block is None else block)
    o.block = k if block is None else block
    if block is not None:
        o.max_iter = 200 if block == 1 else 100
    if d is not None:
        o.d = d
    if zeta is not None:
        o.zeta = zeta
    o.seed = seed
    if tau is not None:
        o.tau = tau
    if max_iter is not None:
        o.max_iter = max_iter
    if check_every is not None:
        o.check_every = check_every
    o.stop_rule = STOP_RULES[rule]
    if dot2 is not None:
        o.dot2 = int(bool(dot2))
    if init_iters is not None:
        o.init_iters = init_iters
    if lanczos_steps is not None:
        o.lanczos_steps = lanczos_steps
    o.profile = int(bool(profile))
    o.sketch_prec = SKETCH_PRECS[sketch_prec]
    o.loop_precond = LOOP_PRECONDS[loop_precond]
    o.orth = ORTHS[orth]
    if refresh is not None:
        o.refresh = int(bool(refresh))
    if prec_guard is not None:
        o.prec_guard = int(bool(prec_guard))
    if lock is not None:
        o.lock = int(bool(lock))
    return o


def rl_svds_smallest(A, k: int, *, want_u: bool = True, history: bool = True, **kw) -> SolveResult:
    """k smallest singular triplets of the device matrix A (C-ABI rl_svds_smallest_d/_z)."""
    torch = _torch()
    _check_matrix(A, torch)
    m, n = A.shape
    dev = A.device.index or 0
    h = handle(dev)
    o = make_opts(m, n, k, **kw)
    cplx = A.dtype == torch.complex128
    sigma = torch.empty(k, dtype=torch.float64, device=A.device)
    V = torch.empty((n, k), dtype=A.dtype, device=A.device)
    U = torch.empty((m, k), dtype=A.dtype, device=A.device) if want_u else None
    info = RlInfo()
    cap = o.max_iter + 1
    th = np.full((cap, o.block), np.nan)
    rn = np.full((cap, o.block), np.nan)
    if history:
        info.hist_cap = cap
        info.theta_hist = th.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        info.rnorm_hist = rn.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    fn = h.lib.rl_svds_smallest_z if cplx else h.lib.rl_svds_smallest_d
    rc = fn(h.h, m, n, _ptr(A), A.stride(0), k, ctypes.byref(o), _ptr(sigma), _ptr(V), k,
            _ptr(U) if U is not None else None, k, ctypes.byref(info))
    if rc not in (RL_OK, RL_NOT_CONVERGED):
        raise RlError(rc, "rl_svds_smallest")
    it = info.iters
    return SolveResult(sigma=sigma, V=V, U=U, status=rc, iters=it, a_passes=info.a_passes, sigma1=info.sigma1,
                       degenerate=bool(info.degenerate), zero_theta=bool(info.zero_theta),
                       t_setup_us=info.t_setup_us, t_iter_us=info.t_iter_us, t_final_us=info.t_final_us,
                       bytes_a=info.bytes_a, n_astream=info.n_astream, t_astream_us=info.t_astream_us,
                       n_pass_g=info.n_pass_g, t_pass_g_us=info.t_pass_g_us,
                       sketch_prec_used=info.sketch_prec_used, kappa_est=info.kappa_est,
                       n_locked=info.n_locked, act_mask=info.act_mask, block=info.block, theta_hist=th[: it + 1].copy() if history else None,
                       rnorm_hist=rn[: it + 1].copy() if history else None)


def rl_step_sketch(A, d: int, zeta: int, seed: int):
    torch = _torch()
    _check_matrix(A, torch)
    m, n = A.shape
    h = handle(A.device.index or 0)
    Y = torch.empty((d, n), dtype=A.dtype, device=A.device)
    rc = h.lib.rl_step_sketch(h.h, int(A.is_complex()), m, n, _ptr(A), A.stride(0), d, zeta,
                              ctypes.c_uint64(seed), _ptr(Y), n)
    if rc != RL_OK:
        raise RlError(rc, "rl_step_sketch")
    return Y


def rl_step_qr(Y):
    torch = _torch()
    _check_matrix(Y, torch)
    d, n = Y.shape
    h = handle(Y.device.index or 0)
    R = torch.empty((n, n), dtype=Y.dtype, device=Y.device)
    Rinv = torch.empty((n, n), dtype=Y.dtype, device=Y.device)
    rc = h.lib.rl_step_qr(h.h, int(Y.is_complex()), d, n, _ptr(Y), Y.stride(0), _ptr(R), _ptr(Rinv))
    if rc != RL_OK:
        raise RlError(rc, "rl_step_qr")
    return R, Rinv


def rl_step_sketch_f32(A, d: int, zeta: int, seed: int):
    """FP32 sketch of the real FP64 device matrix A (C-ABI rl_step_sketch_f32)."""
    torch = _torch()
    _check_matrix(A, torch)
    if A.is_complex():
        raise ValueError("the reduced-precision sketch takes real A")
    m, n = A.shape
    h = handle(A.device.index or 0)
    Y = torch.empty((d, n), dtype=torch.float32, device=A.device)
    rc = h.lib.rl_step_sketch_f32(h.h, m, n, _ptr(A), A.stride(0), d, zeta, ctypes.c_uint64(seed), _ptr(Y), n)
    if rc != RL_OK:
        raise RlError(rc, "rl_step_sketch_f32")
    return Y


def rl_step_qr_lowp(Y, sketch_prec: str = "f32"):
    """R (FP64, promoted) and R^{-1} of the FP32 sketch Y (C-ABI rl_step_qr_lowp)."""
    torch = _torch()
    if not (isinstance(Y, torch.Tensor) and Y.is_cuda and Y.dtype == torch.float32 and Y.dim() == 2):
        raise TypeError("Y must be a 2-D float32 tensor on a GPU")
    Y = Y.contiguous()
    d, n = Y.shape
    h = handle(Y.device.index or 0)
    R = torch.empty((n, n), dtype=torch.float64, device=Y.device)
    Rinv = torch.empty((n, n), dtype=torch.float64, device=Y.device)
    rc = h.lib.rl_step_qr_lowp(h.h, d, n, _ptr(Y), n, SKETCH_PRECS[sketch_prec], _ptr(R), _ptr(Rinv))
    if rc != RL_OK:
        raise RlError(rc, "rl_step_qr_lowp")
    return R, Rinv


def rl_step_astream(A, W, dot2: bool = False):
    torch = _torch()
    _check_matrix(A, torch)
    m, n = A.shape
    W = W.contiguous()
    b = W.shape[1]
    h = handle(A.device.index or 0)
    AW = torch.empty((m, b), dtype=A.dtype, device=A.device)
    G = torch.empty((n, b), dtype=A.dtype, device=A.device)
    rc = h.lib.rl_step_astream(h.h, int(A.is_complex()), m, n, _ptr(A), A.stride(0), b, _ptr(W), _ptr(AW),
                               _ptr(G), int(bool(dot2)))
    if rc != RL_OK:
        raise RlError(rc, "rl_step_astream")
    return AW, G


def rl_step_astream_iter(A, W, AV, AX=None, dot2: bool = False):
    """AW = A W and G3 = [A^* AV | A^* AX | A^* AW] (3 x n x b) in one pass."""
    torch = _torch()
    _check_matrix(A, torch)
    m, n = A.shape
    W, AV = W.contiguous(), AV.contiguous()
    b = W.shape[1]
    if AV.shape != (m, b) or (AX is not None and AX.shape != (m, b)) or W.shape != (n, b):
        raise ValueError("rl_step_astream_iter: W must be n x b, AV and AX m x b")
    if AX is not None:
        AX = AX.contiguous()
    h = handle(A.device.index or 0)
    AW = torch.empty((m, b), dtype=A.dtype, device=A.device)
    G3 = torch.empty((3, n, b), dtype=A.dtype, device=A.device)
    rc = h.lib.rl_step_astream_iter(h.h, int(A.is_complex()), m, n, _ptr(A), A.stride(0), b, _ptr(W), _ptr(AV),
                                    _ptr(AX) if AX is not None else None, _ptr(AW), _ptr(G3), int(bool(dot2)))
    if rc != RL_OK:
        raise RlError(rc, "rl_step_astream_iter")
    return AW, G3


def rl_step_astream_iter_noalloc(A, W, AV, AX=None, dot2: bool = False, AW=None, G3=None):
    """rl_step_astream_iter through the allocation-free entry point: the
    library allocates nothing (its scratch is a static 32 MiB per device).
    AW (m x b) and G3 (3 x n x b) may be passed preallocated; otherwise torch
    allocates them here.  The call only enqueues on the current stream."""
    torch = _torch()
    _check_matrix(A, torch)
    m, n = A.shape
    b = W.shape[1]
    for t in (W, AV) + ((AX,) if AX is not None else ()):
        if not t.is_contiguous():
            raise ValueError("rl_step_astream_iter_noalloc: W, AV and AX must be contiguous")
    if AV.shape != (m, b) or (AX is not None and AX.shape != (m, b)) or W.shape != (n, b):
        raise ValueError("rl_step_astream_iter_noalloc: W must be n x b, AV and AX m x b")
    if AW is None:
        AW = torch.empty((m, b), dtype=A.dtype, device=A.device)
    if G3 is None:
        G3 = torch.empty((3, n, b), dtype=A.dtype, device=A.device)
    if AW.shape != (m, b) or G3.shape != (3, n, b) or not (AW.is_contiguous() and G3.is_contiguous()):
        raise ValueError("rl_step_astream_iter_noalloc: AW must be m x b and G3 3 x n x b, contiguous")
    h = handle(A.device.index or 0)
    rc = h.lib.rl_step_astream_iter_noalloc(h.h, int(A.is_complex()), m, n, _ptr(A), A.stride(0), b, _ptr(W),
                                            _ptr(AV), _ptr(AX) if AX is not None else None, _ptr(AW), _ptr(G3),
                                            int(bool(dot2)))
    if rc != RL_OK:
        raise RlError(rc, "rl_step_astream_iter_noalloc")
    return AW, G3


def rl_step_tall_svd(P):
    torch = _torch()
    P = P.contiguous()
    m, t = P.shape
    h = handle(P.device.index or 0)
    sigma = torch.empty(t, dtype=torch.float64, device=P.device)
    C = torch.empty((t, t), dtype=P.dtype, device=P.device)
    rc = h.lib.rl_step_tall_svd(h.h, int(P.is_complex()), m, t, _ptr(P), _ptr(sigma), _ptr(C))
    if rc != RL_OK:
        raise RlError(rc, "rl_step_tall_svd")
    return sigma, C


def rl_step_orth(W, V=None, X=None):
    """Orthonormal basis of W's block after two block projections against
    [V X] (V None: no projection).  Returns (Q, degenerate); W is not changed."""
    torch = _torch()
    Q = W.contiguous().clone()
    n, b = Q.shape
    for t in (V, X):
        if t is not None and (t.shape != (n, b) or t.dtype != Q.dtype):
            raise ValueError("rl_step_orth: V and X must be n x b of W's dtype")
    Vc = V.contiguous() if V is not None else None
    Xc = X.contiguous() if X is not None else None
    h = handle(Q.device.index or 0)
    deg = ctypes.c_int32(0)
    rc = h.lib.rl_step_orth(h.h, int(Q.is_complex()), n, b, _ptr(Vc) if Vc is not None else None,
                            _ptr(Xc) if Xc is not None else None, int(Vc is not None), int(Xc is not None),
                            _ptr(Q), ctypes.byref(deg))
    if rc != RL_OK:
        raise RlError(rc, "rl_step_orth")
    return Q, bool(deg.value)


@dataclass
class ServedResult:
    sigma: object
    V: object
    U: object
    status: int
    iters: int
    queued_us: float
    run_us: float
    latency_us: float
    workspace_bytes: int


class Server:
    """Continuous-batching server of the C-ABI (rl_server_*): submit solves of
    different shapes, each admitted when a slot is free and its workspace fits
    the HBM budget; results come back per ticket."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 8, device: int = 0):
        self.lib = load_library()
        self.h = ctypes.c_void_p()
        rc = self.lib.rl_server_create(ctypes.byref(self.h), device, hbm_budget_bytes, max_inflight)
        if rc != RL_OK:
            raise RlError(rc, "rl_server_create")
        self.device = device
        self._live = {}

    def submit(self, A, k: int, *, want_u: bool = True, **kw) -> int:
        torch = _torch()
        _check_matrix(A, torch)
        m, n = A.shape
        o = make_opts(m, n, k, **kw)
        sigma = torch.empty(k, dtype=torch.float64, device=A.device)
        V = torch.empty((n, k), dtype=A.dtype, device=A.device)
        U = torch.empty((m, k), dtype=A.dtype, device=A.device) if want_u else None
        req = RlRequest(is_complex=int(A.dtype == torch.complex128), k=k, m=m, n=n, A=_ptr(A), lda=A.stride(0),
                        opts=ctypes.pointer(o), sigma=_ptr(sigma), V=_ptr(V), ldv=k,
                        U=_ptr(U) if U is not None else None, ldu=k)
        t = ctypes.c_uint64()
        # the inputs were produced on torch's stream; the server's slots use their own
        torch.cuda.current_stream(A.device).synchronize()
        rc = self.lib.rl_server_submit(self.h, ctypes.byref(req), ctypes.byref(t))
        if rc != RL_OK:
            raise RlError(rc, "rl_server_submit")
        self._live[t.value] = (A, sigma, V, U, o)
        return t.value

    def _result(self, ticket, rc, info, times):
        A, sigma, V, U, _ = self._live.pop(ticket)
        if rc not in (RL_OK, RL_NOT_CONVERGED):
            raise RlError(rc, "served solve")
        return ServedResult(sigma=sigma, V=V, U=U, status=rc, iters=info.iters, queued_us=times.queued_us,
                            run_us=times.run_us, latency_us=times.latency_us,
                            workspace_bytes=times.workspace_bytes)

    def wait(self, ticket: int, timeout_us: int = -1):
        info, times = RlInfo(), RlJobTimes()
        rc = self.lib.rl_server_wait(self.h, ticket, timeout_us, ctypes.byref(info), ctypes.byref(times))
        if rc == RL_PENDING:
            return None
        return self._result(ticket, rc, info, times)

    def poll(self, ticket: int):
        done = ctypes.c_int32()
        info, times = RlInfo(), RlJobTimes()
        rc = self.lib.rl_server_poll(self.h, ticket, ctypes.byref(done), ctypes.byref(info), ctypes.byref(times))
        if not done.value:
            return None
        return self._result(ticket, rc, info, times)

    def close(self):
        if self.h:
            self.lib.rl_server_destroy(self.h)
            self.h = ctypes.c_void_p()
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
