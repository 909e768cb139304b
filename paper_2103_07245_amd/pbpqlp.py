"""Python binding of libpbpqlp.so (ctypes; argument marshalling only).

Every computation runs in the library's HIP kernels on the tensor's device;
this module only checks shapes, allocates outputs and workspace through
PyTorch's caching allocator, and passes raw device pointers and the current
HIP stream across the C ABI declared in include/pbpqlp.h.  There is no CPU
fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbpqlp.so")

# enums of include/pbpqlp.h
OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, 1, 2, 3, 4
F64, F32 = 0, 1
PREC = {"native": 0, "bf16": 1, "fp16": 2, "bf16x3": 3}
FLAG_DEPENDENT, FLAG_NONFINITE, FLAG_INTERNAL, FLAG_BADINPUT = 1, 2, 4, 8

# named precision plans: (sketch pass, power-iteration passes, projection pass)
PLANS = {
    "native": ("native", "native", "native"),
    "bf16": ("bf16", "bf16", "bf16"),
    "fp16": ("fp16", "fp16", "fp16"),
    "mixed": ("bf16", "bf16", "bf16x3"),
    "bf16x3": ("bf16x3", "bf16x3", "bf16x3"),
}


class PbpqlpError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib().pbpqlp_status_string(status).decode()
        super().__init__(f"{where}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("sketch_prec", ctypes.c_int), ("power_prec", ctypes.c_int),
                ("proj_prec", ctypes.c_int), ("split_k", ctypes.c_int),
                ("gram_workgroups", ctypes.c_int), ("fp16_scale_a", ctypes.c_double), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class InfoStruct(ctypes.Structure):
    _fields_ = [("status_flags", ctypes.c_int), ("n_dependent", ctypes.c_int),
                ("l", ctypes.c_int), ("q", ctypes.c_int), ("norm_a_fro2", ctypes.c_double),
                ("norm_l_fro2", ctypes.c_double), ("resid_rel_est", ctypes.c_double),
                ("reserved", ctypes.c_double * 2)]


INFO_BYTES = ctypes.sizeof(InfoStruct)


class ProblemStruct(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("k", ctypes.c_int), ("p", ctypes.c_int),
                ("q", ctypes.c_int), ("seed", ctypes.c_uint64), ("Q", ctypes.c_void_p),
                ("ldq", ctypes.c_int64), ("L", ctypes.c_void_p), ("ldl", ctypes.c_int64),
                ("P", ctypes.c_void_p), ("ldp", ctypes.c_int64), ("info", ctypes.c_void_p)]


class RRStruct(ctypes.Structure):
    _fields_ = [("orientation", ctypes.c_int), ("orientation_used", ctypes.c_int), ("R", ctypes.c_void_p),
                ("ldr", ctypes.c_int64), ("rank_tol", ctypes.c_double), ("d_rank", ctypes.c_void_p)]


ORIENT = {"AT": 0, "A": 1, "auto": 2}


class AutoResult(ctypes.Structure):
    _fields_ = [("q_pred", ctypes.c_int), ("k_pred", ctypes.c_int), ("q_used", ctypes.c_int),
                ("k_used", ctypes.c_int), ("fell_back", ctypes.c_int), ("passes", ctypes.c_int),
                ("resid_first", ctypes.c_double), ("resid_final", ctypes.c_double)]


class TunePlanStruct(ctypes.Structure):
    _fields_ = [("split_k", ctypes.c_int), ("gram_workgroups", ctypes.c_int), ("ms", ctypes.c_double)]


NOALLOC_SCRATCH_BYTES = 64 << 20   # PBPQLP_NOALLOC_SCRATCH_BYTES

MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 64, 128, 6, 25606
PROBE_K, PROBE_P = 56, 8

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950); there is no fallback path")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, u64, dp = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64,
                                 ctypes.c_void_p)
        lib.pbpqlp_status_string.restype = ctypes.c_char_p
        lib.pbpqlp_status_string.argtypes = [i32]
        lib.pbpqlp_version.restype = i32
        lib.pbpqlp_default_opts.argtypes = [ctypes.POINTER(Opts)]
        lib.pbpqlp_workspace_size.restype = i32
        lib.pbpqlp_workspace_size.argtypes = [i64, i64, i32, i32, i32, ctypes.POINTER(Opts),
                                              ctypes.POINTER(ctypes.c_size_t)]
        lib.pbpqlp_factor.restype = i32
        lib.pbpqlp_factor.argtypes = [vp, i64, i64, i64, i32, i32, i32, i32, u64, vp, i64, dp, i64,
                                      vp, i64, ctypes.POINTER(Opts), vp, vp]
        lib.pbpqlp_factor_rr.restype = i32
        lib.pbpqlp_factor_rr.argtypes = [vp, i64, i64, i64, i32, i32, i32, i32, u64, vp, i64, dp, i64,
                                         vp, i64, ctypes.POINTER(Opts), ctypes.POINTER(RRStruct), vp, vp]
        lib.pbpqlp_factor_noalloc.restype = i32
        lib.pbpqlp_factor_noalloc.argtypes = lib.pbpqlp_factor.argtypes
        lib.pbpqlp_workspace_size_csr.restype = i32
        lib.pbpqlp_workspace_size_csr.argtypes = [i64, i64, i64, i32, i32, i32, ctypes.POINTER(Opts),
                                                  ctypes.POINTER(ctypes.c_size_t)]
        lib.pbpqlp_factor_csr.restype = i32
        lib.pbpqlp_factor_csr.argtypes = [vp, vp, vp, i64, i64, i64, i32, i32, i32, i32, u64, vp, i64, dp,
                                          i64, vp, i64, ctypes.POINTER(Opts), vp, vp]
        lib.pbpqlp_workspace_size_host.restype = i32
        lib.pbpqlp_workspace_size_host.argtypes = [i64, i64, i64, i32, i32, i32, i64, ctypes.POINTER(Opts),
                                                   ctypes.POINTER(ctypes.c_size_t)]
        lib.pbpqlp_factor_host.restype = i32
        lib.pbpqlp_factor_host.argtypes = [vp, i64, i64, i64, i32, i32, i32, i32, u64, i64, vp, i64, dp,
                                           i64, vp, i64, ctypes.POINTER(Opts), vp, vp]
        lib.pbpqlp_omega.restype = i32
        lib.pbpqlp_omega.argtypes = [i64, i32, u64, i32, vp, i64, vp]
        lib.pbpqlp_matmul.restype = i32
        lib.pbpqlp_matmul.argtypes = [i32, vp, i64, i64, i64, i32, vp, i64, i32, i32,
                                      ctypes.c_double, vp, i64, vp]
        lib.pbpqlp_orth.restype = i32
        lib.pbpqlp_orth.argtypes = [vp, i64, i32, i64, i32, i32, vp, i64, dp, i64, vp, vp]
        lib.pbpqlp_small_qr.restype = i32
        lib.pbpqlp_small_qr.argtypes = [dp, i32, i64, dp, i64, dp, i64, vp, vp]
        lib.pbpqlp_batch_create.restype = i32
        lib.pbpqlp_batch_create.argtypes = [i32, ctypes.POINTER(ProblemStruct), i32,
                                            ctypes.POINTER(Opts), ctypes.POINTER(vp)]
        lib.pbpqlp_batch_run.restype = i32
        lib.pbpqlp_batch_run.argtypes = [vp, vp]
        lib.pbpqlp_batch_set_graph.restype = i32
        lib.pbpqlp_batch_set_graph.argtypes = [vp, i32]
        lib.pbpqlp_batch_stats.restype = i32
        lib.pbpqlp_batch_stats.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_size_t)]
        lib.pbpqlp_batch_problem_plan.restype = i32
        lib.pbpqlp_batch_problem_plan.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.pbpqlp_batch_destroy.restype = None
        lib.pbpqlp_batch_destroy.argtypes = [vp]
        lib.pbpqlp_factor_batched.restype = i32
        lib.pbpqlp_factor_batched.argtypes = [i32, ctypes.POINTER(ProblemStruct), i32,
                                              ctypes.POINTER(Opts), vp]
        f32 = ctypes.c_float
        lib.pbpqlp_model_create.restype = i32
        lib.pbpqlp_model_create.argtypes = [vp, ctypes.POINTER(vp)]
        lib.pbpqlp_model_load.restype = i32
        lib.pbpqlp_model_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
        lib.pbpqlp_model_save.restype = i32
        lib.pbpqlp_model_save.argtypes = [vp, ctypes.c_char_p]
        lib.pbpqlp_model_get_params.restype = i32
        lib.pbpqlp_model_get_params.argtypes = [vp, vp]
        lib.pbpqlp_model_steps.restype = i64
        lib.pbpqlp_model_steps.argtypes = [vp]
        lib.pbpqlp_model_free.restype = None
        lib.pbpqlp_model_free.argtypes = [vp]
        lib.pbpqlp_probe_features.restype = i32
        lib.pbpqlp_probe_features.argtypes = [vp, i64, vp, vp]
        lib.pbpqlp_mlp_forward.restype = i32
        lib.pbpqlp_mlp_forward.argtypes = [vp, vp, i64, i32, vp, i64, vp]
        lib.pbpqlp_mlp_loss_grad.restype = i32
        lib.pbpqlp_mlp_loss_grad.argtypes = [vp, vp, i64, vp, vp, i32, vp, vp, vp]
        lib.pbpqlp_mlp_adam_step.restype = i32
        lib.pbpqlp_mlp_adam_step.argtypes = [vp, f32, vp]
        lib.pbpqlp_mlp_train_step.restype = i32
        lib.pbpqlp_mlp_train_step.argtypes = [vp, vp, i64, vp, vp, i32, f32, vp, vp]
        lib.pbpqlp_factor_sketch.restype = i32
        lib.pbpqlp_factor_sketch.argtypes = [vp, i64, i64, i64, i32, vp, i64, i32, i32, i32, vp, i64,
                                             dp, i64, vp, i64, ctypes.POINTER(Opts), vp, vp]
        lib.pbpqlp_factor_auto.restype = i32
        lib.pbpqlp_factor_auto.argtypes = [vp, vp, i64, i64, i64, i32, i32, u64, i32, ctypes.c_double,
                                           vp, i64, dp, i64, vp, i64, ctypes.POINTER(Opts), vp,
                                           ctypes.POINTER(AutoResult), vp]
        lib.pbpqlp_reconstruct.restype = i32
        lib.pbpqlp_reconstruct.argtypes = [vp, i64, dp, i64, vp, i64, i64, i64, i32, i32, vp, i64, vp]
        lib.pbpqlp_residual.restype = i32
        lib.pbpqlp_residual.argtypes = [vp, i64, vp, i64, dp, i64, vp, i64, i64, i64, i32, i32, vp, vp]
        tp = ctypes.POINTER(TunePlanStruct)
        lib.pbpqlp_tune_factor.restype = i32
        lib.pbpqlp_tune_factor.argtypes = [vp, i64, i64, i64, i32, i32, i32, i32, u64,
                                           ctypes.POINTER(Opts), tp, vp]
        lib.pbpqlp_tune_batch.restype = i32
        lib.pbpqlp_tune_batch.argtypes = [i32, ctypes.POINTER(ProblemStruct), i32, ctypes.POINTER(Opts),
                                          tp, vp]
        lib.pbpqlp_tune_lookup.restype = i32
        lib.pbpqlp_tune_lookup.argtypes = [i64, i64, i32, i32, i32, ctypes.POINTER(Opts), i32, tp]
        lib.pbpqlp_tune_clear.restype = None
        lib.pbpqlp_tune_clear.argtypes = []
        lib.pbpqlp_tune_save.restype = i32
        lib.pbpqlp_tune_save.argtypes = [ctypes.c_char_p]
        lib.pbpqlp_tune_load.restype = i32
        lib.pbpqlp_tune_load.argtypes = [ctypes.c_char_p]
        lib.pbpqlp_trace_enable.argtypes = [i32]
        lib.pbpqlp_trace_reset.argtypes = []
        lib.pbpqlp_trace_count.restype = i32
        lib.pbpqlp_trace_get.restype = i32
        lib.pbpqlp_trace_get.argtypes = [i32, ctypes.c_char_p, i32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)]
        _LIB = lib
    return _LIB


def library():
    """The loaded ctypes handle (loads it on first use)."""
    return _lib()


def _check(status: int, where: str):
    if status != OK:
        raise PbpqlpError(status, where)


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}: use float32 or float64")


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _rowmajor(t: torch.Tensor, name: str) -> torch.Tensor:
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        t = t.contiguous()
    return t


def make_opts(plan="native", split_k: int = 0, fp16_scale_a: float = 1.0,
              gram_wg: int = 0) -> Opts:
    if isinstance(plan, str):
        plan = PLANS[plan]
    o = Opts()
    _lib().pbpqlp_default_opts(ctypes.byref(o))
    o.sketch_prec, o.power_prec, o.proj_prec = (PREC[x] for x in plan)
    o.split_k = split_k
    o.gram_workgroups = gram_wg
    o.fp16_scale_a = fp16_scale_a
    return o


@dataclass
class Info:
    status_flags: int
    n_dependent: int
    l: int
    q: int
    norm_a_fro2: float
    norm_l_fro2: float
    resid_rel_est: float

    @staticmethod
    def from_device(buf: torch.Tensor) -> "Info":
        raw = bytes(buf.cpu().numpy().tobytes())
        s = InfoStruct.from_buffer_copy(raw[:INFO_BYTES])
        return Info(s.status_flags, s.n_dependent, s.l, s.q, s.norm_a_fro2, s.norm_l_fro2,
                    s.resid_rel_est)


def workspace_size(m: int, n: int, k: int, p: int, dtype=torch.float32, plan="native",
                   opts: Opts = None) -> int:
    sz = ctypes.c_size_t(0)
    o = make_opts(plan) if opts is None else opts
    _check(_lib().pbpqlp_workspace_size(m, n, k, p, F64 if dtype == torch.float64 else F32,
                                        ctypes.byref(o), ctypes.byref(sz)), "pbpqlp_workspace_size")
    return int(sz.value)


class Factorizer:
    """Reusable factorization of one problem shape: holds the workspace, the
    outputs and the device info record so repeated calls allocate nothing."""

    def __init__(self, m: int, n: int, k: int, p: int, q: int, dtype=torch.float32,
                 plan="native", device="cuda", split_k: int = 0, fp16_scale_a: float = 1.0,
                 gram_wg: int = 0):
        self.m, self.n, self.k, self.p, self.q = m, n, k, p, q
        self.l = k + p
        self.dtype = dtype
        self.device = torch.device(device)
        self.opts = make_opts(plan, split_k, fp16_scale_a, gram_wg)
        ws = workspace_size(m, n, k, p, dtype, plan, self.opts)
        self.workspace = torch.empty(ws + 256, dtype=torch.uint8, device=self.device)
        self.opts.workspace = self.workspace.data_ptr()
        self.opts.workspace_bytes = self.workspace.numel()
        self.Q = torch.empty((m, self.l), dtype=dtype, device=self.device)
        self.P = torch.empty((n, self.l), dtype=dtype, device=self.device)
        self.L = torch.empty((self.l, self.l), dtype=torch.float64, device=self.device)
        self.info_buf = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=self.device)

    def __call__(self, A: torch.Tensor, seed: int):
        A = _rowmajor(A, "A")
        if A.shape != (self.m, self.n) or A.dtype != self.dtype or A.device != self.device:
            raise ValueError("A does not match this factorizer's shape/dtype/device")
        st = _lib().pbpqlp_factor(
            ctypes.c_void_p(A.data_ptr()), self.m, self.n, A.stride(0), _dt(A), self.k, self.p,
            self.q, ctypes.c_uint64(seed), ctypes.c_void_p(self.Q.data_ptr()), self.l,
            ctypes.c_void_p(self.L.data_ptr()), self.l, ctypes.c_void_p(self.P.data_ptr()),
            self.l, ctypes.byref(self.opts), ctypes.c_void_p(self.info_buf.data_ptr()),
            _stream(self.device))
        _check(st, "pbpqlp_factor")
        return self.Q, self.L, self.P

    def info(self) -> Info:
        return Info.from_device(self.info_buf)


def factor(A: torch.Tensor, k: int, p: int, q: int, seed: int, plan="native", split_k: int = 0,
           fp16_scale_a: float = 1.0,
           gram_wg: int = 0) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor, Info]:
    """PbP-QLP of a device matrix A (m x n, float32/float64): returns
    (Q, L, P, info) with A ~= Q @ L.T @ P.T."""
    A = _rowmajor(A, "A")
    f = Factorizer(A.shape[0], A.shape[1], k, p, q, A.dtype, plan, A.device, split_k, fp16_scale_a,
                   gram_wg)
    Q, L, P = f(A, seed)
    return Q, L, P, f.info()


def factor_rr(A: torch.Tensor, k: int, p: int, q: int, seed: int, orientation: str = "A", plan="native",
              rank_tol: float = None, want_r: bool = True, split_k: int = 0):
    """pbpqlp_factor_rr.  orientation "A": A ~= Q @ L @ P.T (Algorithm 1 as the
    paper states it); "AT": A ~= Q @ L.T @ P.T (pbpqlp_factor); "auto": "A"
    when m >= n.  Returns (Q, L, P, R or None, rank or None, orientation used,
    info); R is the upper-triangular factor of the last QR (R-values on its
    diagonal), rank the number of leading L_ii > rank_tol * L_11."""
    A = _rowmajor(A, "A")
    m, n = A.shape
    l = k + p
    dev = A.device
    Q = torch.empty((m, l), dtype=A.dtype, device=dev)
    P = torch.empty((n, l), dtype=A.dtype, device=dev)
    L = torch.empty((l, l), dtype=torch.float64, device=dev)
    R = torch.empty((l, l), dtype=torch.float64, device=dev) if want_r else None
    rank = torch.full((1,), -1, dtype=torch.int32, device=dev) if rank_tol is not None else None
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
    rr = RRStruct()
    rr.orientation = ORIENT[orientation]
    rr.R = R.data_ptr() if R is not None else None
    rr.ldr = l
    rr.rank_tol = float(rank_tol) if rank_tol is not None else 0.0
    rr.d_rank = rank.data_ptr() if rank is not None else None
    o = make_opts(plan, split_k)
    _check(_lib().pbpqlp_factor_rr(ctypes.c_void_p(A.data_ptr()), m, n, A.stride(0), _dt(A), k, p, q,
                                   ctypes.c_uint64(seed), ctypes.c_void_p(Q.data_ptr()), l,
                                   ctypes.c_void_p(L.data_ptr()), l, ctypes.c_void_p(P.data_ptr()), l,
                                   ctypes.byref(o), ctypes.byref(rr), ctypes.c_void_p(info.data_ptr()),
                                   _stream(dev)), "pbpqlp_factor_rr")
    used = "A" if rr.orientation_used == 1 else "AT"
    return Q, L, P, R, (int(rank.item()) if rank is not None else None), used, Info.from_device(info)


def truncate(Q: torch.Tensor, L: torch.Tensor, P: torch.Tensor, k: int):
    """The rank-k pieces Q[:, :k], L[:k, :k], P[:, :k] as views (no copy)."""
    return Q[:, :k], L[:k, :k], P[:, :k]


def factor_noalloc(A: torch.Tensor, k: int, p: int, q: int, seed: int, plan="native", split_k: int = 0,
                   out=None):
    """pbpqlp_factor_noalloc: the factorization with the library's static
    device scratch as workspace.  ``out`` = (Q, L, P, info_buf) preallocated
    by the caller (then this call allocates nothing); returns (Q, L, P, info)."""
    A = _rowmajor(A, "A")
    m, n = A.shape
    l = k + p
    if out is None:
        out = (torch.empty((m, l), dtype=A.dtype, device=A.device),
               torch.empty((l, l), dtype=torch.float64, device=A.device),
               torch.empty((n, l), dtype=A.dtype, device=A.device),
               torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device))
    Q, L, P, info = out
    o = make_opts(plan, split_k)
    _check(_lib().pbpqlp_factor_noalloc(ctypes.c_void_p(A.data_ptr()), m, n, A.stride(0), _dt(A), k, p, q,
                                        ctypes.c_uint64(seed), ctypes.c_void_p(Q.data_ptr()), Q.stride(0),
                                        ctypes.c_void_p(L.data_ptr()), L.stride(0),
                                        ctypes.c_void_p(P.data_ptr()), P.stride(0), ctypes.byref(o),
                                        ctypes.c_void_p(info.data_ptr()), _stream(A.device)),
           "pbpqlp_factor_noalloc")
    return Q, L, P, info


def factor_host(A: torch.Tensor, k: int, p: int, q: int, seed: int, plan="native", panel_rows: int = 0,
                split_k: int = 0, device="cuda"):
    """pbpqlp_factor_host: A (m x n, float32/float64) stays in host memory
    (a CPU tensor; pinned memory, ``A.pin_memory()``, lets the copies overlap
    the kernels) and is streamed to ``device`` in row panels on every pass.
    Returns (Q, L, P, info) on the device with A ~= Q @ L.T @ P.T."""
    if A.is_cuda:
        raise ValueError("A must be a host (CPU) tensor")
    if A.dim() != 2 or A.stride(1) != 1 or A.stride(0) < A.shape[1]:
        A = A.contiguous()
    m, n = A.shape
    l = k + p
    dev = torch.device(device)
    Q = torch.empty((m, l), dtype=A.dtype, device=dev)
    P = torch.empty((n, l), dtype=A.dtype, device=dev)
    L = torch.empty((l, l), dtype=torch.float64, device=dev)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
    o = make_opts(plan, split_k)
    with torch.cuda.device(dev):
        _check(_lib().pbpqlp_factor_host(ctypes.c_void_p(A.data_ptr()), m, n, A.stride(0), _dt(A), k, p, q,
                                         ctypes.c_uint64(seed), int(panel_rows), ctypes.c_void_p(Q.data_ptr()),
                                         l, ctypes.c_void_p(L.data_ptr()), l, ctypes.c_void_p(P.data_ptr()),
                                         l, ctypes.byref(o), ctypes.c_void_p(info.data_ptr()), _stream(dev)),
               "pbpqlp_factor_host")
    return Q, L, P, Info.from_device(info)


def factor_csr(rowptr: torch.Tensor, colind: torch.Tensor, vals: torch.Tensor, shape, k: int, p: int, q: int,
               seed: int):
    """pbpqlp_factor_csr: A (m x n) in CSR on the device (rowptr int64 m + 1,
    colind int32, vals float32/float64).  Returns (Q, L, P, info) with
    A ~= Q @ L.T @ P.T."""
    m, n = shape
    for t, name in ((rowptr, "rowptr"), (colind, "colind"), (vals, "vals")):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous device tensor")
    if rowptr.dtype != torch.int64 or colind.dtype != torch.int32 or rowptr.numel() != m + 1:
        raise ValueError("rowptr must be int64 of length m + 1 and colind int32")
    nnz = vals.numel()
    if colind.numel() != nnz:
        raise ValueError("colind and vals must have the same length")
    l = k + p
    dev = vals.device
    Q = torch.empty((m, l), dtype=vals.dtype, device=dev)
    P = torch.empty((n, l), dtype=vals.dtype, device=dev)
    L = torch.empty((l, l), dtype=torch.float64, device=dev)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
    o = make_opts("native")
    _check(_lib().pbpqlp_factor_csr(ctypes.c_void_p(rowptr.data_ptr()), ctypes.c_void_p(colind.data_ptr()),
                                    ctypes.c_void_p(vals.data_ptr()), m, n, nnz, _dt(vals), k, p, q,
                                    ctypes.c_uint64(seed), ctypes.c_void_p(Q.data_ptr()), l,
                                    ctypes.c_void_p(L.data_ptr()), l, ctypes.c_void_p(P.data_ptr()), l,
                                    ctypes.byref(o), ctypes.c_void_p(info.data_ptr()), _stream(dev)),
           "pbpqlp_factor_csr")
    return Q, L, P, Info.from_device(info)


def workspace_size_host(m: int, n: int, k: int, p: int, dtype=torch.float32, plan="native",
                        panel_rows: int = 0, lda: int = None) -> int:
    sz = ctypes.c_size_t(0)
    o = make_opts(plan)
    _check(_lib().pbpqlp_workspace_size_host(m, n, n if lda is None else lda, k, p,
                                             F64 if dtype == torch.float64 else F32, int(panel_rows),
                                             ctypes.byref(o), ctypes.byref(sz)), "pbpqlp_workspace_size_host")
    return int(sz.value)


def factor_sketch(A: torch.Tensor, Omega: torch.Tensor, k: int, p: int, q: int, plan="native"):
    """pbpqlp_factor_sketch: the factorization with a given sketch matrix
    Omega (n x l, the dtype of A).  Returns (Q, L, P, info)."""
    A = _rowmajor(A, "A")
    Omega = _rowmajor(Omega, "Omega")
    m, n = A.shape
    l = k + p
    if Omega.shape != (n, l) or Omega.dtype != A.dtype:
        raise ValueError("Omega must be n x (k + p) in the dtype of A")
    Q = torch.empty((m, l), dtype=A.dtype, device=A.device)
    P = torch.empty((n, l), dtype=A.dtype, device=A.device)
    L = torch.empty((l, l), dtype=torch.float64, device=A.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    o = make_opts(plan)
    _check(_lib().pbpqlp_factor_sketch(ctypes.c_void_p(A.data_ptr()), m, n, A.stride(0), _dt(A),
                                       ctypes.c_void_p(Omega.data_ptr()), Omega.stride(0), k, p, q,
                                       ctypes.c_void_p(Q.data_ptr()), l, ctypes.c_void_p(L.data_ptr()), l,
                                       ctypes.c_void_p(P.data_ptr()), l, ctypes.byref(o),
                                       ctypes.c_void_p(info.data_ptr()), _stream(A.device)),
           "pbpqlp_factor_sketch")
    return Q, L, P, Info.from_device(info)


def reconstruct(Q: torch.Tensor, L: torch.Tensor, P: torch.Tensor) -> torch.Tensor:
    """A_hat = Q L^T P^T on the device (pbpqlp_reconstruct)."""
    Q, P = _rowmajor(Q, "Q"), _rowmajor(P, "P")
    L = L.contiguous()
    m, l = Q.shape
    n = P.shape[0]
    Ah = torch.empty((m, n), dtype=Q.dtype, device=Q.device)
    _check(_lib().pbpqlp_reconstruct(ctypes.c_void_p(Q.data_ptr()), Q.stride(0), ctypes.c_void_p(L.data_ptr()),
                                     L.stride(0), ctypes.c_void_p(P.data_ptr()), P.stride(0), m, n, l, _dt(Q),
                                     ctypes.c_void_p(Ah.data_ptr()), n, _stream(Q.device)), "pbpqlp_reconstruct")
    return Ah


def residual(A: torch.Tensor, Q: torch.Tensor, L: torch.Tensor, P: torch.Tensor) -> float:
    """Explicit ||A - Q L^T P^T||_F / ||A||_F on the device (pbpqlp_residual)."""
    A, Q, P = _rowmajor(A, "A"), _rowmajor(Q, "Q"), _rowmajor(P, "P")
    L = L.contiguous()
    m, n = A.shape
    r = torch.empty(1, dtype=torch.float64, device=A.device)
    _check(_lib().pbpqlp_residual(ctypes.c_void_p(A.data_ptr()), A.stride(0), ctypes.c_void_p(Q.data_ptr()),
                                  Q.stride(0), ctypes.c_void_p(L.data_ptr()), L.stride(0),
                                  ctypes.c_void_p(P.data_ptr()), P.stride(0), m, n, Q.shape[1], _dt(A),
                                  ctypes.c_void_p(r.data_ptr()), _stream(A.device)), "pbpqlp_residual")
    return float(r.item())


def omega(n: int, l: int, seed: int, dtype=torch.float64, device="cuda") -> torch.Tensor:
    out = torch.empty((n, l), dtype=dtype, device=device)
    _check(_lib().pbpqlp_omega(n, l, ctypes.c_uint64(seed), _dt(out), ctypes.c_void_p(out.data_ptr()),
                               l, _stream(out.device)), "pbpqlp_omega")
    return out


def matmul(A: torch.Tensor, X: torch.Tensor, trans: bool = False, prec: str = "native",
           fp16_scale_a: float = 1.0) -> torch.Tensor:
    """Y = A @ X (trans=False) or A.T @ X through the streaming kernels."""
    A = _rowmajor(A, "A")
    X = _rowmajor(X, "X")
    m, n = A.shape
    rows = n if trans else m
    if X.shape[0] != (m if trans else n) or X.dtype != A.dtype:
        raise ValueError("X shape/dtype mismatch")
    l = X.shape[1]
    Y = torch.empty((rows, l), dtype=A.dtype, device=A.device)
    _check(_lib().pbpqlp_matmul(1 if trans else 0, ctypes.c_void_p(A.data_ptr()), m, n, A.stride(0),
                                _dt(A), ctypes.c_void_p(X.data_ptr()), X.stride(0), l, PREC[prec],
                                fp16_scale_a, ctypes.c_void_p(Y.data_ptr()), l,
                                _stream(A.device)), "pbpqlp_matmul")
    return Y


def orth(Y: torch.Tensor, passes: int = 2, want_r: bool = True):
    """Y = Q R (CholeskyQR sweeps with FP64 Grams); returns (Q, R or None, Info)."""
    Y = _rowmajor(Y, "Y")
    rows, l = Y.shape
    Q = torch.empty_like(Y)
    R = torch.empty((l, l), dtype=torch.float64, device=Y.device) if want_r else None
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=Y.device)
    _check(_lib().pbpqlp_orth(ctypes.c_void_p(Y.data_ptr()), rows, l, Y.stride(0), _dt(Y), passes,
                              ctypes.c_void_p(Q.data_ptr()), l,
                              ctypes.c_void_p(R.data_ptr() if R is not None else 0), l,
                              ctypes.c_void_p(info.data_ptr()), _stream(Y.device)), "pbpqlp_orth")
    return Q, R, Info.from_device(info)


def small_qr(R: torch.Tensor):
    """R^T = Qt L^T for an upper-triangular FP64 R (l x l); returns (Qt, L)."""
    R = _rowmajor(R, "R")
    if R.dtype != torch.float64:
        raise TypeError("R must be float64")
    l = R.shape[0]
    Qt = torch.empty((l, l), dtype=torch.float64, device=R.device)
    L = torch.empty((l, l), dtype=torch.float64, device=R.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=R.device)
    _check(_lib().pbpqlp_small_qr(ctypes.c_void_p(R.data_ptr()), l, R.stride(0),
                                  ctypes.c_void_p(Qt.data_ptr()), l, ctypes.c_void_p(L.data_ptr()),
                                  l, ctypes.c_void_p(info.data_ptr()), _stream(R.device)),
           "pbpqlp_small_qr")
    return Qt, L


def trace_enable(level: int = 1) -> None:
    """Record HIP events around the streaming products (level 1) or every
    hot-path kernel (level 2) of later calls; 0 switches tracing off."""
    _lib().pbpqlp_trace_enable(int(level))


def trace_reset() -> None:
    _lib().pbpqlp_trace_reset()


def trace_records():
    """[(name, algorithmic bytes, flops, ms), ...] for the recorded kernels.
    Call after the stream has finished the traced work."""
    lib = _lib()
    out = []
    buf = ctypes.create_string_buffer(64)
    b, f, ms = ctypes.c_double(), ctypes.c_double(), ctypes.c_float()
    for i in range(lib.pbpqlp_trace_count()):
        _check(lib.pbpqlp_trace_get(i, buf, 64, ctypes.byref(b), ctypes.byref(f), ctypes.byref(ms)),
               "pbpqlp_trace_get")
        out.append((buf.value.decode(), b.value, f.value, float(ms.value)))
    return out


class Batch:
    """A plan for factorizing many independent matrices (pbpqlp_batch_create).

    ``mats`` is a list of 2-D device tensors of one dtype; ``ks``, ``ps``, ``qs``
    and ``seeds`` give each problem's k, p, q and seed.  The plan allocates the
    outputs (``Q[i]``, ``L[i]``, ``P[i]``) and one result record per problem;
    ``run()`` factorizes all of them with one graph launch on the current stream.
    The matrices must stay alive and in place while the plan is used.
    """

    def __init__(self, mats, ks, ps, qs, seeds, plan: str = "native", use_graph: bool = True,
                 gram_wg: int = 0):
        if not mats:
            raise ValueError("empty batch")
        dtype = mats[0].dtype
        self.device = mats[0].device
        self.mats = [_rowmajor(a, "A") for a in mats]
        if any(a.dtype != dtype for a in self.mats):
            raise TypeError("all matrices of a batch must have one dtype")
        cnt = len(self.mats)
        self.count = cnt
        self.ls = [int(k) + int(p) for k, p in zip(ks, ps)]
        self.Q = [torch.empty((a.shape[0], l), dtype=dtype, device=self.device) for a, l in zip(self.mats, self.ls)]
        self.P = [torch.empty((a.shape[1], l), dtype=dtype, device=self.device) for a, l in zip(self.mats, self.ls)]
        self.L = [torch.empty((l, l), dtype=torch.float64, device=self.device) for l in self.ls]
        self.info_buf = torch.zeros((cnt, INFO_BYTES), dtype=torch.uint8, device=self.device)
        probs = (ProblemStruct * cnt)()
        for i, a in enumerate(self.mats):
            pr = probs[i]
            pr.A = a.data_ptr(); pr.m = a.shape[0]; pr.n = a.shape[1]; pr.lda = a.stride(0)
            pr.k = int(ks[i]); pr.p = int(ps[i]); pr.q = int(qs[i]); pr.seed = int(seeds[i])
            pr.Q = self.Q[i].data_ptr(); pr.ldq = self.ls[i]
            pr.L = self.L[i].data_ptr(); pr.ldl = self.ls[i]
            pr.P = self.P[i].data_ptr(); pr.ldp = self.ls[i]
            pr.info = self.info_buf[i].data_ptr()
        opts = make_opts(plan, gram_wg=gram_wg)
        self._probs, self._opts = probs, opts
        handle = ctypes.c_void_p()
        _check(_lib().pbpqlp_batch_create(cnt, probs, _dt(self.mats[0]), ctypes.byref(opts),
                                          ctypes.byref(handle)), "pbpqlp_batch_create")
        self._h = handle
        if not use_graph:
            _check(_lib().pbpqlp_batch_set_graph(self._h, 0), "pbpqlp_batch_set_graph")

    def run(self):
        _check(_lib().pbpqlp_batch_run(self._h, _stream(self.device)), "pbpqlp_batch_run")
        return self

    def use_graph(self, flag: bool):
        _check(_lib().pbpqlp_batch_set_graph(self._h, 1 if flag else 0), "pbpqlp_batch_set_graph")

    def stats(self):
        n = ctypes.c_int(0)
        ws = ctypes.c_size_t(0)
        _check(_lib().pbpqlp_batch_stats(self._h, ctypes.byref(n), ctypes.byref(ws)), "pbpqlp_batch_stats")
        return {"launches": n.value, "workspace_bytes": ws.value}

    def tune(self) -> dict:
        """pbpqlp_tune_batch over this batch's problems (their outputs are
        overwritten); later batches of the same class with an automatic Gram
        target use the choice.  This plan keeps its own."""
        t = TunePlanStruct()
        _check(_lib().pbpqlp_tune_batch(self.count, self._probs, _dt(self.mats[0]), ctypes.byref(self._opts),
                                        ctypes.byref(t), _stream(self.device)), "pbpqlp_tune_batch")
        return {"split_k": t.split_k, "gram_wg": t.gram_workgroups, "ms": t.ms}

    def problem_plan(self, i: int):
        """(split_k, gram_wg) the plan uses for problem i: factor() with these
        options reproduces that problem's results bit for bit."""
        sk = ctypes.c_int(0)
        gw = ctypes.c_int(0)
        _check(_lib().pbpqlp_batch_problem_plan(self._h, i, ctypes.byref(sk), ctypes.byref(gw)),
               "pbpqlp_batch_problem_plan")
        return sk.value, gw.value

    def info(self, i: int) -> "Info":
        return Info.from_device(self.info_buf[i])

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            _lib().pbpqlp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Learned choice of q and k
# ---------------------------------------------------------------------------
def _f32dev(x, device, name):
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(np.asarray(x, dtype=np.float32))
    x = x.to(device=device, dtype=torch.float32)
    if x.dim() != 2 or x.shape[1] != MLP_IN:
        raise ValueError(f"{name} must be batch x {MLP_IN}")
    return x.contiguous()


class Model:
    """The q/k network on the device (pbpqlp_model): parameters, gradient and
    Adam state.  ``params`` is a host array of 25606 floats (None = zeros)."""

    def __init__(self, params=None, device="cuda", _handle=None):
        self.device = torch.device(device)
        if _handle is not None:
            self._h = _handle
            return
        h = ctypes.c_void_p()
        buf = None
        if params is not None:
            buf = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
            if buf.shape != (MLP_PARAMS,):
                raise ValueError(f"expected {MLP_PARAMS} parameters")
        _check(_lib().pbpqlp_model_create(None if buf is None else buf.ctypes.data, ctypes.byref(h)),
               "pbpqlp_model_create")
        self._h = h

    @classmethod
    def load(cls, path, device="cuda"):
        h = ctypes.c_void_p()
        _check(_lib().pbpqlp_model_load(os.fsencode(path), ctypes.byref(h)), "pbpqlp_model_load")
        return cls(device=device, _handle=h)

    def save(self, path):
        _check(_lib().pbpqlp_model_save(self._h, os.fsencode(path)), "pbpqlp_model_save")

    def params(self) -> np.ndarray:
        out = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(_lib().pbpqlp_model_get_params(self._h, out.ctypes.data), "pbpqlp_model_get_params")
        return out

    @property
    def steps(self) -> int:
        return int(_lib().pbpqlp_model_steps(self._h))

    def forward(self, X) -> torch.Tensor:
        X = _f32dev(X, self.device, "X")
        Z = torch.empty((X.shape[0], MLP_OUT), dtype=torch.float32, device=self.device)
        _check(_lib().pbpqlp_mlp_forward(self._h, ctypes.c_void_p(X.data_ptr()), MLP_IN, X.shape[0],
                                         ctypes.c_void_p(Z.data_ptr()), MLP_OUT, _stream(self.device)),
               "pbpqlp_mlp_forward")
        return Z

    def _labels(self, X, q, logk):
        X = _f32dev(X, self.device, "X")
        q = torch.as_tensor(q).to(device=self.device, dtype=torch.int32).contiguous()
        logk = torch.as_tensor(logk).to(device=self.device, dtype=torch.float32).contiguous()
        if q.shape != (X.shape[0],) or logk.shape != (X.shape[0],):
            raise ValueError("one label per row")
        return X, q, logk

    def loss_grad(self, X, q, logk):
        """(loss, gradient) of a batch; the gradient also stays in the model
        for adam_step()."""
        X, q, logk = self._labels(X, q, logk)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=self.device)
        _check(_lib().pbpqlp_mlp_loss_grad(self._h, ctypes.c_void_p(X.data_ptr()), MLP_IN,
                                           ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(logk.data_ptr()),
                                           X.shape[0], ctypes.c_void_p(loss.data_ptr()),
                                           ctypes.c_void_p(g.data_ptr()), _stream(self.device)),
               "pbpqlp_mlp_loss_grad")
        return loss, g

    def adam_step(self, lr: float):
        _check(_lib().pbpqlp_mlp_adam_step(self._h, float(lr), _stream(self.device)), "pbpqlp_mlp_adam_step")

    def train_step(self, X, q, logk, lr: float) -> torch.Tensor:
        X, q, logk = self._labels(X, q, logk)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(_lib().pbpqlp_mlp_train_step(self._h, ctypes.c_void_p(X.data_ptr()), MLP_IN,
                                            ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(logk.data_ptr()),
                                            X.shape[0], float(lr), ctypes.c_void_p(loss.data_ptr()),
                                            _stream(self.device)), "pbpqlp_mlp_train_step")
        return loss

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            _lib().pbpqlp_model_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_features(L: torch.Tensor) -> torch.Tensor:
    """Features (64 floats) from the diagonal of a probe's L (64 x 64 FP64)."""
    if L.dtype != torch.float64 or L.dim() != 2 or L.shape[0] < MLP_IN or L.shape[1] < MLP_IN:
        raise ValueError("L must be an FP64 matrix of at least 64 x 64")
    if L.stride(1) != 1:
        L = L.contiguous()
    f = torch.empty(MLP_IN, dtype=torch.float32, device=L.device)
    _check(_lib().pbpqlp_probe_features(ctypes.c_void_p(L.data_ptr()), L.stride(0),
                                        ctypes.c_void_p(f.data_ptr()), _stream(L.device)),
           "pbpqlp_probe_features")
    return f


def probe(A: torch.Tensor, seed: int, plan="native"):
    """The q = 0, l = 64 probe factorization and its features: (f, L, info)."""
    Q, L, P, info = factor(A, PROBE_K, PROBE_P, 0, seed, plan=plan)
    return probe_features(L), L, info


def factor_auto(model: Model, A: torch.Tensor, p: int, seed: int, k_max: int, tau: float,
                plan="native"):
    """pbpqlp_factor_auto: returns (Q, L, P, result dict, info); Q, L, P are
    cut to the l = k_used + p columns the chosen run produced."""
    A = _rowmajor(A, "A")
    m, n = A.shape
    lmax = k_max + p
    Q = torch.empty((m, lmax), dtype=A.dtype, device=A.device)
    P = torch.empty((n, lmax), dtype=A.dtype, device=A.device)
    L = torch.empty((lmax, lmax), dtype=torch.float64, device=A.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    res = AutoResult()
    o = make_opts(plan)
    _check(_lib().pbpqlp_factor_auto(model._h, ctypes.c_void_p(A.data_ptr()), m, n, A.stride(0), _dt(A),
                                     p, ctypes.c_uint64(seed), k_max, float(tau),
                                     ctypes.c_void_p(Q.data_ptr()), lmax, ctypes.c_void_p(L.data_ptr()),
                                     lmax, ctypes.c_void_p(P.data_ptr()), lmax, ctypes.byref(o),
                                     ctypes.c_void_p(info.data_ptr()), ctypes.byref(res),
                                     _stream(A.device)), "pbpqlp_factor_auto")
    l = res.k_used + p
    r = {f: getattr(res, f) for f, _ in AutoResult._fields_}
    return Q[:, :l], L[:l, :l], P[:, :l], r, Info.from_device(info)


# ---------------------------------------------------------------------------
# Autotuning
# ---------------------------------------------------------------------------
def tune_factor(A: torch.Tensor, k: int, p: int, q: int, seed: int, plan="native") -> dict:
    """pbpqlp_tune_factor: time the candidate plans on A and cache the fastest
    for A's shape class; returns {split_k, gram_wg, ms}."""
    A = _rowmajor(A, "A")
    t = TunePlanStruct()
    o = make_opts(plan)
    _check(_lib().pbpqlp_tune_factor(ctypes.c_void_p(A.data_ptr()), A.shape[0], A.shape[1], A.stride(0),
                                     _dt(A), k, p, q, ctypes.c_uint64(seed), ctypes.byref(o),
                                     ctypes.byref(t), _stream(A.device)), "pbpqlp_tune_factor")
    return {"split_k": t.split_k, "gram_wg": t.gram_workgroups, "ms": t.ms}


def tune_lookup(m: int, n: int, k: int, p: int, dtype=torch.float32, plan="native", batched=False):
    """The cached plan of a shape class, or None."""
    t = TunePlanStruct()
    o = make_opts(plan)
    st = _lib().pbpqlp_tune_lookup(m, n, k, p, F64 if dtype == torch.float64 else F32, ctypes.byref(o),
                                   1 if batched else 0, ctypes.byref(t))
    if st != OK:
        return None
    return {"split_k": t.split_k, "gram_wg": t.gram_workgroups, "ms": t.ms}


def tune_clear():
    _lib().pbpqlp_tune_clear()


def tune_save(path):
    _check(_lib().pbpqlp_tune_save(os.fsencode(str(path))), "pbpqlp_tune_save")


def tune_load(path):
    _check(_lib().pbpqlp_tune_load(os.fsencode(str(path))), "pbpqlp_tune_load")
