"""MI355X SAQ encoder: Python binding of libsaq.so (include/saq.h).

Argument marshalling only: every step of the encode and estimate paths runs in
the library's HIP kernels; PyTorch supplies device memory and streams.  If the
library is missing this module raises instead of falling back to anything.

SAQ: "Pushing the Limits of Vector Quantization through Code Adjustment and
Dimension Segmentation" (SIGMOD'26, arXiv 2509.12086).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsaq.so")

LAYOUT_ROWS = 0
LAYOUT_DIMS = 1
LAYOUT_TILES = 2

_STATUS = {0: "SAQ_OK", 1: "SAQ_EINVAL", 2: "SAQ_ENOMEM", 3: "SAQ_EDEVICE",
           4: "SAQ_EUNSUPPORTED", 5: "SAQ_EIO"}


class SaqError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("bits_per_dim", ctypes.c_double), ("granularity", ctypes.c_int32),
                ("max_bits", ctypes.c_int32), ("max_width", ctypes.c_int32),
                ("seg_eps", ctypes.c_double), ("rotate_segments", ctypes.c_int32),
                ("fit_sample", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("projection_accumulation", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("D_kept", ctypes.c_int32), ("n_seg", ctypes.c_int32),
                ("n_kept", ctypes.c_int32), ("code_bytes", ctypes.c_int64),
                ("n_factors", ctypes.c_int32), ("max_kept_width", ctypes.c_int32),
                ("max_kept_bits", ctypes.c_int32), ("model_error", ctypes.c_double),
                ("min_error", ctypes.c_double), ("quota_bits", ctypes.c_int64),
                ("used_bits", ctypes.c_int64), ("projection_fp64_totals", ctypes.c_int32)]


_lib = None
EXPORTS = ("saq_default_params", "saq_fit_plan", "saq_plan_from_basis", "saq_plan_from_parts",
           "saq_plan_info_get", "saq_plan_segments", "saq_plan_arrays", "saq_plan_save",
           "saq_plan_load", "saq_plan_free", "saq_plan_device_bytes", "saq_plan_upload",
           "saq_encode_workspace_bytes", "saq_encode", "saq_project", "saq_quantize",
           "saq_estimate_workspace_bytes", "saq_estimate_dist", "saq_estimate_dist_prefix",
           "saq_estimate_multistage", "saq_covariance_workspace_bytes", "saq_covariance",
           "saq_encode_ref", "saq_estimate_dist_ref", "saq_estimate_multistage_ref",
           "saq_fit_workspace_bytes", "saq_fit_plan_device",
           "saq_sym_eigen_workspace_bytes", "saq_sym_eigen_device",
           "saq_encode_batched_workspace_bytes",
           "saq_encode_batched", "saq_encode_noalloc", "saq_last_error", "saq_version")

# saq_encode_noalloc's fixed device array (SAQ_NOALLOC_SCRATCH_BYTES in saq.h)
NOALLOC_SCRATCH_BYTES = 64 << 20

BATCH_MAX = 16


class _BatchItem(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("X_dev", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("codes_dev", ctypes.c_void_p), ("factors_dev", ctypes.c_void_p)]


class _Tuning(ctypes.Structure):
    _fields_ = [("quant_waves", ctypes.c_int32), ("gemm_xcd_order", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


BATCH_FUSED = 0      # one persistent fused launch (SAQ_BATCH_FUSED)
BATCH_GROUPED = 1    # two grouped launches (SAQ_BATCH_GROUPED)


def lib() -> ctypes.CDLL:
    """Load libsaq.so (built in-tree by ``paper_2509_12086_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2509_12086_amd.build` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "saq_default_params": (None, [ctypes.POINTER(_Params)]),
        "saq_fit_plan": (i32, [P, i64, i32, ctypes.POINTER(_Params), pp]),
        "saq_plan_from_basis": (i32, [P, P, P, i32, ctypes.POINTER(_Params), pp]),
        "saq_plan_from_parts": (i32, [i32, i32, P, P, P, P, P, pp]),
        "saq_plan_info_get": (i32, [P, ctypes.POINTER(_Info)]),
        "saq_plan_segments": (i32, [P, P, P]),
        "saq_plan_arrays": (i32, [P, P, P, P]),
        "saq_plan_save": (i32, [P, ctypes.c_char_p]),
        "saq_plan_load": (i32, [ctypes.c_char_p, pp]),
        "saq_plan_free": (None, [P]),
        "saq_plan_device_bytes": (i64, [P]),
        "saq_plan_upload": (i32, [P, P, P]),
        "saq_encode_workspace_bytes": (i64, [P, i64]),
        "saq_encode": (i32, [P, P, i64, i32, P, P, P, i64, P]),
        "saq_project": (i32, [P, P, i64, P, i64, i32, P, P]),
        "saq_quantize": (i32, [P, P, i64, i32, i64, P, i32, P, P, P]),
        "saq_estimate_workspace_bytes": (i64, [P, i32]),
        "saq_estimate_dist": (i32, [P, P, i32, P, P, i64, P, P, i64, P]),
        "saq_estimate_dist_prefix": (i32, [P, P, i32, P, P, i64, i32, P, P, i64, P]),
        "saq_estimate_multistage": (i32, [P, P, i32, P, P, i64, P, ctypes.c_float, P, P, P, i64,
                                          P]),
        "saq_covariance_workspace_bytes": (i64, [i64, i32, i64]),
        "saq_encode_ref": (i32, [P, P, i64, P, i32, P, i32, P, P, P, i64, P]),
        "saq_estimate_dist_ref": (i32, [P, P, i32, P, P, P, i64, P, P, i64, P]),
        "saq_estimate_multistage_ref": (i32, [P, P, i32, P, P, P, i64, P, ctypes.c_float, P, P,
                                              P, i64, P]),
        "saq_covariance": (i32, [P, i64, i32, i64, P, P, P, i64, P]),
        "saq_fit_workspace_bytes": (i64, [i64, i32, P]),
        "saq_fit_plan_device": (i32, [P, i64, i32, P, P, i64, P, P]),
        "saq_sym_eigen_workspace_bytes": (i64, [i32]),
        "saq_sym_eigen_device": (i32, [P, i32, P, P, P, i64, P]),
        "saq_encode_batched_workspace_bytes": (i64, [P, i32, P]),
        "saq_encode_batched": (i32, [P, i32, i32, P, P, i64, P]),
        "saq_encode_noalloc": (i32, [P, P, i64, i32, P, P, P]),
        "saq_last_error": (ctypes.c_char_p, []),
        "saq_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise SaqError(rc, lib().saq_last_error().decode())


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclasses.dataclass
class PlanParams:
    """Plan-search parameters (Sections 4.1-4.2); see saq_plan_params."""
    bits_per_dim: float = 4.0
    granularity: int = 16
    max_bits: int = 9
    max_width: int = 512
    seg_eps: float = 1e-3
    rotate_segments: bool = True
    fit_sample: int = 65536
    seed: int = 1
    projection_accumulation: int = 0     # 0 auto, 1 FP32, 2 FP64 k-tile totals

    def _c(self) -> _Params:
        return _Params(float(self.bits_per_dim), int(self.granularity), int(self.max_bits),
                       int(self.max_width), float(self.seg_eps), int(bool(self.rotate_segments)),
                       int(self.fit_sample), int(self.seed), int(self.projection_accumulation))


def _torch():
    import torch
    return torch


def _dev_ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_ptr(stream, device=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A quantization plan: segments and bits, projection matrix M (FP32,
    kept dims x D), reference vector c and per-dim variances."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)
        self._dev = None                 # torch uint8 tensor holding the device copy
        info = _Info()
        _check(lib().saq_plan_info_get(self._h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _Info._fields_}
        w = np.zeros(self.info["n_seg"], np.int32)
        b = np.zeros(self.info["n_seg"], np.int32)
        _check(lib().saq_plan_segments(self._h, _np_ptr(w), _np_ptr(b)))
        self.widths, self.bits = w.tolist(), b.tolist()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.saq_plan_free(h)
            self._h = None

    # -- construction ------------------------------------------------------
    @classmethod
    def fit(cls, X: np.ndarray, params: Optional[PlanParams] = None) -> "Plan":
        X = np.ascontiguousarray(X, np.float32)
        p = (params or PlanParams())._c()
        h = ctypes.c_void_p()
        _check(lib().saq_fit_plan(_np_ptr(X), X.shape[0], X.shape[1], ctypes.byref(p),
                                  ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def fit_device(cls, X, params: Optional[PlanParams] = None, workspace=None,
                   stream=None) -> "Plan":
        """saq_fit_plan_device: the fit with the rows on the device (CUDA
        float32 [n, D]); mean and covariance on the GPU, the rest on the host."""
        torch = _torch()
        _require_cuda_f32(X, "X")
        n, D = X.shape
        p = (params or PlanParams())._c()
        need = int(lib().saq_fit_workspace_bytes(n, D, ctypes.byref(p)))
        if need < 0:
            raise ValueError("bad fit sizes")
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=X.device)
        h = ctypes.c_void_p()
        _check(lib().saq_fit_plan_device(_dev_ptr(X), n, D, ctypes.byref(p), _dev_ptr(workspace),
                                         workspace.numel() * workspace.element_size(),
                                         _stream_ptr(stream, X.device), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def from_basis(cls, mean, eigvecs, eigvals, params: Optional[PlanParams] = None) -> "Plan":
        mean = np.ascontiguousarray(mean, np.float64)
        V = np.ascontiguousarray(eigvecs, np.float64)
        lam = np.ascontiguousarray(eigvals, np.float64)
        p = (params or PlanParams())._c()
        h = ctypes.c_void_p()
        _check(lib().saq_plan_from_basis(_np_ptr(mean), _np_ptr(V), _np_ptr(lam), mean.size,
                                         ctypes.byref(p), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def from_parts(cls, widths: Sequence[int], bits: Sequence[int], M: np.ndarray, c: np.ndarray,
                   variances: Optional[np.ndarray] = None) -> "Plan":
        w = np.ascontiguousarray(widths, np.int32)
        b = np.ascontiguousarray(bits, np.int32)
        M = np.ascontiguousarray(M, np.float32)
        c = np.ascontiguousarray(c, np.float32)
        var = None if variances is None else np.ascontiguousarray(variances, np.float64)
        h = ctypes.c_void_p()
        _check(lib().saq_plan_from_parts(c.size, w.size, _np_ptr(w), _np_ptr(b),
                                         _np_ptr(M) if M.size else None, _np_ptr(c),
                                         _np_ptr(var), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def load(cls, path: str) -> "Plan":
        h = ctypes.c_void_p()
        _check(lib().saq_plan_load(os.fsencode(path), ctypes.byref(h)))
        return cls(h.value)

    def save(self, path: str) -> None:
        _check(lib().saq_plan_save(self._h, os.fsencode(path)))

    # -- data ----------------------------------------------------------------
    @property
    def D(self) -> int:
        return self.info["D"]

    @property
    def D_kept(self) -> int:
        return self.info["D_kept"]

    @property
    def code_bytes(self) -> int:
        return self.info["code_bytes"]

    @property
    def n_factors(self) -> int:
        return self.info["n_factors"]

    @property
    def kept_widths(self):
        return [w for w, b in zip(self.widths, self.bits) if b > 0]

    @property
    def kept_bits(self):
        return [b for b in self.bits if b > 0]

    def arrays(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        M = np.zeros((self.D_kept, self.D), np.float32)
        c = np.zeros(self.D, np.float32)
        var = np.zeros(self.D, np.float64)
        _check(lib().saq_plan_arrays(self._h, _np_ptr(M) if M.size else None, _np_ptr(c),
                                     _np_ptr(var)))
        return M, c, var

    # -- device --------------------------------------------------------------
    def device_bytes(self) -> int:
        return int(lib().saq_plan_device_bytes(self._h))

    def upload(self, device=None, stream=None) -> "Plan":
        torch = _torch()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        buf = torch.empty(self.device_bytes() + 256, dtype=torch.uint8, device=dev)
        off = (-buf.data_ptr()) % 256
        with torch.cuda.device(dev):
            _check(lib().saq_plan_upload(self._h, ctypes.c_void_p(buf.data_ptr() + off),
                                         _stream_ptr(stream, dev)))
        self._dev = buf
        return self

    def encode_workspace_bytes(self, n: int) -> int:
        return int(lib().saq_encode_workspace_bytes(self._h, n))

    def estimate_workspace_bytes(self, nq: int) -> int:
        return int(lib().saq_estimate_workspace_bytes(self._h, nq))


def _require_cuda_f32(t, name, cols=None, ndim=2):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32):
        raise TypeError(f"{name} must be a CUDA float32 tensor")
    if t.dim() != ndim or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {ndim}-D tensor")
    if cols is not None and t.shape[1] != cols:
        raise ValueError(f"{name} has {t.shape[1]} columns, expected {cols}")


def _alloc_out(plan: Plan, n: int, device, codes=None, factors=None):
    torch = _torch()
    if codes is None:
        codes = torch.empty((n, plan.code_bytes), dtype=torch.uint8, device=device)
    if factors is None:
        factors = torch.empty((n, plan.n_factors), dtype=torch.float32, device=device)
    if codes.shape != (n, plan.code_bytes) or codes.dtype != torch.uint8 or not codes.is_contiguous():
        raise ValueError("codes must be a contiguous uint8 tensor [n, code_bytes]")
    if factors.shape != (n, plan.n_factors) or factors.dtype != torch.float32 or not factors.is_contiguous():
        raise ValueError("factors must be a contiguous float32 tensor [n, n_factors]")
    return codes, factors


def encode(plan: Plan, X, rounds: int = 4, codes=None, factors=None, workspace=None, stream=None,
           refs=None, ref_ids=None):
    """saq_encode: returns (codes uint8 [n, code_bytes], factors f32 [n, n_factors]).
    With refs (CUDA float32 [K, D]) and ref_ids (CUDA int32 [n]),
    saq_encode_ref: record i is encoded against refs[ref_ids[i]]."""
    torch = _torch()
    _require_cuda_f32(X, "X", plan.D)
    n = X.shape[0]
    codes, factors = _alloc_out(plan, n, X.device, codes, factors)
    need = plan.encode_workspace_bytes(n)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=X.device)
    if refs is None:
        _check(lib().saq_encode(plan._h, _dev_ptr(X), n, rounds, _dev_ptr(codes), _dev_ptr(factors),
                                _dev_ptr(workspace), workspace.numel() * workspace.element_size(),
                                _stream_ptr(stream, X.device)))
        return codes, factors
    _require_cuda_f32(refs, "refs", plan.D)
    if not (isinstance(ref_ids, torch.Tensor) and ref_ids.is_cuda and ref_ids.dtype == torch.int32
            and ref_ids.shape == (n,) and ref_ids.is_contiguous()):
        raise ValueError("ref_ids must be a contiguous CUDA int32 tensor [n]")
    _check(lib().saq_encode_ref(plan._h, _dev_ptr(X), n, _dev_ptr(refs), refs.shape[0],
                                _dev_ptr(ref_ids), rounds, _dev_ptr(codes), _dev_ptr(factors),
                                _dev_ptr(workspace), workspace.numel() * workspace.element_size(),
                                _stream_ptr(stream, X.device)))
    return codes, factors


def encode_noalloc(plan: Plan, X, rounds: int = 4, codes=None, factors=None, stream=None):
    """saq_encode_noalloc: the encode with its workspace in the library's
    fixed device array (no device allocation in the call; n is limited to
    what NOALLOC_SCRATCH_BYTES holds for the plan).  Returns (codes, factors);
    outputs are allocated here only when not given."""
    _require_cuda_f32(X, "X", plan.D)
    n = X.shape[0]
    codes, factors = _alloc_out(plan, n, X.device, codes, factors)
    _check(lib().saq_encode_noalloc(plan._h, _dev_ptr(X), n, rounds, _dev_ptr(codes),
                                    _dev_ptr(factors), _stream_ptr(stream, X.device)))
    return codes, factors


def _require_ref(plan: Plan, ref, Q):
    _require_cuda_f32(ref, "ref", ndim=1)
    if ref.shape[0] != plan.D or ref.device != Q.device:
        raise ValueError("ref must be a CUDA float32 [D] tensor on Q's device")


def _layout_ld(O, layout: int) -> int:
    if layout == LAYOUT_TILES:
        if O.dim() != 3 or O.shape[2] != 64 or not O.is_contiguous():
            raise ValueError("the tiled layout takes a contiguous [tiles, ld, 64] tensor")
        return O.shape[1]
    return O.stride(0)


def project(plan: Plan, X, out=None, norm2=None, layout: int = LAYOUT_ROWS, stream=None):
    """saq_project: (O f32, ||x - c||^2 f32 [n]).  Row layout: O [n, >= D_kept];
    dims layout: O [D_kept, ld >= n] with ld % 4 == 0; tiled layout: O
    [ceil(n / 64), ld >= D_kept, 64]."""
    torch = _torch()
    _require_cuda_f32(X, "X", plan.D)
    n = X.shape[0]
    if out is None:
        dk = max(plan.D_kept, 1)
        shape = {LAYOUT_ROWS: (n, dk), LAYOUT_DIMS: (dk, (n + 3) // 4 * 4),
                 LAYOUT_TILES: ((n + 63) // 64, dk, 64)}[layout]
        out = torch.empty(shape, dtype=torch.float32, device=X.device)
    if norm2 is None:
        norm2 = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(lib().saq_project(plan._h, _dev_ptr(X), n, _dev_ptr(out), _layout_ld(out, layout),
                             layout, _dev_ptr(norm2), _stream_ptr(stream, X.device)))
    return out, norm2


def quantize(plan: Plan, O, rounds: int = 4, norm2=None, codes=None, factors=None,
             layout: int = LAYOUT_ROWS, n: Optional[int] = None, stream=None):
    """saq_quantize on projected rows O (row layout [n, >= D_kept]; dims
    layout [D_kept, ld] or tiled layout [tiles, ld, 64] with ``n`` given)."""
    _require_cuda_f32(O, "O", ndim=3 if layout == LAYOUT_TILES else 2)
    if n is None:
        if layout != LAYOUT_ROWS:
            raise ValueError("n is required for the dims and tiled layouts")
        n = O.shape[0]
    if layout == LAYOUT_TILES and O.shape[0] * 64 < n:
        raise ValueError("tiled O holds fewer than n vectors")
    codes, factors = _alloc_out(plan, n, O.device, codes, factors)
    _check(lib().saq_quantize(plan._h, _dev_ptr(O), _layout_ld(O, layout), layout, n,
                              _dev_ptr(norm2), rounds, _dev_ptr(codes), _dev_ptr(factors),
                              _stream_ptr(stream, O.device)))
    return codes, factors


def _scan_buffers(plan: Plan, Q, codes, factors, out, workspace):
    """Shape and type checks shared by the scans; allocates what is None."""
    torch = _torch()
    _require_cuda_f32(Q, "Q", plan.D)
    nq, n = Q.shape[0], codes.shape[0]
    for t, name in ((codes, "codes"), (factors, "factors")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.device == Q.device):
            raise TypeError(f"{name} must be a CUDA tensor on Q's device")
    _alloc_out(plan, n, Q.device, codes, factors)
    if out is None:
        out = torch.empty((nq, n), dtype=torch.float32, device=Q.device)
    _require_cuda_f32(out, "out", n)
    if out.shape[0] != nq:
        raise ValueError("out must be [nq, n]")
    need = plan.estimate_workspace_bytes(nq)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=Q.device)
    elif workspace.numel() * workspace.element_size() < need:
        raise ValueError(f"workspace needs {need} bytes")
    return nq, n, out, workspace


def estimate_dist(plan: Plan, Q, codes, factors, out=None, workspace=None, stream=None,
                  prefix_bits: int = 0, ref=None):
    """saq_estimate_dist: estimated squared distances f32 [nq, n]; with
    prefix_bits > 0, saq_estimate_dist_prefix (each segment's first
    min(prefix_bits, B) bits only); with ref (CUDA float32 [D]),
    saq_estimate_dist_ref over records encoded against that reference."""
    nq, n, out, workspace = _scan_buffers(plan, Q, codes, factors, out, workspace)
    if ref is not None:
        if prefix_bits:
            raise ValueError("prefix_bits and ref do not combine")
        _require_ref(plan, ref, Q)
        _check(lib().saq_estimate_dist_ref(plan._h, _dev_ptr(Q), nq, _dev_ptr(ref),
                                           _dev_ptr(codes), _dev_ptr(factors), n, _dev_ptr(out),
                                           _dev_ptr(workspace),
                                           workspace.numel() * workspace.element_size(),
                                           _stream_ptr(stream, Q.device)))
        return out
    _check(lib().saq_estimate_dist_prefix(plan._h, _dev_ptr(Q), nq, _dev_ptr(codes),
                                          _dev_ptr(factors), n, int(prefix_bits), _dev_ptr(out),
                                          _dev_ptr(workspace),
                                          workspace.numel() * workspace.element_size(),
                                          _stream_ptr(stream, Q.device)))
    return out


def estimate_multistage(plan: Plan, Q, codes, factors, tau, m: float = 4.0, out=None,
                        stage=None, workspace=None, stream=None, ref=None):
    """saq_estimate_multistage (Section 4.3): returns (dist2 f32 [nq, n],
    stage u8 [nq, n]).  tau: CUDA float32 [nq] thresholds; a pair whose lower
    bound before segment t exceeds its query's threshold gets that bound and
    stage t, the others the full estimate and stage k."""
    torch = _torch()
    nq, n, out, workspace = _scan_buffers(plan, Q, codes, factors, out, workspace)
    _require_cuda_f32(tau, "tau", ndim=1)
    if tau.shape[0] != nq:
        raise ValueError("tau must have one threshold per query")
    if stage is None:
        stage = torch.empty((nq, n), dtype=torch.uint8, device=Q.device)
    if stage.shape != (nq, n) or stage.dtype != torch.uint8 or not stage.is_contiguous() \
            or not stage.is_cuda:
        raise ValueError("stage must be a contiguous CUDA uint8 tensor [nq, n]")
    if ref is not None:
        _require_ref(plan, ref, Q)
        _check(lib().saq_estimate_multistage_ref(plan._h, _dev_ptr(Q), nq, _dev_ptr(ref),
                                                 _dev_ptr(codes), _dev_ptr(factors), n,
                                                 _dev_ptr(tau), float(m), _dev_ptr(out),
                                                 _dev_ptr(stage), _dev_ptr(workspace),
                                                 workspace.numel() * workspace.element_size(),
                                                 _stream_ptr(stream, Q.device)))
        return out, stage
    _check(lib().saq_estimate_multistage(plan._h, _dev_ptr(Q), nq, _dev_ptr(codes),
                                         _dev_ptr(factors), n, _dev_ptr(tau), float(m),
                                         _dev_ptr(out), _dev_ptr(stage), _dev_ptr(workspace),
                                         workspace.numel() * workspace.element_size(),
                                         _stream_ptr(stream, Q.device)))
    return out, stage


def covariance(X, fit_sample: int = 0, mean=None, cov=None, workspace=None, stream=None):
    """saq_covariance: (mean f64 [D], covariance f64 [D, D]) of the fit
    sample of the device rows X (CUDA float32 [n, D])."""
    torch = _torch()
    _require_cuda_f32(X, "X")
    n, D = X.shape
    if mean is None:
        mean = torch.empty(D, dtype=torch.float64, device=X.device)
    if cov is None:
        cov = torch.empty((D, D), dtype=torch.float64, device=X.device)
    for t, shape, name in ((mean, (D,), "mean"), (cov, (D, D), "cov")):
        if tuple(t.shape) != shape or t.dtype != torch.float64 or not t.is_contiguous() \
                or t.device != X.device:
            raise ValueError(f"{name} must be a contiguous float64 tensor {shape} on X's device")
    need = int(lib().saq_covariance_workspace_bytes(n, D, int(fit_sample)))
    if need < 0:
        raise ValueError("bad covariance sizes")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=X.device)
    _check(lib().saq_covariance(_dev_ptr(X), n, D, int(fit_sample), _dev_ptr(mean), _dev_ptr(cov),
                                _dev_ptr(workspace), workspace.numel() * workspace.element_size(),
                                _stream_ptr(stream, X.device)))
    return mean, cov


def sym_eigen(A, w=None, V=None, workspace=None, stream=None):
    """saq_sym_eigen_device: (eigenvalues f64 [n], eigenvectors f64 [n, n],
    eigenvector j in column j) of the symmetric CUDA float64 matrix A."""
    torch = _torch()
    if not (A.is_cuda and A.dtype == torch.float64 and A.is_contiguous() and A.dim() == 2
            and A.shape[0] == A.shape[1]):
        raise ValueError("A must be a square contiguous CUDA float64 tensor")
    n = A.shape[0]
    if w is None:
        w = torch.empty(n, dtype=torch.float64, device=A.device)
    if V is None:
        V = torch.empty((n, n), dtype=torch.float64, device=A.device)
    need = int(lib().saq_sym_eigen_workspace_bytes(n))
    if need < 0:
        raise ValueError("bad size")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=A.device)
    _check(lib().saq_sym_eigen_device(_dev_ptr(A), n, _dev_ptr(w), _dev_ptr(V), _dev_ptr(workspace),
                                      workspace.numel() * workspace.element_size(),
                                      _stream_ptr(stream, A.device)))
    return w, V


def unpack_codes(plan: Plan, packed: np.ndarray) -> np.ndarray:
    """Host-side decoding of records [n, code_bytes] into codes [n, D_kept]
    (int32) following the bit-plane layout of include/saq.h."""
    packed = np.asarray(packed, np.uint8)
    n = packed.shape[0]
    out = np.zeros((n, plan.D_kept), np.int32)
    pos = off = 0
    for w, b in zip(plan.kept_widths, plan.kept_bits):
        pb = (w + 7) // 8
        for p in range(b - 1, -1, -1):
            bits = np.unpackbits(packed[:, pos:pos + pb], axis=1, bitorder="little")[:, :w]
            out[:, off:off + w] |= bits.astype(np.int32) << p
            pos += pb
        off += w
    return out


@dataclasses.dataclass(frozen=True)
class BatchTuning:
    """Launch shape of saq_encode_batched (saq_batch_tuning): the mode (one
    persistent fused launch, or two grouped launches), the projection tile
    rows (0 auto, 64 or 128), and for the grouped mode the quantize waves
    per workgroup and the projection tile order."""
    quant_waves: int = 1
    gemm_xcd_order: bool = True
    mode: int = BATCH_FUSED
    tile_rows: int = 0

    def _c(self) -> _Tuning:
        return _Tuning(int(self.quant_waves), int(bool(self.gemm_xcd_order)), int(self.mode),
                       int(self.tile_rows), 0)


def _batch_struct(entries):
    arr = (_BatchItem * len(entries))()
    for i, (plan, X, codes, fac) in enumerate(entries):
        arr[i] = _BatchItem(plan._h.value, _dev_ptr(X), X.shape[0], _dev_ptr(codes), _dev_ptr(fac))
    return arr


def batched_workspace_bytes(entries, tuning: Optional[BatchTuning] = None) -> int:
    arr = _batch_struct([(p, X, None, None) for p, X, *_ in entries])
    t = (tuning or BatchTuning())._c()
    need = int(lib().saq_encode_batched_workspace_bytes(arr, len(entries), ctypes.byref(t)))
    if need < 0:
        raise SaqError(1, lib().saq_last_error().decode())
    return need


def encode_batched(entries, rounds: int = 4, tuning: Optional[BatchTuning] = None,
                   workspace=None, stream=None):
    """saq_encode_batched over ``entries`` = [(plan, X), ...] or
    [(plan, X, codes, factors), ...]; returns [(codes, factors), ...]."""
    torch = _torch()
    if not 1 <= len(entries) <= BATCH_MAX:
        raise ValueError(f"a batch holds 1..{BATCH_MAX} datasets")
    full = []
    for e in entries:
        plan, X = e[0], e[1]
        _require_cuda_f32(X, "X", plan.D)
        codes, fac = _alloc_out(plan, X.shape[0], X.device, *(e[2:4] if len(e) > 2 else ()))
        full.append((plan, X, codes, fac))
    arr = _batch_struct(full)
    t = (tuning or BatchTuning())._c()
    dev = full[0][1].device
    if workspace is None:
        need = int(lib().saq_encode_batched_workspace_bytes(arr, len(full), ctypes.byref(t)))
        if need < 0:
            raise SaqError(1, lib().saq_last_error().decode())
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(lib().saq_encode_batched(arr, len(full), rounds, ctypes.byref(t), _dev_ptr(workspace),
                                    workspace.numel() * workspace.element_size(),
                                    _stream_ptr(stream, dev)))
    return [(c, f) for _, _, c, f in full]
