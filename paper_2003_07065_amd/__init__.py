"""Python binding of the gfx950 downsampled SST library (libsst_hip.so).

Argument marshalling only: every step of the transform runs in the HIP kernels
behind the C ABI of include/sst.h.  PyTorch provides device memory and the
current stream.  There is no CPU fallback: importing works without a GPU, but
every call that reaches the library needs the built shared object and a HIP
device, and raises otherwise.

Names mirror the C ABI: ``Plan`` wraps sst_plan / sst_plan_query /
sst_plan_bind / sst_destroy, and its methods ``forward``, ``ridge`` and
``inverse`` wrap sst_forward, sst_ridge and sst_inverse.  ``Batch`` wraps the
sst_batch_* calls (many channels, one persistent launch per DFT-size group).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsst_hip.so")

SST_OK = 0
SST_E_ARG = -1
SST_E_UNSUPPORTED = -2
SST_E_WORKSPACE = -3
SST_E_DEVICE = -4
SST_E_STATE = -5
SST_E_NOMEM = -6

SST_THR_ABS = 0
SST_THR_REL_MAX = 1
SST_PREC_FP32_FFT = 0
SST_PREC_GEMM_BF16 = 1
SST_PREC_GEMM_F16X3 = 2
PRECISIONS = {"fp32": SST_PREC_FP32_FFT, "bf16": SST_PREC_GEMM_BF16,
              "f16x3": SST_PREC_GEMM_F16X3}
SST_FWD_REUSE_GAMMA = 1
SST_FWD_OUT_MAG_F32 = 2
SST_FWD_OUT_MAG_F16 = 4
SST_INV_ACCUMULATE = 1
SST_INV_EQ15 = 2

EXPORTED = ("sst_plan", "sst_plan_query", "sst_plan_bind", "sst_forward", "sst_forward_static",
            "sst_ridge", "sst_ridge_guided",
            "sst_inverse", "sst_destroy", "sst_status_string", "sst_last_error",
            "sst_critical_hf", "sst_batch_plan", "sst_batch_query", "sst_batch_bind",
            "sst_batch_set_io", "sst_batch_commit", "sst_batch_forward", "sst_batch_inverse",
            "sst_batch_destroy", "sst_plan_get_tuning", "sst_plan_set_tuning", "sst_autotune",
            "sst_tuning_save", "sst_tuning_load", "sst_renyi", "sst_stft", "sst_stft_inverse")


class SSTError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("n_samples", ctypes.c_int64),
        ("fs", ctypes.c_double),
        ("win_len", ctypes.c_int32),
        ("sigma", ctypes.c_double),
        ("window", ctypes.POINTER(ctypes.c_double)),
        ("dwindow", ctypes.POINTER(ctypes.c_double)),
        ("hop", ctypes.c_int32),
        ("nfft", ctypes.c_int32),
        ("f_lo", ctypes.c_double),
        ("f_hi", ctypes.c_double),
        ("subdiv", ctypes.c_int32),
        ("thr_mode", ctypes.c_int32),
        ("thr", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


class Shape(ctypes.Structure):
    _fields_ = [
        ("n_samples", ctypes.c_int64),
        ("n_frames", ctypes.c_int64),
        ("win_len", ctypes.c_int32),
        ("hop", ctypes.c_int32),
        ("nfft", ctypes.c_int32),
        ("subdiv", ctypes.c_int32),
        ("k1", ctypes.c_int32),
        ("k2", ctypes.c_int32),
        ("n_src", ctypes.c_int32),
        ("n_dst", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_size_t),
        ("t_row_bytes", ctypes.c_size_t),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("fwd_wg_per_cu", ctypes.c_int32),
        ("seed_step", ctypes.c_int32),
        ("inv_tf", ctypes.c_int32),
        ("inv_groups", ctypes.c_int32),
    ]

    def as_dict(self):
        return {"fwd_wg_per_cu": self.fwd_wg_per_cu, "seed_step": self.seed_step,
                "inv_tf": self.inv_tf, "inv_groups": self.inv_groups}


class FwdAux(ctypes.Structure):
    _fields_ = [
        ("S", ctypes.c_void_p),
        ("Sd", ctypes.c_void_p),
        ("idx", ctypes.c_void_p),
        ("colstats", ctypes.c_void_p),
        ("gamma", ctypes.c_void_p),
        ("kernel_events", ctypes.c_void_p * 2),
    ]


_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc, gfx950); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    L.sst_plan.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(vp)]
    L.sst_plan_query.argtypes = [vp, ctypes.POINTER(Shape)]
    L.sst_plan_bind.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.sst_forward.argtypes = [vp, vp, i64, i64, vp, ctypes.POINTER(FwdAux), u32, vp]
    L.sst_forward_static.argtypes = [vp, vp, i64, i64, vp, ctypes.POINTER(FwdAux), u32, vp]
    L.sst_ridge.argtypes = [vp, vp, i64, ctypes.POINTER(i32), i32, vp, vp]
    L.sst_ridge_guided.argtypes = [vp, vp, i64, vp, ctypes.POINTER(i32), i32, vp, vp]
    L.sst_inverse.argtypes = [vp, vp, i64, i64, vp, i32, i32, vp, vp, vp, u32, vp]
    L.sst_destroy.argtypes = [vp]
    L.sst_destroy.restype = None
    L.sst_status_string.argtypes = [i32]
    L.sst_status_string.restype = ctypes.c_char_p
    L.sst_last_error.argtypes = []
    L.sst_last_error.restype = ctypes.c_char_p
    L.sst_critical_hf.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
    L.sst_batch_plan.argtypes = [ctypes.POINTER(Params), i32, ctypes.POINTER(vp)]
    L.sst_batch_query.argtypes = [vp, i32, ctypes.POINTER(Shape)]
    L.sst_batch_bind.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.sst_batch_set_io.argtypes = [vp, i32, vp, vp, vp, i32, i32, vp, vp, vp]
    L.sst_batch_commit.argtypes = [vp, vp]
    L.sst_batch_forward.argtypes = [vp, i32, i32, u32, vp]
    L.sst_batch_inverse.argtypes = [vp, i32, i32, vp]
    L.sst_batch_destroy.argtypes = [vp]
    L.sst_batch_destroy.restype = None
    L.sst_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.sst_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.sst_autotune.argtypes = [vp, vp, vp, vp, i32, i32, vp, i32, vp, ctypes.POINTER(Tuning)]
    L.sst_tuning_save.argtypes = [vp, ctypes.c_char_p]
    L.sst_tuning_load.argtypes = [vp, ctypes.c_char_p]
    L.sst_renyi.argtypes = [vp, i32, i64, i32, i64, i32, vp, vp, vp]
    L.sst_stft.argtypes = [vp, vp, i64, i64, vp, vp, vp]
    L.sst_stft_inverse.argtypes = [vp, vp, vp, vp]
    for name in ("sst_plan", "sst_plan_query", "sst_plan_bind", "sst_forward",
                 "sst_forward_static", "sst_ridge", "sst_ridge_guided",
                 "sst_inverse", "sst_critical_hf", "sst_batch_plan", "sst_batch_query",
                 "sst_batch_bind", "sst_batch_set_io", "sst_batch_commit", "sst_batch_forward",
                 "sst_batch_inverse", "sst_plan_get_tuning", "sst_plan_set_tuning",
                 "sst_autotune", "sst_tuning_save", "sst_tuning_load", "sst_renyi",
                 "sst_stft", "sst_stft_inverse"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def _check(status: int, where: str):
    if status != SST_OK:
        detail = lib().sst_last_error().decode(errors="replace")
        raise SSTError(status, where, detail)


def status_string(status: int) -> str:
    return lib().sst_status_string(int(status)).decode()


def critical_hf(n: float, sigma_s: float, fs: float):
    """Advisory H_f bounds of Eq. 38 and Eq. 46 (host only)."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib().sst_critical_hf(float(n), float(sigma_s), float(fs), ctypes.byref(a),
                                 ctypes.byref(b)), "sst_critical_hf")
    return a.value, b.value


SST_RENYI_WORK_DOUBLES = 2048
_RENYI_KIND = {"complex64": 0, "float32": 1, "float16": 2}


def renyi(C, alpha: int = 3, cols: Optional[int] = None, out=None):
    """sst_renyi: Renyi entropy (bits) of P = |C|^2 over a 2-D device tensor
    (complex64 coefficients, or float32 / float16 magnitudes).  Returns the
    device tensor out = [sum P, sum P^alpha, R] (float64)."""
    import torch
    if C.dim() != 2 or C.stride(1) != 1:
        raise ValueError("C must be a 2-D tensor with contiguous rows")
    kind = {torch.complex64: 0, torch.float32: 1, torch.float16: 2}.get(C.dtype)
    if kind is None:
        raise ValueError("C must be complex64, float32 or float16")
    rows, n = C.shape
    cols = n if cols is None else int(cols)
    work = torch.empty(SST_RENYI_WORK_DOUBLES, dtype=torch.float64, device=C.device)
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=C.device)
    _check(lib().sst_renyi(ctypes.c_void_p(C.data_ptr()), kind, int(rows), cols,
                           int(C.stride(0)), int(alpha), ctypes.c_void_p(work.data_ptr()),
                           ctypes.c_void_p(out.data_ptr()),
                           ctypes.c_void_p(_stream_handle(C.device))), "sst_renyi")
    return out


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream_handle(device) -> int:
    import torch
    return int(torch.cuda.current_stream(device).cuda_stream)


def _params(n_samples: int, fs: float, win_len: int, sigma: float, hop: int, nfft: int,
            f_lo: float, f_hi: float, subdiv: int, thr_mode: str, thr: float, window, dwindow,
            keep: list, precision: str = "fp32") -> Params:
    p = Params()
    p.struct_size = ctypes.sizeof(Params)
    p.n_samples = int(n_samples)
    p.fs = float(fs)
    p.win_len = int(win_len)
    p.sigma = float(sigma)
    if window is not None:
        import numpy as np
        w = np.ascontiguousarray(np.asarray(window, dtype=np.float64))
        dw = np.ascontiguousarray(np.asarray(dwindow, dtype=np.float64))
        keep += [w, dw]
        p.window = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.dwindow = dw.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.hop = int(hop)
    p.nfft = int(nfft)
    p.f_lo = float(f_lo)
    p.f_hi = float(f_hi)
    p.subdiv = int(subdiv)
    p.thr_mode = SST_THR_ABS if thr_mode == "abs" else SST_THR_REL_MAX
    p.thr = float(thr)
    p.precision = PRECISIONS[precision]
    p.flags = 0
    return p


class Plan:
    """A transform plan (host tables) bound to a torch-allocated device workspace."""

    def __init__(self, n_samples: int, fs: float, win_len: int, sigma: float, hop: int,
                 nfft: int, f_lo: float, f_hi: float, subdiv: int = 1, thr_mode: str = "rel",
                 thr: float = 1e-3, window=None, dwindow=None, device=None,
                 precision: str = "fp32"):
        """precision: "fp32" (FFT), "bf16" or "f16x3" (DFT-as-GEMM on the matrix cores)."""
        self._h = None
        keep = []
        p = _params(n_samples, fs, win_len, sigma, hop, nfft, f_lo, f_hi, subdiv, thr_mode, thr,
                    window, dwindow, keep, precision)
        self.precision = precision
        h = ctypes.c_void_p()
        _check(lib().sst_plan(ctypes.byref(p), ctypes.byref(h)), "sst_plan")
        self._h = h
        sh = Shape()
        _check(lib().sst_plan_query(self._h, ctypes.byref(sh)), "sst_plan_query")
        self.shape = sh
        self.n_samples = sh.n_samples
        self.n_frames = sh.n_frames
        self.k1, self.k2 = sh.k1, sh.k2
        self.n_src, self.n_dst = sh.n_src, sh.n_dst
        self.nfft, self.hop, self.subdiv, self.win_len = sh.nfft, sh.hop, sh.subdiv, sh.win_len
        self.workspace = None
        self.device = None
        if device is not None:
            self.bind(device)

    @classmethod
    def from_config(cls, n_samples: int, cfg, device=None, precision: str = "fp32") -> "Plan":
        return cls(n_samples, cfg.fs, cfg.win_len, cfg.sigma, cfg.hop, cfg.nfft, cfg.f_lo,
                   cfg.f_hi, cfg.subdiv, cfg.thr_mode, cfg.thr, device=device,
                   precision=precision)

    def bind(self, device="cuda"):
        import torch
        device = torch.device(device)
        if device.type != "cuda":
            raise ValueError("the workspace must live on a HIP device")
        if device.index is None:
            device = torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(device):
            ws = torch.empty(int(self.shape.workspace_bytes) + 256, dtype=torch.uint8,
                             device=device)
            off = (-int(ws.data_ptr())) % 256
            base = int(ws.data_ptr()) + off
            _check(lib().sst_plan_bind(self._h, ctypes.c_void_p(base),
                                       ctypes.c_size_t(self.shape.workspace_bytes),
                                       ctypes.c_void_p(_stream_handle(device))),
                   "sst_plan_bind")
        self.workspace = ws
        self.device = device
        return self

    def _need_bound(self):
        if self.workspace is None:
            raise SSTError(SST_E_STATE, "Plan", "bind() the plan to a device first")

    def _check_buf(self, t, dtype, numel: int, name: str):
        """Every buffer handed to the C ABI: dtype, contiguity, device and size."""
        if t is None:
            return
        if t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} tensor")
        if t.device != self.device:
            raise ValueError(f"{name} must live on the plan's device {self.device}")
        if t.numel() < numel:
            raise ValueError(f"{name} holds {t.numel()} elements, the call needs {numel}")

    def forward(self, x, T=None, frame0: int = 0, nframes: Optional[int] = None, *,
                S=None, Sd=None, idx=None, colstats=None, gamma=None,
                reuse_gamma: bool = False, kernel_events=None, out: str = "complex64"):
        """SST rows of frames [frame0, frame0+nframes) into T (complex64 [nframes, n_dst]);
        out="mag_f32" / "mag_f16" writes |T| as float32 / float16 instead.

        kernel_events: optional pair of torch.cuda.Event, already recorded once
        (so that they exist); the library records them again right around the
        fused forward kernel."""
        self._need_bound()
        return self._forward_call(lib().sst_forward, "sst_forward", x, T, frame0, nframes, S, Sd,
                                  idx, colstats, gamma, reuse_gamma, kernel_events, out)

    def forward_static(self, x, T=None, frame0: int = 0, nframes: Optional[int] = None, *,
                       S=None, Sd=None, idx=None, colstats=None, gamma=None,
                       reuse_gamma: bool = False, kernel_events=None):
        """sst_forward_static: as forward(), with the library's fixed per-device
        scratch as the workspace (no bind, no device allocation by the call;
        T must then be given)."""
        import torch
        if T is None:
            raise ValueError("forward_static needs a caller-allocated T")
        if self.device is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        return self._forward_call(lib().sst_forward_static, "sst_forward_static", x, T, frame0,
                                  nframes, S, Sd, idx, colstats, gamma, reuse_gamma,
                                  kernel_events, "complex64")

    def _forward_call(self, fn, where, x, T, frame0, nframes, S, Sd, idx, colstats, gamma,
                      reuse_gamma, kernel_events, out):
        import torch
        fmt = {"complex64": (torch.complex64, 0), "mag_f32": (torch.float32, SST_FWD_OUT_MAG_F32),
               "mag_f16": (torch.float16, SST_FWD_OUT_MAG_F16)}
        if out not in fmt:
            raise ValueError("out must be complex64, mag_f32 or mag_f16")
        tdt, oflag = fmt[out]
        if nframes is None:
            nframes = self.n_frames - frame0
        if x.dtype != torch.float32 or not x.is_contiguous() or x.device != self.device:
            raise ValueError("x must be a contiguous float32 tensor on the plan's device")
        if x.numel() != self.n_samples:
            raise ValueError("x length differs from the plan's n_samples")
        if T is None:
            T = torch.empty((nframes, self.n_dst), dtype=tdt, device=self.device)
        self._check_buf(T, tdt, nframes * self.n_dst, "T")
        for t, n, dt, nm in ((S, self.n_src, torch.complex64, "S"),
                             (Sd, self.n_src, torch.complex64, "Sd"),
                             (idx, self.n_src, torch.int32, "idx"),
                             (colstats, 3, torch.float64, "colstats")):
            self._check_buf(t, dt, nframes * n, nm)
        self._check_buf(gamma, torch.float32, 1, "gamma")
        aux = FwdAux(_ptr(S), _ptr(Sd), _ptr(idx), _ptr(colstats), _ptr(gamma))
        if kernel_events is not None:
            for i, ev in enumerate(kernel_events):
                if not ev.cuda_event:
                    raise ValueError("kernel_events must have been recorded once")
                aux.kernel_events[i] = ev.cuda_event
        _check(fn(self._h, ctypes.c_void_p(x.data_ptr()), int(frame0), int(nframes),
                  ctypes.c_void_p(T.data_ptr()), ctypes.byref(aux),
                  (SST_FWD_REUSE_GAMMA if reuse_gamma else 0) | oflag,
                  ctypes.c_void_p(_stream_handle(self.device))), where)
        return T

    def ridge(self, T, bands: Sequence[Sequence[int]], nframes: Optional[int] = None,
              out=None, centre=None):
        """Per-frame argmax ridge of each component inside its destination-bin band
        (sst_ridge), or inside bands relative to a per-frame guide bin
        centre[q, m] (sst_ridge_guided)."""
        import torch
        self._need_bound()
        if nframes is None:
            nframes = T.shape[0]
        n_comp = len(bands)
        arr = (ctypes.c_int32 * (2 * n_comp))(*[int(v) for b in bands for v in b])
        if out is None:
            out = torch.empty((n_comp, nframes), dtype=torch.int32, device=self.device)
        self._check_buf(T, torch.complex64, nframes * self.n_dst, "T")
        self._check_buf(out, torch.int32, n_comp * nframes, "out")
        stream = ctypes.c_void_p(_stream_handle(self.device))
        if centre is None:
            _check(lib().sst_ridge(self._h, ctypes.c_void_p(T.data_ptr()), int(nframes), arr,
                                   n_comp, ctypes.c_void_p(out.data_ptr()), stream), "sst_ridge")
        else:
            self._check_buf(centre, torch.int32, n_comp * nframes, "centre")
            _check(lib().sst_ridge_guided(self._h, ctypes.c_void_p(T.data_ptr()), int(nframes),
                                          ctypes.c_void_p(centre.data_ptr()), arr, n_comp,
                                          ctypes.c_void_p(out.data_ptr()), stream),
                   "sst_ridge_guided")
        return out

    def inverse(self, T, ridge, hw: int, xhat=None, frame0: int = 0,
                nframes: Optional[int] = None, xref=None, err=None, accumulate: bool = False,
                eq15: bool = False):
        """Direct inverse (Eqs. 25-26, or Eq. 15 with eq15=True) of every ridge component."""
        import torch
        self._need_bound()
        if nframes is None:
            nframes = T.shape[0]
        n_comp = ridge.shape[0] if ridge.dim() == 2 else 1
        if ridge.numel() != n_comp * nframes:
            raise ValueError("ridge must hold n_comp * nframes entries")
        self._check_buf(ridge, torch.int32, n_comp * nframes, "ridge")
        self._check_buf(T, torch.complex64, nframes * self.n_dst, "T")
        if xhat is None:
            xhat = torch.empty((n_comp, self.n_samples), dtype=torch.float32, device=self.device)
        self._check_buf(xhat, torch.float32, n_comp * self.n_samples, "xhat")
        self._check_buf(xref, torch.float32, n_comp * self.n_samples, "xref")
        self._check_buf(err, torch.float64, 2 * n_comp, "err")
        flags = (SST_INV_ACCUMULATE if accumulate else 0) | (SST_INV_EQ15 if eq15 else 0)
        _check(lib().sst_inverse(self._h, ctypes.c_void_p(T.data_ptr()), int(frame0),
                                 int(nframes), ctypes.c_void_p(ridge.data_ptr()), int(n_comp),
                                 int(hw), ctypes.c_void_p(xhat.data_ptr()),
                                 ctypes.c_void_p(_ptr(xref)), ctypes.c_void_p(_ptr(err)), flags,
                                 ctypes.c_void_p(_stream_handle(self.device))), "sst_inverse")
        return xhat

    def stft(self, x, S=None, frame0: int = 0, nframes: Optional[int] = None, Sd=None):
        """sst_stft: in-band STFT rows (complex64 [nframes, n_src]) of frames
        [frame0, frame0 + nframes), and S' when Sd is given."""
        import torch
        self._need_bound()
        if nframes is None:
            nframes = self.n_frames - frame0
        self._check_buf(x, torch.float32, self.n_samples, "x")
        if S is None:
            S = torch.empty((nframes, self.n_src), dtype=torch.complex64, device=self.device)
        self._check_buf(S, torch.complex64, nframes * self.n_src, "S")
        self._check_buf(Sd, torch.complex64, nframes * self.n_src, "Sd")
        _check(lib().sst_stft(self._h, ctypes.c_void_p(x.data_ptr()), int(frame0), int(nframes),
                              ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(_ptr(Sd)),
                              ctypes.c_void_p(_stream_handle(self.device))), "sst_stft")
        return S

    def stft_inverse(self, S, xhat=None):
        """sst_stft_inverse: STFT synthesis (Eqs. 10-11) of the whole signal."""
        import torch
        self._need_bound()
        self._check_buf(S, torch.complex64, self.n_frames * self.n_src, "S")
        if xhat is None:
            xhat = torch.empty(self.n_samples, dtype=torch.float32, device=self.device)
        self._check_buf(xhat, torch.float32, self.n_samples, "xhat")
        _check(lib().sst_stft_inverse(self._h, ctypes.c_void_p(S.data_ptr()),
                                      ctypes.c_void_p(xhat.data_ptr()),
                                      ctypes.c_void_p(_stream_handle(self.device))),
               "sst_stft_inverse")
        return xhat

    # -- launch choices (sst_plan_get_tuning / sst_plan_set_tuning / sst_autotune) --

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib().sst_plan_get_tuning(self._h, ctypes.byref(t)), "sst_plan_get_tuning")
        return t.as_dict()

    def set_tuning(self, fwd_wg_per_cu: int = 0, seed_step: int = 0, inv_tf: int = 0,
                   inv_groups: int = 0):
        t = Tuning(int(fwd_wg_per_cu), int(seed_step), int(inv_tf), int(inv_groups))
        _check(lib().sst_plan_set_tuning(self._h, ctypes.byref(t)), "sst_plan_set_tuning")

    def autotune(self, x, T, ridge=None, hw: int = 0, xhat=None, reps: int = 3) -> dict:
        """Time the launch choices on these buffers and keep the fastest."""
        import torch
        self._need_bound()
        self._check_buf(x, torch.float32, self.n_samples, "x")
        self._check_buf(T, torch.complex64, self.n_frames * self.n_dst, "T")
        n_comp = 0
        if ridge is not None:
            n_comp = ridge.shape[0] if ridge.dim() == 2 else 1
            self._check_buf(ridge, torch.int32, n_comp * self.n_frames, "ridge")
            self._check_buf(xhat, torch.float32, n_comp * self.n_samples, "xhat")
        t = Tuning()
        _check(lib().sst_autotune(self._h, ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(_ptr(ridge)),
                                  int(n_comp), int(hw), ctypes.c_void_p(_ptr(xhat)), int(reps),
                                  ctypes.c_void_p(_stream_handle(self.device)), ctypes.byref(t)),
               "sst_autotune")
        return t.as_dict()

    def tuning_save(self, path: str):
        _check(lib().sst_tuning_save(self._h, os.fsencode(path)), "sst_tuning_save")

    def tuning_load(self, path: str):
        _check(lib().sst_tuning_load(self._h, os.fsencode(path)), "sst_tuning_load")

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.sst_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many channels with their own parameters (sst_batch_*).

    ``configs`` is a list of (n_samples, cfg) pairs (cfg as for Plan.from_config).
    Buffers are recorded with ``set_io`` and uploaded with ``commit``; ``forward``
    and ``inverse`` then launch kernels only (capturable in a HIP graph).
    """

    def __init__(self, configs, device="cuda"):
        import torch
        self._h = None
        n = len(configs)
        arr = (Params * n)()
        keep = []
        for i, (ns, cfg) in enumerate(configs):
            arr[i] = _params(ns, cfg.fs, cfg.win_len, cfg.sigma, cfg.hop, cfg.nfft, cfg.f_lo,
                             cfg.f_hi, cfg.subdiv, cfg.thr_mode, cfg.thr, None, None, keep)
        h = ctypes.c_void_p()
        _check(lib().sst_batch_plan(arr, n, ctypes.byref(h)), "sst_batch_plan")
        self._h = h
        self.n_channels = n
        self.shapes = []
        for c in range(n):
            sh = Shape()
            _check(lib().sst_batch_query(self._h, c, ctypes.byref(sh)), "sst_batch_query")
            self.shapes.append(sh)
        device = torch.device(device)
        if device.index is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = device
        nbytes = int(self.shapes[0].workspace_bytes)
        with torch.cuda.device(device):
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            base = int(ws.data_ptr()) + ((-int(ws.data_ptr())) % 256)
            _check(lib().sst_batch_bind(self._h, ctypes.c_void_p(base), ctypes.c_size_t(nbytes),
                                        ctypes.c_void_p(_stream_handle(device))), "sst_batch_bind")
        self.workspace = ws
        self._io = [None] * n

    def set_io(self, c: int, x, T, ridge=None, hw: int = 0, xhat=None, xref=None, err=None):
        """Record channel c's buffers (kept alive by the batch until replaced)."""
        import torch
        sh = self.shapes[c]
        for t, nm in ((x, "x"), (T, "T"), (ridge, "ridge"), (xhat, "xhat"), (xref, "xref"),
                      (err, "err")):
            if t is not None and (t.device != self.device or not t.is_contiguous()):
                raise ValueError(f"channel {c}: {nm} must be contiguous on {self.device}")
        if xref is not None and (xref.dtype != torch.float32 or xhat is None
                                 or xref.numel() < xhat.numel()):
            raise ValueError(f"channel {c}: xref must be float32 shaped like xhat")
        if err is not None and (err.dtype != torch.float64 or ridge is None
                                or err.numel() < 2 * (ridge.shape[0] if ridge.dim() == 2 else 1)):
            raise ValueError(f"channel {c}: err must be float64 [n_comp, 2]")
        if x is None or x.dtype != torch.float32 or x.numel() != sh.n_samples:
            raise ValueError(f"channel {c}: x must be float32 with n_samples elements")
        if T is None or T.dtype != torch.complex64 or T.numel() < sh.n_frames * sh.n_dst:
            raise ValueError(f"channel {c}: T must be complex64 [n_frames, n_dst]")
        n_comp = 0
        if ridge is not None:
            n_comp = ridge.shape[0] if ridge.dim() == 2 else 1
            if ridge.dtype != torch.int32 or ridge.numel() != n_comp * sh.n_frames:
                raise ValueError(f"channel {c}: ridge must be int32 [n_comp, n_frames]")
            if xhat is None or xhat.dtype != torch.float32 or xhat.numel() < n_comp * sh.n_samples:
                raise ValueError(f"channel {c}: xhat must be float32 [n_comp, n_samples]")
        _check(lib().sst_batch_set_io(self._h, c, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(_ptr(ridge)),
                                      int(n_comp), int(hw), ctypes.c_void_p(_ptr(xhat)),
                                      ctypes.c_void_p(_ptr(xref)), ctypes.c_void_p(_ptr(err))),
               "sst_batch_set_io")
        self._io[c] = (x, T, ridge, xhat, xref, err)

    def commit(self):
        _check(lib().sst_batch_commit(self._h, ctypes.c_void_p(_stream_handle(self.device))),
               "sst_batch_commit")

    def forward(self, c_begin: int = 0, c_end: Optional[int] = None, reuse_gamma: bool = False):
        c_end = self.n_channels if c_end is None else c_end
        _check(lib().sst_batch_forward(self._h, int(c_begin), int(c_end),
                                       SST_FWD_REUSE_GAMMA if reuse_gamma else 0,
                                       ctypes.c_void_p(_stream_handle(self.device))),
               "sst_batch_forward")

    def inverse(self, c_begin: int = 0, c_end: Optional[int] = None):
        c_end = self.n_channels if c_end is None else c_end
        _check(lib().sst_batch_inverse(self._h, int(c_begin), int(c_end),
                                       ctypes.c_void_p(_stream_handle(self.device))),
               "sst_batch_inverse")

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.sst_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
