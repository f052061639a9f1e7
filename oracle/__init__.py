"""Float64 CPU oracle of the downsampled SST and its direct inverse.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The GPU library never imports,
links or calls anything here, and this package never imports the GPU library.

Thin ctypes marshalling over ``sst_oracle.c``; every step of the arithmetic is
in the C file, which cites the passage of the paper each function follows.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import build as _build

_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I = ctypes.c_int
_I64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    srcs = _build.SRCS + [os.path.join(_build.HERE, "sst_oracle.h")]
    if not os.path.exists(_build.LIB) or (
            os.path.getmtime(_build.LIB) < max(os.path.getmtime(p) for p in srcs)):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    lib.sso_gaussian_windows.argtypes = [_I, ctypes.c_double, _D, _D]
    lib.sso_gaussian_windows.restype = _I
    lib.sso_band.argtypes = [ctypes.c_double, _I, ctypes.c_double, ctypes.c_double, _I,
                             ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                             ctypes.POINTER(_I)]
    lib.sso_band.restype = _I
    lib.sso_stft.argtypes = [_D, _I64, _D, _D, _I, _I, _I, _I, _I, _I64, _I64, _D, _D]
    lib.sso_stft.restype = None
    lib.sso_stft_maxabs.argtypes = [_D, _I64, _D, _I, _I, _I, _I, _I, _I64, _I64]
    lib.sso_stft_maxabs.restype = ctypes.c_double
    lib.sso_reassign.argtypes = [_D, _D, _I64, _I, _I, _I, _I, _I, ctypes.c_double, _D,
                                 _I32, _D]
    lib.sso_reassign.restype = None
    lib.sso_ridge.argtypes = [_D, _I64, _I, _I, _I, _I32]
    lib.sso_ridge.restype = None
    lib.sso_inverse.argtypes = [_D, _I64, _I, _I32, _I, _D, _I, _I, _I, _I, _I, _I64, _D]
    lib.sso_inverse.restype = None
    lib.sso_inverse_eq15.argtypes = [_D, _I64, _I, _I32, _I, ctypes.c_double, _I, _I, _I, _D]
    lib.sso_inverse_eq15.restype = None
    lib.sso_stft_synthesis.argtypes = [_D, _I64, _D, _I, _I, _I, _I64, _D]
    lib.sso_stft_synthesis.restype = None
    lib.sso_renyi.argtypes = [_D, _I64, _I64, ctypes.c_double]
    lib.sso_renyi.restype = ctypes.c_double
    lib.sso_num_threads.argtypes = []
    lib.sso_num_threads.restype = _I
    _F = ctypes.POINTER(ctypes.c_float)
    _V = ctypes.c_void_p
    lib.sst_oracle_plan.argtypes = [ctypes.POINTER(MirrorParams), ctypes.POINTER(_V)]
    lib.sst_oracle_plan.restype = ctypes.c_int32
    lib.sst_oracle_plan_query.argtypes = [_V, ctypes.POINTER(MirrorShape)]
    lib.sst_oracle_plan_query.restype = ctypes.c_int32
    lib.sst_oracle_forward.argtypes = [_V, _F, _I64, _I64, _F, _F, _F, _I32, _D, _F]
    lib.sst_oracle_forward.restype = ctypes.c_int32
    lib.sst_oracle_ridge.argtypes = [_V, _F, _I64, _I32, ctypes.c_int32, _I32]
    lib.sst_oracle_ridge.restype = ctypes.c_int32
    lib.sst_oracle_inverse.argtypes = [_V, _F, _I64, _I64, _I32, ctypes.c_int32, ctypes.c_int32,
                                       _F, _F, _D, ctypes.c_uint32]
    lib.sst_oracle_inverse.restype = ctypes.c_int32
    lib.sst_oracle_destroy.argtypes = [_V]
    lib.sst_oracle_destroy.restype = None
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _ip(a: np.ndarray):
    return a.ctypes.data_as(_I32)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def num_threads() -> int:
    return int(_load().sso_num_threads())


def gaussian_windows(win_len: int, sigma: float):
    """Sampled g and g' on j in [-M, M] (Gaussian window and its derivative)."""
    g = np.empty(win_len, dtype=np.float64)
    gd = np.empty(win_len, dtype=np.float64)
    if _load().sso_gaussian_windows(int(win_len), float(sigma), _dp(g), _dp(gd)) != 0:
        raise ValueError("window length must be odd and positive, sigma > 0")
    return g, gd


@dataclass(frozen=True)
class Band:
    k1: int
    k2: int
    n_src: int
    n_dst: int


def band(fs: float, nfft: int, f_lo: float, f_hi: float, subdiv: int) -> Band:
    k1, k2, ns, nd = _I(), _I(), _I(), _I()
    rc = _load().sso_band(float(fs), int(nfft), float(f_lo), float(f_hi), int(subdiv),
                          ctypes.byref(k1), ctypes.byref(k2), ctypes.byref(ns),
                          ctypes.byref(nd))
    if rc != 0:
        raise ValueError("invalid band")
    return Band(k1.value, k2.value, ns.value, nd.value)


def stft(x, g, gd, hop: int, nfft: int, k1: int, k2: int, frame0: int = 0,
         nframes: Optional[int] = None, want_sd: bool = True):
    """S and S' (complex128 [nframes, k2-k1+1]) by the direct sum of Eqs. 7-9."""
    x = _f64(x)
    g = _f64(g)
    gd = _f64(gd)
    n = x.shape[0]
    if nframes is None:
        nframes = -(-n // hop) - frame0
    n_src = k2 - k1 + 1
    S = np.empty((nframes, n_src), dtype=np.complex128)
    Sd = np.empty((nframes, n_src), dtype=np.complex128) if want_sd else None
    _load().sso_stft(_dp(x), n, _dp(g), _dp(gd), g.shape[0], int(hop), int(nfft), int(k1),
                     int(k2), int(frame0), int(nframes), _dp(S.view(np.float64)),
                     _dp(Sd.view(np.float64)) if want_sd else None)
    return S, Sd


def stft_maxabs(x, g, hop: int, nfft: int, k1: int, k2: int, frame0: int = 0,
                nframes: Optional[int] = None) -> float:
    x = _f64(x)
    g = _f64(g)
    n = x.shape[0]
    if nframes is None:
        nframes = -(-n // hop) - frame0
    return float(_load().sso_stft_maxabs(_dp(x), n, _dp(g), g.shape[0], int(hop), int(nfft),
                                         int(k1), int(k2), int(frame0), int(nframes)))


def reassign(S, Sd, nfft: int, k1: int, subdiv: int, n_dst: int, gamma: float):
    """T (complex128 [nframes, n_dst]), idx (int32) and frac (float64 u) of Eqs. 13, 27-29."""
    S = _c128(S)
    Sd = _c128(Sd)
    nframes, n_src = S.shape
    T = np.empty((nframes, n_dst), dtype=np.complex128)
    idx = np.empty((nframes, n_src), dtype=np.int32)
    frac = np.empty((nframes, n_src), dtype=np.float64)
    _load().sso_reassign(_dp(S.view(np.float64)), _dp(Sd.view(np.float64)), nframes, n_src,
                         int(nfft), int(k1), int(subdiv), int(n_dst), float(gamma),
                         _dp(T.view(np.float64)), _ip(idx), _dp(frac))
    return T, idx, frac


def ridge(T, la: int, lb: int) -> np.ndarray:
    T = _c128(T)
    nframes, n_dst = T.shape
    out = np.empty(nframes, dtype=np.int32)
    _load().sso_ridge(_dp(T.view(np.float64)), nframes, n_dst, int(la), int(lb), _ip(out))
    return out


def inverse(T, ridge_bins, hw: int, g, hop: int, nfft: int, k1: int, subdiv: int,
            n: int) -> np.ndarray:
    """Direct downsampled inverse (Eqs. 25-26) of one component; float64 [n]."""
    T = _c128(T)
    g = _f64(g)
    r = np.ascontiguousarray(np.asarray(ridge_bins, dtype=np.int32))
    nframes, n_dst = T.shape
    if r.shape[0] != nframes:
        raise ValueError("one ridge entry per frame")
    out = np.empty(n, dtype=np.float64)
    _load().sso_inverse(_dp(T.view(np.float64)), nframes, n_dst, _ip(r), int(hw), _dp(g),
                        g.shape[0], int(hop), int(nfft), int(k1), int(subdiv), int(n), _dp(out))
    return out


def inverse_eq15(T, ridge_bins, hw: int, g0: float, nfft: int, k1: int,
                 subdiv: int) -> np.ndarray:
    """Standard inverse SST for hop 1 (Eq. 15); float64 [nframes]."""
    T = _c128(T)
    r = np.ascontiguousarray(np.asarray(ridge_bins, dtype=np.int32))
    nframes, n_dst = T.shape
    out = np.empty(nframes, dtype=np.float64)
    _load().sso_inverse_eq15(_dp(T.view(np.float64)), nframes, n_dst, _ip(r), int(hw),
                             float(g0), int(nfft), int(k1), int(subdiv), _dp(out))
    return out


def stft_synthesis(S_full, g, hop: int, nfft: int, n: int) -> np.ndarray:
    """STFT synthesis of Eqs. 10-11 from all one-sided bins; float64 [n]."""
    S_full = _c128(S_full)
    g = _f64(g)
    nframes, nb = S_full.shape
    if nb != nfft // 2 + 1:
        raise ValueError("S must hold bins 0..N_f/2")
    out = np.empty(n, dtype=np.float64)
    _load().sso_stft_synthesis(_dp(S_full.view(np.float64)), nframes, _dp(g), g.shape[0],
                               int(hop), int(nfft), int(n), _dp(out))
    return out


def renyi(C, alpha: float = 3.0) -> float:
    """Renyi entropy (bits) of P = |C|^2 over the grid of C (Sec. 3, Eq. 32)."""
    C = _c128(C)
    if C.ndim == 1:
        C = C[None, :]
    return float(_load().sso_renyi(_dp(C.view(np.float64)), C.shape[0], C.shape[1],
                                   float(alpha)))


@dataclass
class OracleResult:
    band: Band
    gamma: float
    S: np.ndarray
    Sd: np.ndarray
    T: np.ndarray
    idx: np.ndarray
    frac: np.ndarray
    g: np.ndarray
    gd: np.ndarray


def forward(x, cfg, frame0: int = 0, nframes: Optional[int] = None,
            gamma: Optional[float] = None) -> OracleResult:
    """Whole forward pipeline (windows, band, threshold, STFT pair, reassignment).

    ``cfg`` is any object with the SSTConfig fields.  For a relative threshold,
    gamma = thr * max|S| over ALL frames of x unless ``gamma`` is given.
    """
    g, gd = gaussian_windows(cfg.win_len, cfg.sigma)
    b = band(cfg.fs, cfg.nfft, cfg.f_lo, cfg.f_hi, cfg.subdiv)
    if gamma is None:
        if cfg.thr_mode == "abs":
            gamma = float(cfg.thr)
        else:
            gamma = float(cfg.thr) * stft_maxabs(x, g, cfg.hop, cfg.nfft, b.k1, b.k2)
    S, Sd = stft(x, g, gd, cfg.hop, cfg.nfft, b.k1, b.k2, frame0, nframes)
    T, idx, frac = reassign(S, Sd, cfg.nfft, b.k1, cfg.subdiv, b.n_dst, gamma)
    return OracleResult(b, gamma, S, Sd, T, idx, frac, g, gd)


# ---------------------------------------------------------------------------
# Mirror of the GPU library's C ABI over host pointers (sst_oracle.h): the same
# calls, argument order and layouts, float storage, float64 arithmetic.
# ---------------------------------------------------------------------------
class MirrorParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_samples", ctypes.c_int64),
                ("fs", ctypes.c_double), ("win_len", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("window", ctypes.POINTER(ctypes.c_double)),
                ("dwindow", ctypes.POINTER(ctypes.c_double)), ("hop", ctypes.c_int32),
                ("nfft", ctypes.c_int32), ("f_lo", ctypes.c_double), ("f_hi", ctypes.c_double),
                ("subdiv", ctypes.c_int32), ("thr_mode", ctypes.c_int32), ("thr", ctypes.c_double),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class MirrorShape(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int64), ("n_frames", ctypes.c_int64),
                ("win_len", ctypes.c_int32), ("hop", ctypes.c_int32), ("nfft", ctypes.c_int32),
                ("subdiv", ctypes.c_int32), ("k1", ctypes.c_int32), ("k2", ctypes.c_int32),
                ("n_src", ctypes.c_int32), ("n_dst", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_size_t), ("t_row_bytes", ctypes.c_size_t)]


MIRROR_INV_ACCUMULATE = 1
MIRROR_INV_EQ15 = 2


class MirrorError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: oracle status {status}")
        self.status = status


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if a is not None else None


class MirrorPlan:
    """A plan of the oracle's mirror ABI; float32 numpy arrays in and out."""

    def __init__(self, n_samples: int, cfg):
        self._lib = _load()
        p = MirrorParams(ctypes.sizeof(MirrorParams), int(n_samples), float(cfg.fs),
                         int(cfg.win_len), float(cfg.sigma), None, None, int(cfg.hop),
                         int(cfg.nfft), float(cfg.f_lo), float(cfg.f_hi), int(cfg.subdiv),
                         0 if cfg.thr_mode == "abs" else 1, float(cfg.thr), 0, 0)
        h = ctypes.c_void_p()
        rc = self._lib.sst_oracle_plan(ctypes.byref(p), ctypes.byref(h))
        if rc != 0:
            raise MirrorError(rc, "sst_oracle_plan")
        self._h = h
        sh = MirrorShape()
        self._lib.sst_oracle_plan_query(h, ctypes.byref(sh))
        self.shape = sh
        self.n_frames, self.n_src, self.n_dst = sh.n_frames, sh.n_src, sh.n_dst
        self.k1, self.k2 = sh.k1, sh.k2

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.sst_oracle_destroy(h)
            self._h = None

    def forward(self, x, frame0: int = 0, nframes: Optional[int] = None, want_aux: bool = False):
        x = np.ascontiguousarray(x, dtype=np.float32)
        nframes = self.n_frames - frame0 if nframes is None else nframes
        T = np.empty((nframes, self.n_dst), dtype=np.complex64)
        aux = {}
        S = Sd = idx = cs = None
        if want_aux:
            S = np.empty((nframes, self.n_src), dtype=np.complex64)
            Sd = np.empty_like(S)
            idx = np.empty((nframes, self.n_src), dtype=np.int32)
            cs = np.empty((nframes, 3), dtype=np.float64)
        gam = np.zeros(1, dtype=np.float32)
        rc = self._lib.sst_oracle_forward(
            self._h, _fp(x), int(frame0), int(nframes), _fp(T.view(np.float32)),
            _fp(S.view(np.float32)) if S is not None else None,
            _fp(Sd.view(np.float32)) if Sd is not None else None,
            _ip(idx) if idx is not None else None, _dp(cs) if cs is not None else None, _fp(gam))
        if rc != 0:
            raise MirrorError(rc, "sst_oracle_forward")
        aux.update(gamma=float(gam[0]), S=S, Sd=Sd, idx=idx, colstats=cs)
        return T, aux

    def ridge(self, T, bands):
        T = np.ascontiguousarray(T, dtype=np.complex64)
        b = np.ascontiguousarray(np.asarray(bands, dtype=np.int32).ravel())
        nq = b.shape[0] // 2
        out = np.empty((nq, T.shape[0]), dtype=np.int32)
        rc = self._lib.sst_oracle_ridge(self._h, _fp(T.view(np.float32)), T.shape[0], _ip(b), nq,
                                        _ip(out))
        if rc != 0:
            raise MirrorError(rc, "sst_oracle_ridge")
        return out

    def inverse(self, T, ridge, hw: int, frame0: int = 0, xhat=None, xref=None,
                flags: int = 0):
        T = np.ascontiguousarray(T, dtype=np.complex64)
        r = np.ascontiguousarray(np.asarray(ridge, dtype=np.int32))
        if r.ndim == 1:
            r = r[None, :]
        nq = r.shape[0]
        if xhat is None:
            xhat = np.zeros((nq, self.shape.n_samples), dtype=np.float32)
        err = np.empty((nq, 2), dtype=np.float64) if xref is not None else None
        xr = np.ascontiguousarray(xref, dtype=np.float32) if xref is not None else None
        rc = self._lib.sst_oracle_inverse(self._h, _fp(T.view(np.float32)), int(frame0),
                                          T.shape[0], _ip(r), nq, int(hw), _fp(xhat), _fp(xr),
                                          _dp(err) if err is not None else None, int(flags))
        if rc != 0:
            raise MirrorError(rc, "sst_oracle_inverse")
        return xhat, err
