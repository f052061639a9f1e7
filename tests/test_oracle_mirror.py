"""The oracle's mirror of the C ABI (host pointers, float storage, float64
arithmetic) against the oracle's own float64 functions, on the CPU.

The mirror only marshals: every number it returns must be the float64
pipeline's, rounded once to float.  Chunked calls must add up to the whole
call, and invalid arguments must come back as status codes.
"""
import numpy as np
import pytest

import oracle
from workloads import SSTConfig, make_chirp


def _case(hop=4, subdiv=2, thr_mode="rel", thr=1e-3, n=3000):
    fs = 1000.0
    x = (make_chirp(n, 60.0, 40.0, fs) + 0.5 * np.cos(2 * np.pi * 210.0 * np.arange(n) / fs)
         ).astype(np.float32)
    cfg = SSTConfig(fs=fs, win_len=127, sigma=16.0, hop=hop, nfft=256, f_lo=20.0, f_hi=400.0,
                    subdiv=subdiv, thr_mode=thr_mode, thr=thr, hw=6)
    return x, cfg


def relf(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
                 / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))


@pytest.mark.parametrize("hop,subdiv,thr_mode,thr", [(4, 2, "rel", 1e-3), (1, 1, "abs", 1e-2),
                                                     (7, 4, "rel", 1e-2)])
def test_mirror_forward_is_the_float64_pipeline_rounded(hop, subdiv, thr_mode, thr):
    x, cfg = _case(hop, subdiv, thr_mode, thr)
    mp = oracle.MirrorPlan(x.shape[0], cfg)
    ref = oracle.forward(x.astype(np.float64), cfg)
    assert (mp.k1, mp.k2, mp.n_src, mp.n_dst) == (ref.band.k1, ref.band.k2, ref.band.n_src,
                                                  ref.band.n_dst)
    assert mp.n_frames == -(-x.shape[0] // hop)
    T, aux = mp.forward(x, want_aux=True)
    assert aux["gamma"] == np.float32(ref.gamma)
    # one rounding of each float64 value, nothing else
    assert np.array_equal(T, ref.T.astype(np.complex64))
    assert np.array_equal(aux["S"], ref.S.astype(np.complex64))
    assert np.array_equal(aux["Sd"], ref.Sd.astype(np.complex64))
    assert np.array_equal(aux["idx"], ref.idx)
    cs = aux["colstats"]
    assert np.allclose(cs[:, 0], ref.T.real.sum(1), rtol=1e-12, atol=1e-12)
    assert np.allclose(cs[:, 1], ref.T.imag.sum(1), rtol=1e-12, atol=1e-12)
    assert np.allclose(cs[:, 2], (np.abs(ref.T) ** 2).sum(1), rtol=1e-12, atol=1e-12)


def test_mirror_chunks_equal_whole_call():
    x, cfg = _case()
    mp = oracle.MirrorPlan(x.shape[0], cfg)
    T, _ = mp.forward(x)
    a = mp.n_frames // 3
    T1, aux1 = mp.forward(x, 0, a)
    T2, aux2 = mp.forward(x, a, mp.n_frames - a)
    # gamma comes from every frame, whatever the chunk
    assert aux1["gamma"] == aux2["gamma"]
    assert np.array_equal(np.concatenate([T1, T2]), T)


def test_mirror_ridge_and_inverse_match_the_oracle():
    x, cfg = _case()
    n = x.shape[0]
    mp = oracle.MirrorPlan(n, cfg)
    T, _ = mp.forward(x)
    Td = T.astype(np.complex128)
    bands = [(0, mp.n_dst // 2), (mp.n_dst // 2, mp.n_dst - 1)]
    r = mp.ridge(T, bands)
    for q, (la, lb) in enumerate(bands):
        assert np.array_equal(r[q], oracle.ridge(Td, la, lb))
    g, _ = oracle.gaussian_windows(cfg.win_len, cfg.sigma)
    xh, _ = mp.inverse(T, r, cfg.hw)
    for q in range(2):
        ref = oracle.inverse(Td, r[q], cfg.hw, g, cfg.hop, cfg.nfft, mp.k1, cfg.subdiv, n)
        assert relf(xh[q], ref) < 1e-6
    # chunked calls with accumulation add up to the whole-signal call
    a = mp.n_frames // 2 + 3
    xa = np.zeros_like(xh)
    mp.inverse(T[:a], r[:, :a], cfg.hw, 0, xhat=xa, flags=oracle.MIRROR_INV_ACCUMULATE)
    mp.inverse(T[a:], np.ascontiguousarray(r[:, a:]), cfg.hw, a, xhat=xa,
               flags=oracle.MIRROR_INV_ACCUMULATE)
    assert relf(xa, xh) < 1e-6
    # reconstruction error sums over [M, N - M)
    xref = xh + 0.01
    _, err = mp.inverse(T, r, cfg.hw, xref=xref)
    M = (cfg.win_len - 1) // 2
    for q in range(2):
        d = xref[q, M:n - M].astype(np.float64) - xh[q, M:n - M]
        assert err[q, 0] == pytest.approx(np.sum(d * d), rel=1e-12)
        assert err[q, 1] == pytest.approx(np.sum(xref[q, M:n - M].astype(np.float64) ** 2),
                                          rel=1e-12)


def test_mirror_eq15_inverse():
    x, cfg = _case(hop=1, subdiv=1, thr_mode="rel", thr=1e-3, n=1200)
    mp = oracle.MirrorPlan(x.shape[0], cfg)
    T, _ = mp.forward(x)
    r = mp.ridge(T, [(0, mp.n_dst - 1)])
    g, _ = oracle.gaussian_windows(cfg.win_len, cfg.sigma)
    xh, _ = mp.inverse(T, r, cfg.hw, flags=oracle.MIRROR_INV_EQ15)
    ref = oracle.inverse_eq15(T.astype(np.complex128), r[0], cfg.hw, g[(cfg.win_len - 1) // 2],
                              cfg.nfft, mp.k1, cfg.subdiv)
    assert relf(xh[0], ref) < 1e-6


def test_mirror_errors_are_status_codes():
    x, cfg = _case()
    with pytest.raises(oracle.MirrorError) as e:
        oracle.MirrorPlan(x.shape[0], SSTConfig(**{**cfg.__dict__, "win_len": 128}))
    assert e.value.status == -1
    with pytest.raises(oracle.MirrorError):
        oracle.MirrorPlan(x.shape[0], SSTConfig(**{**cfg.__dict__, "f_hi": 600.0}))
    mp = oracle.MirrorPlan(x.shape[0], cfg)
    with pytest.raises(oracle.MirrorError):
        mp.forward(x, 0, mp.n_frames + 1)
    T, _ = mp.forward(x)
    r = mp.ridge(T, [(0, 10)])
    with pytest.raises(oracle.MirrorError):   # err needs a whole-signal call
        mp.inverse(T[:10], r[:, :10], cfg.hw, 0, xref=np.zeros((1, x.shape[0]), np.float32))
    with pytest.raises(oracle.MirrorError):   # Eq. 15 needs hop 1
        mp.inverse(T, r, cfg.hw, flags=oracle.MIRROR_INV_EQ15)
