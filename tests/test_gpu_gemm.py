"""GPU: the DFT-as-GEMM precision tiers (BF16, FP16 hi/lo x3 on the matrix
cores) against the float64 oracle and against the FP32 FFT path, on c5-shaped
inputs (N_f 512 / 1024, L = N_f - 1, sigma = N_f / 8, H = 8, band [0, 6.4 kHz],
z = 1), on a band with k1 > 0 and z = 2, and on narrow bands at N_f 4096 and
8192 (L = N_f - 1).

Reported for every tier: relative Frobenius error of S, S' and T (T against
the oracle's coefficients re-scattered with the GPU's index decisions, and
raw), literal index mismatches, and the inverse SNR against the oracle's.
gamma is rho max |S| on the tier's own arithmetic (within rho times the
largest |dS| bound below of the oracle's); coefficients whose |S| lies
between the two thresholds may be retained by one side only.
Index rule of both tiers: a destination may differ from the oracle's only
where the tier's worst-case error bound of S and S' can move the oracle's
fractional destination across the rounding boundary (tests/parity.py):
|dS| <= (u_p + L 2^-24) sum_j |x w|, with u_p the relative error of one
product of rounded operands (FP16 x3: 2^-21; BF16, 8-bit significands:
2^-7) and L 2^-24 the FP32 accumulation over L taps.
Bars: the FP16 x3 tier meets the FP32 bars (relF <= 1e-5, SNR within 0.1 dB);
BF16: relF <= 1e-2, SNR within 1 dB.  The production kernel (no per-
coefficient outputs), which the benchmark times, gives T bit for bit equal to
the debug instantiation compared with the oracle."""
import math
import sys

import numpy as np
import pytest

import oracle
from tests.parity import classify_indices, reconciled_T, relf
from workloads import SSTConfig, make_c5, ridge_bins

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sst():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2003_07065_amd as m
    m.lib()
    return m


def _workloads():
    out = []
    for nfft in (512, 1024):
        w = make_c5(n_channels=1, n=1 << 15, nfft=nfft)[0]
        out.append((f"c5-{nfft}", w))
    w = make_c5(n_channels=1, n=20000, nfft=512)[0]
    w.cfg = SSTConfig(25600.0, 255, 32.0, 16, 512, 1000.0, 6000.0, 2, "rel", 1e-3, 2)
    out.append(("nf512-z2-k1", w))
    # narrow bands at long DFTs (the filter-bank use of the GEMM tiers):
    # N_f 4096 with [0, 1 kHz] and N_f 8192 with [0, 500 Hz], L = N_f - 1
    for nfft, f_hi in ((4096, 1000.0), (8192, 500.0)):
        w = make_c5(n_channels=1, n=1 << 14, nfft=nfft, f_hi=f_hi)[0]
        out.append((f"nf{nfft}-narrow", w))
    return out


WL = _workloads()


def _l1_norms(x, w, hop, frames):
    """sum_j |x[mH + j] w[j]| per frame (the scale of a dot product's rounding error)."""
    L = w.shape[0]
    M = (L - 1) // 2
    xp = np.concatenate([np.zeros(M), x.astype(np.float64), np.zeros(M + hop)])
    return np.array([np.sum(np.abs(xp[m * hop: m * hop + L] * w)) for m in frames])


@pytest.mark.parametrize("prec", ["f16x3", "bf16"])
@pytest.mark.parametrize("name,w", WL, ids=[n for n, _ in WL])
def test_gemm_tier_against_oracle(sst, name, w, prec):
    cfg = w.cfg
    x = w.x
    plan = sst.Plan.from_config(w.n, cfg, device="cuda", precision=prec)
    xg = torch.from_numpy(x).cuda()
    nfr = plan.n_frames
    S = torch.empty((nfr, plan.n_src), dtype=torch.complex64, device="cuda")
    Sd = torch.empty_like(S)
    idx = torch.empty((nfr, plan.n_src), dtype=torch.int32, device="cuda")
    gam = torch.empty(1, dtype=torch.float32, device="cuda")
    T = plan.forward(xg, S=S, Sd=Sd, idx=idx, gamma=gam)
    fft = sst.Plan.from_config(w.n, cfg, device="cuda")
    T32 = fft.forward(xg)
    torch.cuda.synchronize()
    o = oracle.forward(x.astype(np.float64), cfg)
    S_g, Sd_g, idx_g, T_g = S.cpu().numpy(), Sd.cpu().numpy(), idx.cpu().numpy(), T.cpu().numpy()
    e_s, e_sd = relf(S_g, o.S), relf(Sd_g, o.Sd)
    e_t = relf(T_g, reconciled_T(o.S, idx_g, plan.n_dst))
    e_raw, e_32 = relf(T_g, o.T), relf(T_g, T32.cpu().numpy())
    # index bound of this arithmetic: S and S' move by at most
    # (u_p + L 2^-24) sum_j |x w| per frame
    u = (2.0 ** -21 if prec == "f16x3" else 2.0 ** -7) + cfg.win_len * 2.0 ** -24
    frames = np.arange(nfr)
    err_s = u * _l1_norms(x, o.g, cfg.hop, frames)
    err_sd = u * _l1_norms(x, o.gd, cfg.hop, frames)
    # gamma = rho max |S| on the tier's own arithmetic: within rho times the
    # largest |dS| bound of the oracle's (and 1e-5 relative)
    gam_g = float(gam.cpu()[0])
    assert abs(gam_g - o.gamma) <= cfg.thr * err_s.max() + 1e-5 * o.gamma, (gam_g, o.gamma)
    rep, _ = classify_indices(idx_g, o.idx, o.frac, o.S, o.Sd, o.gamma, cfg.nfft, cfg.subdiv,
                              1.0, None, plan.n_dst, err_s=err_s, err_sd=err_sd, gamma_g=gam_g)
    # inverse with the true ridges, against the oracle's pipeline
    ridge = ridge_bins(w.inst_freq(w.frame_times()), cfg.fs, cfg.nfft, plan.k1, cfg.subdiv,
                       plan.n_dst)
    xh = plan.inverse(T, torch.from_numpy(ridge).cuda(), cfg.hw).cpu().numpy()
    M = (cfg.win_len - 1) // 2
    d_snr = []
    for q in range(ridge.shape[0]):
        xo = oracle.inverse(o.T, ridge[q], cfg.hw, o.g, cfg.hop, cfg.nfft, o.band.k1, cfg.subdiv,
                            w.n)
        ref = w.comps[q][M:w.n - M].astype(np.float64)
        s_g = 10 * math.log10(np.sum(ref ** 2) / np.sum((ref - xh[q][M:w.n - M]) ** 2))
        s_o = 10 * math.log10(np.sum(ref ** 2) / np.sum((ref - xo[M:w.n - M]) ** 2))
        d_snr.append(s_g - s_o)
    _say(f"[gemm {prec}] {name}: relF S={e_s:.2e} S'={e_sd:.2e} T(reconciled)={e_t:.2e} "
         f"T(raw)={e_raw:.2e} T-vs-FP32-FFT={e_32:.2e} dSNR={['%.3f' % d for d in d_snr]} {rep}")
    assert rep.ok(), (rep, rep.details)
    if prec == "f16x3":
        assert e_s <= 1e-5 and e_sd <= 1e-5 and e_t <= 1e-5
        assert max(abs(d) for d in d_snr) <= 0.1
    else:
        assert e_s <= 1e-2 and e_sd <= 1e-2 and e_t <= 1e-2
        assert max(abs(d) for d in d_snr) <= 1.0
    # the production kernel (the one the benchmark times) against the debug one,
    # with gamma reused, and in the whole-signal call with the speculative
    # threshold (seed, running maximum, fix-up of the tiles the final gamma
    # changes): the same gamma and the same T, bit for bit
    T_prod = plan.forward(xg, reuse_gamma=True)
    gam2 = torch.empty(1, dtype=torch.float32, device="cuda")
    T_spec = plan.forward(xg, gamma=gam2)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(T_prod), torch.view_as_real(T)), name
    assert float(gam2.cpu()[0]) == gam_g, name
    assert torch.equal(torch.view_as_real(T_spec), torch.view_as_real(T)), name


@pytest.mark.parametrize("prec", ["f16x3", "bf16"])
def test_gemm_tier_is_reproducible(sst, prec):
    name, w = WL[0]
    plan = sst.Plan.from_config(w.n, w.cfg, device="cuda", precision=prec)
    xg = torch.from_numpy(w.x).cuda()
    T1 = plan.forward(xg)
    T2 = plan.forward(xg, reuse_gamma=True)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(T1), torch.view_as_real(T2))


@pytest.mark.parametrize("prec", ["f16x3", "bf16"])
def test_gemm_speculative_threshold_fixup(sst, prec):
    """The whole-signal call of a GEMM tier thresholds speculatively (a seed of
    every 32nd tile, the running maximum, then the tiles the final gamma
    changes again).  Unit white noise with one impulse of 3000 in a tile the
    seed does not visit (tile 16 of 64-frame tiles): the tiles run before it
    keep coefficients the final gamma drops and must be redone.  T and gamma
    must equal, bit for bit, those of the debug call, whose gamma comes from a
    max-only pass over every tile first."""
    n = 1 << 18
    cfg = SSTConfig(25600.0, 511, 64.0, 8, 512, 0.0, 6400.0, 1, "rel", 1e-3, 1)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(n).astype(np.float32)
    x[(16 * 64 + 20) * cfg.hop] += 3000.0
    plan = sst.Plan.from_config(n, cfg, device="cuda", precision=prec)
    xg = torch.from_numpy(x).cuda()
    g1 = torch.empty(1, dtype=torch.float32, device="cuda")
    T1 = plan.forward(xg, gamma=g1)
    S = torch.empty((plan.n_frames, plan.n_src), dtype=torch.complex64, device="cuda")
    g2 = torch.empty(1, dtype=torch.float32, device="cuda")
    T2 = plan.forward(xg, S=S, gamma=g2)
    torch.cuda.synchronize()
    gm = float(g1.cpu()[0])
    _say(f"[gemm spec {prec}] gamma {gm:.6g} (debug {float(g2.cpu()[0]):.6g}), "
         f"max |S| {float(S.abs().max().cpu()):.6g}")
    assert float(g2.cpu()[0]) == gm
    assert abs(gm - 1e-3 * float(S.abs().max().cpu())) <= 1e-6 * gm
    assert torch.equal(torch.view_as_real(T1), torch.view_as_real(T2))
