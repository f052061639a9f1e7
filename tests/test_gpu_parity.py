"""GPU parity: the HIP library (through its C ABI) against the float64 oracle on
identical seeded float32 inputs.  Sizes keep the oracle to seconds while still
spanning many workgroup iterations and a ragged tail.  Rules: tests/parity.py."""
import math
import sys
import zlib

import numpy as np
import pytest

import oracle
from tests.parity import classify_indices, packed_norms, reconciled_T, relf, snr_db
from workloads import SSTConfig, make_c1, make_c2, make_tone

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


def _run_forward(sst, x, cfg, frame0=0, nframes=None, debug=True):
    plan = sst.Plan.from_config(x.shape[0], cfg, device="cuda")
    xg = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    if nframes is None:
        nframes = plan.n_frames - frame0
    out = dict(plan=plan, xg=xg)
    if debug:
        out["S"] = torch.empty((nframes, plan.n_src), dtype=torch.complex64, device="cuda")
        out["Sd"] = torch.empty_like(out["S"])
        out["idx"] = torch.empty((nframes, plan.n_src), dtype=torch.int32, device="cuda")
        out["col"] = torch.empty((nframes, 3), dtype=torch.float64, device="cuda")
    out["gamma"] = torch.empty(1, dtype=torch.float32, device="cuda")
    out["T"] = plan.forward(xg, None, frame0, nframes, S=out.get("S"), Sd=out.get("Sd"),
                            idx=out.get("idx"), colstats=out.get("col"), gamma=out["gamma"])
    torch.cuda.synchronize()
    return out


def _forward_parity(sst, x, cfg, frame0=0, nframes=None, label=""):
    _say(f"[parity] {label} N={x.shape[0]} nfft={cfg.nfft} L={cfg.win_len} hop={cfg.hop} "
         f"z={cfg.subdiv} band=[{cfg.f_lo},{cfg.f_hi}] frames={frame0}+{nframes}")
    g = _run_forward(sst, x, cfg, frame0, nframes)
    plan = g["plan"]
    nfr = g["T"].shape[0]
    o = oracle.forward(x.astype(np.float64), cfg, frame0, nfr)
    assert (o.band.k1, o.band.n_src, o.band.n_dst) == (plan.k1, plan.n_src, plan.n_dst)
    S_g = g["S"].cpu().numpy()
    Sd_g = g["Sd"].cpu().numpy()
    idx_g = g["idx"].cpu().numpy()
    T_g = g["T"].cpu().numpy()
    gam_g = float(g["gamma"].cpu().numpy()[0])
    # gamma (Eq. 13 threshold)
    assert abs(gam_g - o.gamma) <= 1e-5 * max(o.gamma, 1e-30) + 1e-30, (gam_g, o.gamma)
    # STFT pair (Eq. 9 and its g' version)
    e_s, e_sd = relf(S_g, o.S), relf(Sd_g, o.Sd)
    _say(f"  relF S={e_s:.2e} S'={e_sd:.2e}")
    assert e_s <= 1e-5 and e_sd <= 1e-5
    # destination indices
    s_pack = math.sqrt(np.sum(o.g ** 2) / max(np.sum(o.gd ** 2), 1e-300))
    ny = packed_norms(x, o.g, o.gd, s_pack, cfg.hop, np.arange(frame0, frame0 + nfr))
    rep, _ = classify_indices(idx_g, o.idx, o.frac, o.S, o.Sd, o.gamma, cfg.nfft, cfg.subdiv,
                              s_pack, ny, plan.n_dst)
    _say(f"  indices: {rep}")
    # per-coefficient STFT error in units of 2^-24 ||y_m|| (the index rule's error model)
    eun = np.abs(S_g - o.S) / (2.0 ** -24 * ny[:, None] + 1e-300)
    _say(f"  |dS|/(2^-24 |y|): rms {np.sqrt(np.mean(eun ** 2)):.2f} "
         f"p99.99 {np.quantile(eun, 0.9999):.2f} max {eun.max():.2f}")
    assert rep.ok(), (rep, rep.details)
    # T after reconciling index decisions (Eq. 28 with the GPU's rounding decisions)
    T_rec = reconciled_T(o.S, idx_g, plan.n_dst)
    e_t = relf(T_g, T_rec)
    _say(f"  relF T reconciled={e_t:.2e} raw={relf(T_g, o.T):.2e}")
    assert e_t <= 1e-5
    # FP64 column sums of T (conservation of every retained coefficient)
    col = g["col"].cpu().numpy()
    ref = T_rec.sum(axis=1)
    scale = np.abs(o.S).sum(axis=1) + 1e-30
    assert np.all(np.abs(col[:, 0] + 1j * col[:, 1] - ref) <= 1e-5 * scale)
    assert np.allclose(col[:, 2], (np.abs(T_g.astype(np.complex128)) ** 2).sum(axis=1),
                       rtol=1e-9, atol=1e-30)
    return g, o


# (name, N, SSTConfig) -- every DFT size, every pass-1 pruning (4, 8, 16 rows),
# bands with k1 > 0, non power-of-two z, hops from 1 to 32, histogram chunking
CASES = [
    ("c2-shape", 1 << 15, SSTConfig(25600.0, 1023, 128.0, 16, 4096, 0.0, 6400.0, 4, "rel", 1e-3, 6)),
    ("c3-shape", 1 << 16, SSTConfig(25600.0, 2047, 256.0, 32, 8192, 0.0, 5000.0, 8, "rel", 1e-3, 26)),
    ("nf1024-F4", 10007, SSTConfig(25600.0, 255, 32.0, 8, 1024, 0.0, 6400.0, 2, "rel", 1e-3, 2)),
    ("nf512-F8-nz16", 20011, SSTConfig(25600.0, 511, 64.0, 8, 512, 0.0, 6400.0, 1, "rel", 1e-3, 1)),
    ("nf2048-z3-k1", 12345, SSTConfig(25600.0, 1023, 100.0, 5, 2048, 300.0, 5000.0, 3, "rel", 1e-3, 4)),
    ("nf4096-nz8-abs", 9001, SSTConfig(8000.0, 1801, 200.0, 7, 4096, 100.0, 4000.0, 2, "abs", 1e-2, 3)),
    ("nf8192-nz16", 30000, SSTConfig(25600.0, 8191, 900.0, 64, 8192, 1000.0, 3000.0, 5, "rel", 1e-4, 8)),
]


def _signal(name, n, fs, seed=0):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    t = np.arange(n) / fs
    x = (np.cos(2 * np.pi * (0.11 * fs * t + 0.02 * fs * t * t / max(t[-1], 1e-9)))
         + 0.5 * np.cos(2 * np.pi * 0.05 * fs * t) + 0.3 * rng.standard_normal(n))
    return x.astype(np.float32)


@pytest.mark.parametrize("name,n,cfg", CASES, ids=[c[0] for c in CASES])
def test_forward_parity(sst, name, n, cfg):
    x = _signal(name, n, cfg.fs)
    _forward_parity(sst, x, cfg, label=name)


def test_forward_c1_workload(sst):
    """The plain standard SST workload (hop 1, full band, N_f = N = 4096)."""
    w = make_c1()
    _forward_parity(sst, w.x, w.cfg, label="c1")


def test_forward_partial_frames(sst):
    """A chunk in the middle of the signal: gamma still comes from every frame."""
    w = make_c2(n=1 << 15)
    _forward_parity(sst, w.x, w.cfg, frame0=777, nframes=301, label="c2-chunk")


def test_forward_chunks_equal_whole(sst):
    """Chunked calls equal the whole-signal call bit for bit: the first chunk
    computes gamma with the max-only pre-pass, the whole call speculatively,
    both on the forward kernel's own arithmetic."""
    w = make_c2(n=1 << 14)
    plan = sst.Plan.from_config(w.n, w.cfg, device="cuda")
    xg = torch.from_numpy(w.x).cuda()
    g1 = torch.empty(1, dtype=torch.float32, device="cuda")
    g2 = torch.empty_like(g1)
    T = plan.forward(xg, gamma=g1)
    parts = []
    f0 = 0
    for cnt in (100, 257, plan.n_frames - 357):
        parts.append(plan.forward(xg, None, f0, cnt, reuse_gamma=f0 > 0,
                                  gamma=g2 if f0 == 0 else None))
        f0 += cnt
    T2 = torch.cat(parts)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    assert torch.equal(torch.view_as_real(T2), torch.view_as_real(T))


@pytest.mark.parametrize("n", [1, 100, 300])
def test_forward_tiny_signals(sst, n):
    """Signals shorter than the window: every frame is mostly zero padding."""
    cfg = SSTConfig(1000.0, 511, 40.0, 7, 512, 0.0, 500.0, 2, "rel", 1e-3, 2)
    x = _signal(f"tiny{n}", n, cfg.fs)
    _forward_parity(sst, x, cfg, label=f"tiny{n}")


def test_forward_zero_signal(sst):
    """All-zero input: gamma = 0, nothing is retained, T is all zeros."""
    cfg = SSTConfig(1000.0, 255, 20.0, 4, 1024, 0.0, 500.0, 2, "rel", 1e-3, 2)
    g = _run_forward(sst, np.zeros(5000, np.float32), cfg)
    assert float(g["gamma"].cpu()[0]) == 0.0
    assert torch.count_nonzero(g["T"]).item() == 0
    assert bool((g["idx"] == -1).all())


# ---------------------------------------------------------------------------
# Inverse
# ---------------------------------------------------------------------------

def _ridges_from_if(w, plan):
    from workloads import ridge_bins
    f = w.inst_freq(w.frame_times())
    return ridge_bins(f, w.cfg.fs, w.cfg.nfft, plan.k1, w.cfg.subdiv, plan.n_dst)


@pytest.mark.parametrize("tf", [1, 4])
@pytest.mark.parametrize("which", ["c2-small", "c1"])
def test_inverse_on_identical_T(sst, which, tf):
    """Eqs. 25-26 on the same T (oracle T rounded to complex64): elementwise parity,
    with one and with four groups of 256 output samples per workgroup."""
    w = make_c2(n=1 << 15) if which == "c2-small" else make_c1()
    c = w.cfg
    _say(f"[inverse] {which} tf={tf}")
    o = oracle.forward(w.x.astype(np.float64), c)
    plan = sst.Plan.from_config(w.n, c, device="cuda")
    if which == "c1" and tf == 4:
        # hop 1: the 1278 frames of 1024 samples exceed one staged block
        with pytest.raises(sst.SSTError) as e:
            plan.set_tuning(inv_tf=tf)
        assert e.value.status == sst.SST_E_UNSUPPORTED
        return
    plan.set_tuning(inv_tf=tf)
    T32 = o.T.astype(np.complex64)
    ridge = _ridges_from_if(w, plan)
    xh_g = plan.inverse(torch.from_numpy(T32).cuda(), torch.from_numpy(ridge).cuda(), c.hw)
    xh_g = xh_g.cpu().numpy()
    for q in range(ridge.shape[0]):
        xo = oracle.inverse(T32.astype(np.complex128), ridge[q], c.hw, o.g, c.hop, c.nfft,
                            o.band.k1, c.subdiv, w.n)
        e = relf(xh_g[q], xo)
        _say(f"  comp {q}: relF xhat = {e:.2e}")
        assert e <= 1e-5


def test_inverse_pipeline_snr(sst):
    """GPU pipeline vs oracle pipeline: output SNR (Eq. 33) within 0.1 dB per component,
    and the GPU's FP64 error reduction equals the host sum."""
    w = make_c2(n=1 << 15)
    c = w.cfg
    o = oracle.forward(w.x.astype(np.float64), c)
    plan = sst.Plan.from_config(w.n, c, device="cuda")
    xg = torch.from_numpy(w.x).cuda()
    T = plan.forward(xg)
    ridge = _ridges_from_if(w, plan)
    rg = torch.from_numpy(ridge).cuda()
    xref = torch.from_numpy(w.comps.astype(np.float32)).cuda()
    err = torch.zeros((ridge.shape[0], 2), dtype=torch.float64, device="cuda")
    xh = plan.inverse(T, rg, c.hw, xref=xref, err=err).cpu().numpy()
    err = err.cpu().numpy()
    M = (c.win_len - 1) // 2
    for q in range(ridge.shape[0]):
        xo = oracle.inverse(o.T, ridge[q], c.hw, o.g, c.hop, c.nfft, o.band.k1, c.subdiv, w.n)
        ref = w.comps[q].astype(np.float32).astype(np.float64)
        s_g = snr_db(ref, xh[q], M, w.n - M)
        s_o = snr_db(ref, xo, M, w.n - M)
        _say(f"  comp {q}: SNR gpu {s_g:.3f} dB oracle {s_o:.3f} dB")
        assert abs(s_g - s_o) <= 0.1
        d = ref[M:w.n - M] - xh[q][M:w.n - M].astype(np.float64)
        assert abs(err[q, 0] - np.sum(d * d)) <= 1e-9 * np.sum(d * d)
        assert abs(err[q, 1] - np.sum(ref[M:w.n - M] ** 2)) <= 1e-9 * np.sum(ref[M:w.n - M] ** 2)


INV_CASES = [CASES[2], CASES[4], CASES[1], CASES[6],
             ("hop512", 50000, SSTConfig(25600.0, 1023, 128.0, 512, 4096, 0.0, 6400.0, 4, "rel",
                                         1e-3, 6))]


@pytest.mark.parametrize("name,n,cfg", INV_CASES,
                         ids=["nf1024", "nf2048-z3-k1", "c3-shape", "nf8192-L8191-H64", "hop512"])
def test_inverse_configs(sst, name, n, cfg):
    """Inverse parity on identical T across DFT sizes, non power-of-two z, k1 > 0,
    tiles whose frames span several staged blocks (hop 5, and L 8191 with hop 64)
    and window tables too large to decimate by the hop (L 8191 with hop 64, and
    hop 512), which take the clamped window gather."""
    x = _signal(name, n, cfg.fs)
    o = oracle.forward(x.astype(np.float64), cfg)
    plan = sst.Plan.from_config(n, cfg, device="cuda")
    T32 = o.T.astype(np.complex64)
    rng = np.random.default_rng(1)
    nfr = plan.n_frames
    # a wandering ridge, some frames without a ridge, one ridge at the band edge
    base = rng.integers(0, plan.n_dst, size=3)
    ridge = np.stack([(base[q] + (np.arange(nfr) // 17) % 5) % plan.n_dst for q in range(3)])
    ridge[1, ::7] = -1
    ridge[2, :] = plan.n_dst - 1
    ridge = ridge.astype(np.int32)
    xh = plan.inverse(torch.from_numpy(T32).cuda(), torch.from_numpy(ridge).cuda(),
                      cfg.hw).cpu().numpy()
    for q in range(3):
        xo = oracle.inverse(T32.astype(np.complex128), ridge[q], cfg.hw, o.g, cfg.hop, cfg.nfft,
                            o.band.k1, cfg.subdiv, n)
        e = relf(xh[q], xo)
        _say(f"  {name} comp {q}: relF xhat = {e:.2e}")
        assert e <= 1e-5


def test_inverse_chunks_accumulate(sst):
    w = make_c2(n=1 << 14)
    c = w.cfg
    plan = sst.Plan.from_config(w.n, c, device="cuda")
    xg = torch.from_numpy(w.x).cuda()
    T = plan.forward(xg)
    ridge = torch.from_numpy(_ridges_from_if(w, plan)).cuda()
    whole = plan.inverse(T, ridge, c.hw)
    acc = torch.zeros_like(whole)
    f0 = 0
    for cnt in (311, 200, plan.n_frames - 511):
        plan.inverse(T[f0:f0 + cnt].contiguous(), ridge[:, f0:f0 + cnt].contiguous(), c.hw,
                     xhat=acc, frame0=f0, nframes=cnt, accumulate=True)
        f0 += cnt
    torch.cuda.synchronize()
    assert relf(acc.cpu().numpy(), whole.cpu().numpy()) < 1e-6


def test_inverse_eq15_matches_oracle(sst):
    """Eq. 15 (hop 1) on identical T."""
    w = make_c1()
    c = w.cfg
    o = oracle.forward(w.x.astype(np.float64), c)
    plan = sst.Plan.from_config(w.n, c, device="cuda")
    T32 = o.T.astype(np.complex64)
    ridge = _ridges_from_if(w, plan)
    xh = plan.inverse(torch.from_numpy(T32).cuda(), torch.from_numpy(ridge).cuda(), c.hw,
                      eq15=True).cpu().numpy()
    for q in range(ridge.shape[0]):
        xo = oracle.inverse_eq15(T32.astype(np.complex128), ridge[q], c.hw, o.g[(c.win_len - 1) // 2],
                                 c.nfft, o.band.k1, c.subdiv)
        assert relf(xh[q], xo) <= 1e-6


def test_inverse_tone_unit_gain(sst):
    """Clean tone at a destination-bin centre: the GPU pipeline returns it at >= 60 dB."""
    cfg = SSTConfig(25600.0, 1023, 128.0, 16, 4096, 0.0, 6400.0, 4, "rel", 1e-3, 6)
    n = 1 << 15
    l0 = 4 * 19 + 1
    x = make_tone(n, (l0 / 4) * cfg.fs / cfg.nfft, cfg.fs, amp=0.8, phase=0.3)
    plan = sst.Plan.from_config(n, cfg, device="cuda")
    T = plan.forward(torch.from_numpy(x.astype(np.float32)).cuda())
    ridge = torch.full((1, plan.n_frames), l0, dtype=torch.int32, device="cuda")
    xh = plan.inverse(T, ridge, cfg.hw).cpu().numpy()[0]
    M = (cfg.win_len - 1) // 2
    assert snr_db(x, xh, M, n - M) > 60.0


# ---------------------------------------------------------------------------
# Ridge
# ---------------------------------------------------------------------------

def test_ridge_matches_oracle(sst):
    w = make_c2(n=1 << 15)
    o = oracle.forward(w.x.astype(np.float64), w.cfg)
    plan = sst.Plan.from_config(w.n, w.cfg, device="cuda")
    T32 = o.T.astype(np.complex64)
    bands = [(60, 100), (140, 170), (370, 400), (0, plan.n_dst - 1)]
    r_g = plan.ridge(torch.from_numpy(T32).cuda(), bands).cpu().numpy()
    mag = np.abs(T32.astype(np.complex128)) ** 2
    for q, (la, lb) in enumerate(bands):
        r_o = oracle.ridge(T32.astype(np.complex128), la, lb)
        diff = np.nonzero(r_g[q] != r_o)[0]
        for m in diff:   # only near-ties may differ (FP32 vs FP64 |T|^2)
            a, b = mag[m, r_g[q][m]], mag[m, r_o[m]]
            assert abs(a - b) <= 1e-6 * max(a, b)
        assert len(diff) <= 2


def test_ridge_guided_matches_oracle(sst):
    """Ridges searched around a per-frame guide bin (sst_ridge_guided): the
    oracle's ridge of each frame's own band, frames without a guide give -1, and
    bands reaching past either end of the grid are clipped."""
    w = make_c2(n=1 << 15)
    o = oracle.forward(w.x.astype(np.float64), w.cfg)
    plan = sst.Plan.from_config(w.n, w.cfg, device="cuda")
    T32 = o.T.astype(np.complex64)
    nfr = T32.shape[0]
    rng = np.random.default_rng(7)
    centre = np.stack([
        np.full(nfr, 80, dtype=np.int32),
        rng.integers(0, plan.n_dst, nfr).astype(np.int32),     # clipped at both ends
        np.where(np.arange(nfr) % 5 == 0, -1, 385).astype(np.int32)])
    rel = [(-12, 12), (-30, 30), (-3, 9)]
    r_g = plan.ridge(torch.from_numpy(T32).cuda(), rel,
                     centre=torch.from_numpy(centre).cuda()).cpu().numpy()
    T64 = T32.astype(np.complex128)
    mag = np.abs(T64) ** 2
    for q, (a, b) in enumerate(rel):
        for m in range(nfr):
            c = int(centre[q, m])
            if c < 0:
                assert r_g[q, m] == -1
                continue
            la, lb = max(c + a, 0), min(c + b, plan.n_dst - 1)
            r_o = int(oracle.ridge(T64[m:m + 1], la, lb)[0])
            if r_g[q, m] != r_o:   # only near-ties may differ (FP32 vs FP64 |T|^2)
                assert la <= r_g[q, m] <= lb
                x, y = mag[m, r_g[q, m]], mag[m, r_o]
                assert abs(x - y) <= 1e-6 * max(x, y), (q, m)


def test_reuse_gamma_needs_a_threshold_since_bind(sst):
    """SST_FWD_REUSE_GAMMA before any thresholding call on a binding (fresh, or
    after a rebind) is refused with SST_E_STATE instead of thresholding against
    an unset control block."""
    cfg = CASES[2][2]
    x = torch.from_numpy(_signal("reuse", 10007, cfg.fs)).cuda()
    plan = sst.Plan.from_config(10007, cfg, device="cuda")
    with pytest.raises(sst.SSTError) as e:
        plan.forward(x, None, 0, 16, reuse_gamma=True)
    assert e.value.status == sst.SST_E_STATE
    T = plan.forward(x)
    Tc = plan.forward(x, None, 5, 16, reuse_gamma=True)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(Tc), torch.view_as_real(T[5:21]))
    plan.bind("cuda")
    with pytest.raises(sst.SSTError) as e:
        plan.forward(x, None, 0, 16, reuse_gamma=True)
    assert e.value.status == sst.SST_E_STATE


TUNE = [
    ("c2-shape", 1 << 15, CASES[0][2]),
    ("c3-short", 12345, SSTConfig(25600.0, 2047, 256.0, 32, 8192, 0.0, 5000.0, 8, "rel", 1e-3, 26)),
]


@pytest.mark.parametrize("name,n,cfg", TUNE, ids=[c[0] for c in TUNE])
def test_tuned_choices_give_identical_T(sst, name, n, cfg):
    """Every forward launch choice the autotuner may pick (resident workgroups per
    CU, threshold seed step) gives T bit for bit equal to the default choice."""
    x = torch.from_numpy(_signal(name, n, cfg.fs)).cuda()
    plan = sst.Plan.from_config(n, cfg, device="cuda")
    occ = plan.get_tuning()["fwd_wg_per_cu"]
    assert occ >= 1
    T0 = plan.forward(x)
    for wg in range(1, occ + 1):
        for seed in (0, 1, 16, 128):
            plan.set_tuning(fwd_wg_per_cu=wg, seed_step=seed)
            T = plan.forward(x)
            torch.cuda.synchronize()
            assert torch.equal(torch.view_as_real(T), torch.view_as_real(T0)), (wg, seed)


def test_autotune_keeps_parity(sst):
    """sst_autotune picks choices on the caller's buffers; the forward afterwards
    equals the default one bit for bit and the tuned inverse matches the oracle."""
    w = make_c2(n=1 << 15)
    c = w.cfg
    plan = sst.Plan.from_config(w.n, c, device="cuda")
    xg = torch.from_numpy(w.x).cuda()
    T0 = plan.forward(xg)
    ridge = torch.from_numpy(_ridges_from_if(w, plan)).cuda()
    xh = torch.empty((ridge.shape[0], w.n), dtype=torch.float32, device="cuda")
    T = torch.empty_like(T0)
    best = plan.autotune(xg, T, ridge, c.hw, xh, reps=2)
    _say(f"  autotuned: {best}")
    assert best == plan.get_tuning()
    T1 = plan.forward(xg)
    xh1 = plan.inverse(T1, ridge, c.hw)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(T1), torch.view_as_real(T0))
    o = oracle.forward(w.x.astype(np.float64), c)
    T1c = T1.cpu().numpy().astype(np.complex128)
    r = ridge.cpu().numpy()
    for q in range(r.shape[0]):
        xo = oracle.inverse(T1c, r[q], c.hw, o.g, c.hop, c.nfft, o.band.k1, c.subdiv, w.n)
        assert relf(xh1[q].cpu().numpy(), xo) <= 1e-5


REPRO = [
    ("c2-shape", 1 << 15, CASES[0][2]),
    ("c3-short", 12345, SSTConfig(25600.0, 2047, 256.0, 32, 8192, 0.0, 5000.0, 8, "rel", 1e-3, 26)),
    ("nf1024-F4", 10007, CASES[2][2]),
]


@pytest.mark.parametrize("name,n,cfg", REPRO, ids=[c[0] for c in REPRO])
def test_forward_is_bitwise_reproducible(sst, name, n, cfg):
    """T does not depend on the order in which waves and workgroups run: every
    workgroup's first frame included (the staged tables are read after the
    barrier that completes them)."""
    x = torch.from_numpy(_signal(name, n, cfg.fs)).cuda()
    plan = sst.Plan.from_config(n, cfg, device="cuda")
    ref = plan.forward(x)
    for k in range(4):
        T = torch.full_like(ref, float("nan"))
        plan.forward(x, T, reuse_gamma=True)
        torch.cuda.synchronize()
        same = torch.equal(torch.view_as_real(T), torch.view_as_real(ref))
        _say(f"[repro] {name} run {k}: equal={same}")
        assert same


def test_c2_full_size_sampled(sst):
    """The headline workload at full size (N = 2^20, 65,536 frames) in the launch
    configuration bench.py times: gamma over every frame, sampled T rows (start,
    middle, end) under the parity rules, and the inverse of a sampled output
    range against the oracle on identical T."""
    from workloads import make_c2, ridge_bins
    w = make_c2()
    cfg = w.cfg
    plan = sst.Plan.from_config(w.n, cfg, device="cuda")
    xg = torch.from_numpy(w.x).cuda()
    gam = torch.empty(1, dtype=torch.float32, device="cuda")
    T = plan.forward(xg, gamma=gam)            # the timed kernel variant (no debug outputs)
    torch.cuda.synchronize()
    x64 = w.x.astype(np.float64)
    g_o, gd_o = oracle.gaussian_windows(cfg.win_len, cfg.sigma)
    b = oracle.band(cfg.fs, cfg.nfft, cfg.f_lo, cfg.f_hi, cfg.subdiv)
    gamma_o = cfg.thr * oracle.stft_maxabs(x64, g_o, cfg.hop, cfg.nfft, b.k1, b.k2)
    g_g = float(gam.cpu()[0])
    _say(f"[full c2] gamma gpu={g_g:.9g} oracle={gamma_o:.9g}")
    assert abs(g_g - gamma_o) <= 1e-5 * gamma_o
    s_pack = math.sqrt(np.sum(g_o ** 2) / np.sum(gd_o ** 2))
    for f0 in (0, plan.n_frames // 2 - 32, plan.n_frames - 64):
        nfr = 64
        S = torch.empty((nfr, plan.n_src), dtype=torch.complex64, device="cuda")
        idx = torch.empty((nfr, plan.n_src), dtype=torch.int32, device="cuda")
        Td = plan.forward(xg, None, f0, nfr, S=S, idx=idx, reuse_gamma=True)
        torch.cuda.synchronize()
        rows = T[f0:f0 + nfr]
        assert torch.equal(torch.view_as_real(Td), torch.view_as_real(rows)), f0
        o = oracle.forward(x64, cfg, f0, nfr, gamma=gamma_o)
        idx_g = idx.cpu().numpy()
        ny = packed_norms(w.x, g_o, gd_o, s_pack, cfg.hop, np.arange(f0, f0 + nfr))
        rep, _ = classify_indices(idx_g, o.idx, o.frac, o.S, o.Sd, o.gamma, cfg.nfft,
                                  cfg.subdiv, s_pack, ny, plan.n_dst)
        e_s = relf(S.cpu().numpy(), o.S)
        e_t = relf(rows.cpu().numpy(), reconciled_T(o.S, idx_g, plan.n_dst))
        _say(f"  frames {f0}+{nfr}: relF S={e_s:.2e} T(reconciled)={e_t:.2e} {rep}")
        assert e_s <= 1e-5 and e_t <= 1e-5 and rep.ok(), (rep, rep.details)
    # inverse of output samples [a, b) needs only the frames whose windows reach them:
    # the oracle gets the GPU's T on those frames and zeros elsewhere
    ridge = ridge_bins(w.inst_freq(w.frame_times()), cfg.fs, cfg.nfft, plan.k1, cfg.subdiv,
                       plan.n_dst)
    xh = plan.inverse(T, torch.from_numpy(ridge).cuda(), cfg.hw).cpu().numpy()
    M = (cfg.win_len - 1) // 2
    a, bnd = w.n // 2, w.n // 2 + 4096
    m_lo, m_hi = (a - M) // cfg.hop, (bnd + M) // cfg.hop + 1
    T64 = np.zeros((plan.n_frames, plan.n_dst), dtype=np.complex128)
    T64[m_lo:m_hi + 1] = T[m_lo:m_hi + 1].cpu().numpy()
    for q in range(ridge.shape[0]):
        xo = oracle.inverse(T64, ridge[q], cfg.hw, g_o, cfg.hop, cfg.nfft, plan.k1, cfg.subdiv, w.n)
        e = relf(xh[q, a:bnd], xo[a:bnd])
        _say(f"  inverse comp {q}: relF on samples [{a}, {bnd}) = {e:.2e}")
        assert e <= 1e-5


def test_c3_full_size_sampled(sst):
    """The long run-up workload at full size: N = 2^26 samples, 2,097,152 frames,
    T = 214.8 GB resident in HBM.  The oracle's gamma over every frame is out of
    reach (about 7e12 multiply-adds), so gamma is checked at the c3 shape above and
    here only for what any size must satisfy (gamma / rho >= |S| on every sampled
    frame); sampled blocks of frames are then compared with the oracle run with the
    GPU's gamma, and the inverse of a sampled output range with the oracle on the
    frames that reach it (a shifted sub-problem whose interior is exact)."""
    from workloads import make_c3, ridge_bins
    torch.cuda.empty_cache()
    w = make_c3()
    cfg = w.cfg
    comps = w.comps
    plan = sst.Plan.from_config(w.n, cfg, device="cuda")
    _say(f"[full c3] N={w.n} frames={plan.n_frames} n_dst={plan.n_dst} "
         f"T={plan.n_frames * plan.n_dst * 8 / 1e9:.1f} GB")
    xg = torch.from_numpy(w.x).cuda()
    gam = torch.empty(1, dtype=torch.float32, device="cuda")
    T = plan.forward(xg, gamma=gam)
    torch.cuda.synchronize()
    gamma_g = float(gam.cpu()[0])
    x64 = w.x.astype(np.float64)
    g_o, gd_o = oracle.gaussian_windows(cfg.win_len, cfg.sigma)
    s_pack = math.sqrt(np.sum(g_o ** 2) / np.sum(gd_o ** 2))
    nfr = 16
    for f0 in (0, plan.n_frames // 2 - 8, plan.n_frames - nfr):
        S = torch.empty((nfr, plan.n_src), dtype=torch.complex64, device="cuda")
        idx = torch.empty((nfr, plan.n_src), dtype=torch.int32, device="cuda")
        Td = plan.forward(xg, None, f0, nfr, S=S, idx=idx, reuse_gamma=True)
        torch.cuda.synchronize()
        rows = T[f0:f0 + nfr]
        assert torch.equal(torch.view_as_real(Td), torch.view_as_real(rows)), f0
        o = oracle.forward(x64, cfg, f0, nfr, gamma=gamma_g)
        assert np.abs(o.S).max() <= gamma_g / cfg.thr * (1 + 1e-5)
        idx_g = idx.cpu().numpy()
        ny = packed_norms(w.x, g_o, gd_o, s_pack, cfg.hop, np.arange(f0, f0 + nfr))
        rep, _ = classify_indices(idx_g, o.idx, o.frac, o.S, o.Sd, o.gamma, cfg.nfft,
                                  cfg.subdiv, s_pack, ny, plan.n_dst)
        e_s = relf(S.cpu().numpy(), o.S)
        e_t = relf(rows.cpu().numpy(), reconciled_T(o.S, idx_g, plan.n_dst))
        _say(f"  frames {f0}+{nfr}: relF S={e_s:.2e} T(reconciled)={e_t:.2e} {rep}")
        assert e_s <= 1e-5 and e_t <= 1e-5 and rep.ok(), (rep, rep.details)
    # inverse of every harmonic; output samples [a, a + 4096) of the middle
    ridge = ridge_bins(w.inst_freq(w.frame_times()), cfg.fs, cfg.nfft, plan.k1, cfg.subdiv,
                       plan.n_dst)
    xh = plan.inverse(T, torch.from_numpy(ridge).cuda(), cfg.hw)
    torch.cuda.synchronize()
    M = (cfg.win_len - 1) // 2
    H = cfg.hop
    a = (w.n // 2) // H * H
    b = a + 4096
    m_lo = (a - M) // H - 1
    m_hi = (b + M) // H + 1
    T_sub = T[m_lo:m_hi + 1].cpu().numpy().astype(np.complex128)
    n_sub = (m_hi - m_lo) * H + 1
    sl = slice(a - m_lo * H, b - m_lo * H)
    xh_g = xh[:, a:b].cpu().numpy()
    del T, xh
    torch.cuda.empty_cache()
    for q in range(ridge.shape[0]):
        xo = oracle.inverse(T_sub, np.ascontiguousarray(ridge[q, m_lo:m_hi + 1]), cfg.hw, g_o,
                            H, cfg.nfft, plan.k1, cfg.subdiv, n_sub)
        e = relf(xh_g[q], xo[sl])
        ref = comps[q][a:b]
        snr = 10 * math.log10(np.sum(ref ** 2) / np.sum((ref - xh_g[q]) ** 2))
        _say(f"  harmonic {q + 1}: inverse relF on [{a}, {b}) = {e:.2e}, SNR there {snr:.1f} dB")
        assert e <= 1e-5


def test_speculative_threshold_fixup(sst):
    """The speculative forward with a large fix-up pass.  Unit white noise plus
    one impulse of 15000 at the centre of frame 8208 (N = 2^18, the c2
    configuration, one frame per item): the pre-pass samples every 32nd item,
    whose nearest frames lie 16 frames from the impulse, so it sees about 0.14
    of max |S|.  gamma = 1e-3 max |S| ~ 15 sits in the bulk of the noise
    coefficients (|S| rms ~ 15), so the items run before the impulse's frames
    keep coefficients that the final gamma drops and are redone.  The result
    must equal, bit for bit, the forward given the final gamma, and match the
    oracle (with that gamma) on frames at the start, around the impulse and at
    the end; gamma must match the oracle's, whose maximum lies at the impulse."""
    from workloads import make_c2
    cfg = make_c2(n=1 << 12).cfg
    n = 1 << 18
    m_star = 8208
    rng = np.random.default_rng(7)
    x = rng.standard_normal(n).astype(np.float32)
    x[m_star * cfg.hop] += 15000.0
    plan = sst.Plan.from_config(n, cfg, device="cuda")
    xg = torch.from_numpy(x).cuda()
    gam = torch.empty(1, dtype=torch.float32, device="cuda")
    T = plan.forward(xg, gamma=gam)
    T2 = torch.full_like(T, float("nan"))
    plan.forward(xg, T2, reuse_gamma=True)
    torch.cuda.synchronize()
    same = torch.equal(torch.view_as_real(T), torch.view_as_real(T2))
    gamma_g = float(gam.cpu()[0])
    x64 = x.astype(np.float64)
    o_peak = oracle.forward(x64, cfg, m_star - 40, 80)
    _say(f"[spec] gamma GPU {gamma_g:.6g} oracle {o_peak.gamma:.6g}; speculative == exact-gamma "
         f"forward: {same}")
    assert same
    assert abs(gamma_g - o_peak.gamma) <= 1e-5 * o_peak.gamma
    g_o, gd_o = oracle.gaussian_windows(cfg.win_len, cfg.sigma)
    s_pack = math.sqrt(np.sum(g_o ** 2) / np.sum(gd_o ** 2))
    nfr = 32
    for f0 in (0, m_star - 16, plan.n_frames - nfr):
        S = torch.empty((nfr, plan.n_src), dtype=torch.complex64, device="cuda")
        idx = torch.empty((nfr, plan.n_src), dtype=torch.int32, device="cuda")
        plan.forward(xg, None, f0, nfr, S=S, idx=idx, reuse_gamma=True)
        torch.cuda.synchronize()
        o = oracle.forward(x64, cfg, f0, nfr, gamma=gamma_g)
        idx_g = idx.cpu().numpy()
        ny = packed_norms(x, g_o, gd_o, s_pack, cfg.hop, np.arange(f0, f0 + nfr))
        rep, _ = classify_indices(idx_g, o.idx, o.frac, o.S, o.Sd, o.gamma, cfg.nfft,
                                  cfg.subdiv, s_pack, ny, plan.n_dst)
        e_t = relf(T[f0:f0 + nfr].cpu().numpy(), reconciled_T(o.S, idx_g, plan.n_dst))
        _say(f"  frames {f0}+{nfr}: T(reconciled) relF={e_t:.2e} {rep}")
        assert e_t <= 1e-5 and rep.ok(), (rep, rep.details)


STATS_CASES = [c for c in CASES if c[0] in ("c2-shape", "c3-shape", "nf1024-F4", "nf512-F8-nz16")]


@pytest.mark.parametrize("name,n,cfg", STATS_CASES, ids=[c[0] for c in STATS_CASES])
def test_colstats_epilogue_of_the_production_forward(sst, name, n, cfg):
    """Per-frame FP64 sums (sum Re T, sum Im T, sum |T|^2) asked for without any
    per-coefficient output: the production arithmetic (speculative threshold
    and fix-up included) with the sums as an epilogue.  T must equal the plain
    call's bit for bit; the sums must equal the FP64 sums of the stored rows
    (to FP64 rounding: the order of a float64 reduction) and those of the debug
    variant; and a chunked call must give the whole call's rows."""
    x = _signal(name, n, cfg.fs)
    plan = sst.Plan.from_config(n, cfg, device="cuda")
    xg = torch.from_numpy(x).cuda()
    T0 = plan.forward(xg)
    col = torch.full((plan.n_frames, 3), float("nan"), dtype=torch.float64, device="cuda")
    T1 = plan.forward(xg, colstats=col)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(T0), torch.view_as_real(T1))
    Td = T1.cpu().numpy().astype(np.complex128)
    c = col.cpu().numpy()
    ref = np.stack([Td.real.sum(1), Td.imag.sum(1), (np.abs(Td) ** 2).sum(1)], axis=1)
    scale = np.abs(Td).sum(1)
    _say(f"[colstats] {name}: frames {plan.n_frames}, max |d sum| / sum|T| "
         f"{np.max(np.abs(c[:, :2] - ref[:, :2]) / (scale[:, None] + 1e-300)):.2e}")
    assert np.all(np.isfinite(c))
    assert np.all(np.abs(c[:, :2] - ref[:, :2]) <= 1e-12 * (scale[:, None] + 1e-300))
    assert np.allclose(c[:, 2], ref[:, 2], rtol=1e-12, atol=0.0)
    # the debug variant's sums over a middle chunk
    f0, nf = plan.n_frames // 3, min(64, plan.n_frames // 3)
    S = torch.empty((nf, plan.n_src), dtype=torch.complex64, device="cuda")
    cd = torch.empty((nf, 3), dtype=torch.float64, device="cuda")
    cp = torch.empty((nf, 3), dtype=torch.float64, device="cuda")
    Td2 = plan.forward(xg, None, f0, nf, S=S, colstats=cd, reuse_gamma=True)
    Tp2 = plan.forward(xg, None, f0, nf, colstats=cp, reuse_gamma=True)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(Td2), torch.view_as_real(T0[f0:f0 + nf]))
    assert torch.equal(torch.view_as_real(Tp2), torch.view_as_real(T0[f0:f0 + nf]))
    sc = np.concatenate([scale[f0:f0 + nf, None]] * 2 + [ref[f0:f0 + nf, 2:3]], axis=1)
    for got in (cd.cpu().numpy(), cp.cpu().numpy()):
        assert np.all(np.abs(got - c[f0:f0 + nf]) <= 1e-12 * (sc + 1e-300))
    # compressed rows carry no phase: no sums from them
    with pytest.raises(sst.SSTError):
        plan.forward(xg, colstats=col, out="mag_f32")


@pytest.mark.parametrize("hw", [26, 40])
def test_inverse_grouped_staging(sst, hw):
    """The wide inverse with 4 or 2 destination groups of a tile staged at once
    (hw 26: one pass of 4 or two of 2; hw 40: 4 + 2 or 2 + 2 + 2), and the
    extra-wide tiles of 2048 samples, against the one-group-at-a-time kernel
    and the oracle, on the same T: c3 shape
    (N_f 8192, H 32, z 8), N = 2^16, ridges of a tone and of a sweep, with
    frames of no ridge (-1); and chunked calls that accumulate."""
    cfg = SSTConfig(25600.0, 2047, 256.0, 32, 8192, 0.0, 5000.0, 8, "rel", 1e-3, hw)
    n = 1 << 16
    x = _signal("grouped", n, cfg.fs)
    plan = sst.Plan.from_config(n, cfg, device="cuda")
    o = oracle.forward(x.astype(np.float64), cfg)
    T32 = o.T.astype(np.complex64)
    nfr = plan.n_frames
    t = np.arange(nfr) * cfg.hop / cfg.fs
    f_sweep = 0.11 * cfg.fs + 2 * 0.02 * cfg.fs * t / (n / cfg.fs)
    ridge = np.stack([np.full(nfr, int(round(0.05 * cfg.fs / (cfg.fs / cfg.nfft) * cfg.subdiv))),
                      np.round(f_sweep / (cfg.fs / cfg.nfft) * cfg.subdiv).astype(np.int64)])
    ridge = np.clip(ridge, 0, plan.n_dst - 1).astype(np.int32)
    ridge[0, 100:140] = -1
    ridge[1, 600:700] = -1
    Tg = torch.from_numpy(T32).cuda()
    rg = torch.from_numpy(ridge).cuda()
    xs = {}
    for groups in (4, 2, 1):
        plan.set_tuning(inv_tf=4, inv_groups=groups)
        assert plan.get_tuning()["inv_groups"] == groups
        xs[groups] = plan.inverse(Tg, rg, hw).cpu().numpy()
    # extra-wide tiles (2048 samples, 130 frames): the default here
    plan.set_tuning()
    assert (plan.get_tuning()["inv_tf"], plan.get_tuning()["inv_groups"]) == (8, 1)
    xs["x8"] = plan.inverse(Tg, rg, hw).cpu().numpy()

    def chunked():
        a = nfr // 2 + 5
        xa = torch.zeros((2, n), dtype=torch.float32, device="cuda")
        plan.inverse(Tg[:a], rg[:, :a].contiguous(), hw, frame0=0, xhat=xa, accumulate=True)
        plan.inverse(Tg[a:], rg[:, a:].contiguous(), hw, frame0=a, xhat=xa, accumulate=True)
        return xa.cpu().numpy()
    xa8 = chunked()
    plan.set_tuning(inv_tf=4, inv_groups=4)
    xa = chunked()
    for q in range(2):
        xo = oracle.inverse(T32.astype(np.complex128), ridge[q], hw, o.g, cfg.hop, cfg.nfft,
                            o.band.k1, cfg.subdiv, n)
        e4, e2, e1 = relf(xs[4][q], xo), relf(xs[2][q], xo), relf(xs[1][q], xo)
        e8, ea, ea8 = relf(xs["x8"][q], xo), relf(xa[q], xo), relf(xa8[q], xo)
        d4, d2 = relf(xs[4][q], xs[1][q]), relf(xs[2][q], xs[1][q])
        d8 = relf(xs["x8"][q], xs[1][q])
        _say(f"[inverse groups] hw={hw} comp {q}: relF 4 groups {e4:.2e}, 2 groups {e2:.2e}, "
             f"one group {e1:.2e}, 2048-sample tiles {e8:.2e}, chunked {ea:.2e} / {ea8:.2e}; "
             f"vs one group {d4:.2e} / {d2:.2e} / {d8:.2e}")
        assert max(e4, e2, e1, e8, ea, ea8) <= 1e-5
        assert d4 <= 1e-6 and d2 <= 1e-6 and d8 <= 1e-6
