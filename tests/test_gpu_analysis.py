"""GPU: the analysis measures (sst_renyi: Renyi entropy of Sec. 3, Eq. 32)
against the float64 oracle on identical inputs."""
import sys

import numpy as np
import pytest

import oracle
from workloads import make_c2, make_paper_eq30

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


@pytest.mark.parametrize("wl", ["eq30", "c2-shape"])
def test_renyi_matches_oracle(sst, wl):
    """R of the SST matrix T (complex64) and of |T| as float32 and float16, each
    against the oracle on the same values; the float64 sums are reduced in a
    fixed order, so repeated calls agree bit for bit."""
    w = make_paper_eq30() if wl == "eq30" else make_c2(n=1 << 15)
    c = w.cfg
    plan = sst.Plan.from_config(w.n, c, device="cuda")
    T = plan.forward(torch.from_numpy(w.x).cuda())
    out = sst.renyi(T, 3)
    out2 = sst.renyi(T, 3)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    Tc = T.cpu().numpy()
    r_o = oracle.renyi(Tc.astype(np.complex128), 3.0)
    r_g = float(out[2].cpu())
    s1 = float(np.sum(np.abs(Tc.astype(np.complex128)) ** 2))
    _say(f"[renyi] {wl}: gpu {r_g:.9f} oracle {r_o:.9f} bits; sum P {float(out[0].cpu()):.6e} "
         f"vs {s1:.6e}")
    assert abs(r_g - r_o) <= 1e-6
    assert abs(float(out[0].cpu()) - s1) <= 1e-6 * s1
    for dt in (torch.float32, torch.float16):
        mag = T.abs().to(dt)
        r_m = float(sst.renyi(mag, 3)[2].cpu())
        ref = oracle.renyi(mag.cpu().numpy().astype(np.float64), 3.0)
        assert abs(r_m - ref) <= 1e-6, (dt, r_m, ref)
    # a sub-block of columns through the row stride
    sub = float(sst.renyi(T[:, 100:700], 3)[2].cpu())
    assert abs(sub - oracle.renyi(Tc[:, 100:700].astype(np.complex128), 3.0)) <= 1e-6
    for alpha in (2, 4):
        r_a = float(sst.renyi(T, alpha)[2].cpu())
        assert abs(r_a - oracle.renyi(Tc.astype(np.complex128), float(alpha))) <= 1e-6


# ---------------------------------------------------------------------------
# STFT product and STFT synthesis (Sec. 2.1, Eqs. 7-11)
# ---------------------------------------------------------------------------
from tests.parity import relf  # noqa: E402
from workloads import SSTConfig  # noqa: E402

STFT_CASES = [
    ("c2-shape", 1 << 15, SSTConfig(25600.0, 1023, 128.0, 16, 4096, 0.0, 6400.0, 4, "rel", 1e-3, 6)),
    ("c3-shape", 1 << 16, SSTConfig(25600.0, 2047, 256.0, 32, 8192, 0.0, 5000.0, 8, "rel", 1e-3, 26)),
    ("nf1024-F4-k1", 10007, SSTConfig(25600.0, 255, 32.0, 8, 1024, 300.0, 6400.0, 2, "rel", 1e-3, 2)),
    ("nf512-F8-nz16", 20011, SSTConfig(25600.0, 511, 64.0, 7, 512, 0.0, 6400.0, 1, "rel", 1e-3, 1)),
]


def _sig(n, fs, seed):
    rng = np.random.default_rng(seed)
    t = np.arange(n) / fs
    x = (np.cos(2 * np.pi * (0.11 * fs * t + 0.02 * fs * t * t / max(t[-1], 1e-9)))
         + 0.5 * np.cos(2 * np.pi * 0.05 * fs * t) + 0.3 * rng.standard_normal(n))
    return x.astype(np.float32)


def _full_band(S, k1, nfft):
    out = np.zeros((S.shape[0], nfft // 2 + 1), dtype=np.complex128)
    out[:, k1:k1 + S.shape[1]] = S
    return out


@pytest.mark.parametrize("name,n,cfg", STFT_CASES, ids=[c[0] for c in STFT_CASES])
def test_stft_product_and_synthesis(sst, name, n, cfg):
    """sst_stft against the oracle's direct STFT pair (relF <= 1e-5), and
    sst_stft_inverse on the oracle's S rounded to complex64 against the
    oracle's synthesis of the same values (relF <= 1e-5)."""
    x = _sig(n, cfg.fs, len(name))
    plan = sst.Plan.from_config(n, cfg, device="cuda")
    xg = torch.from_numpy(x).cuda()
    Sd = torch.empty((plan.n_frames, plan.n_src), dtype=torch.complex64, device="cuda")
    S = plan.stft(xg, Sd=Sd)
    torch.cuda.synchronize()
    o = oracle.forward(x.astype(np.float64), cfg)
    e_s, e_sd = relf(S.cpu().numpy(), o.S), relf(Sd.cpu().numpy(), o.Sd)
    S32 = o.S.astype(np.complex64)
    xh = plan.stft_inverse(torch.from_numpy(S32).cuda()).cpu().numpy()
    xo = oracle.stft_synthesis(_full_band(S32.astype(np.complex128), plan.k1, cfg.nfft), o.g,
                               cfg.hop, cfg.nfft, n)
    e_x = relf(xh, xo)
    _say(f"[stft] {name}: relF S={e_s:.2e} S'={e_sd:.2e} synthesis={e_x:.2e}")
    assert e_s <= 1e-5 and e_sd <= 1e-5 and e_x <= 1e-5


@pytest.mark.parametrize("name,n,cfg", STFT_CASES[:2], ids=[c[0] for c in STFT_CASES[:2]])
def test_stft_full_band_reconstructs_exactly(sst, name, n, cfg):
    """The exact-reconstruction identity of Eqs. 10-11 on the GPU path alone: with
    every one-sided bin, sst_stft then sst_stft_inverse returns x (every sample,
    the ends included) to FP32 rounding."""
    full = SSTConfig(cfg.fs, cfg.win_len, cfg.sigma, cfg.hop, cfg.nfft, 0.0, cfg.fs / 2, 1,
                     "rel", 1e-3, 1)
    x = _sig(n, cfg.fs, 7)
    plan = sst.Plan.from_config(n, full, device="cuda")
    xg = torch.from_numpy(x).cuda()
    xh = plan.stft_inverse(plan.stft(xg)).cpu().numpy()
    e = relf(xh, x.astype(np.float64))
    worst = float(np.max(np.abs(xh - x)))
    _say(f"[stft] {name} full band: relF(x) = {e:.2e}, max |err| = {worst:.2e}")
    assert e <= 1e-5


# ---------------------------------------------------------------------------
# Compressed outputs: |T| as float32 or float16 rows
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,n,cfg", STFT_CASES[:3], ids=[c[0] for c in STFT_CASES[:3]])
def test_compressed_magnitude_rows(sst, name, n, cfg):
    """|T| rows written by the forward (float32: the norm of the complex bin rounded
    once; float16: to half precision) against the complex rows of the same call
    kind (whole signal with the speculative threshold, and a chunk reusing gamma)."""
    x = torch.from_numpy(_sig(n, cfg.fs, 11)).cuda()
    plan = sst.Plan.from_config(n, cfg, device="cuda")
    T = plan.forward(x)
    M32 = plan.forward(x, out="mag_f32")
    M16 = plan.forward(x, out="mag_f16")
    f0, nf = plan.n_frames // 4, 29
    Mc = plan.forward(x, None, f0, nf, reuse_gamma=True, out="mag_f32")
    torch.cuda.synchronize()
    ref = np.abs(T.cpu().numpy().astype(np.complex128))
    m32 = M32.cpu().numpy().astype(np.float64)
    m16 = M16.cpu().numpy().astype(np.float64)
    assert M32.shape == (plan.n_frames, plan.n_dst) and M32.dtype == torch.float32
    assert np.all(np.abs(m32 - ref) <= 2.0 ** -22 * ref + 1e-38)
    assert np.all(np.abs(m16 - ref) <= 2.0 ** -10 * ref + 2.0 ** -24)
    assert torch.equal(Mc, M32[f0:f0 + nf])
    _say(f"[compressed] {name}: max rel f32 {np.max(np.abs(m32 - ref) / np.maximum(ref, 1e-30)):.2e}")
    r_c = float(sst.renyi(T, 3)[2].cpu())
    r_m = float(sst.renyi(M32, 3)[2].cpu())
    assert abs(r_c - r_m) <= 1e-6
