"""Pins of the float64 oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own formula: each compares the oracle with
a library routine on a special case (numpy FFT), with a brute-force literal
reading of an equation on tiny inputs, with a closed form, or with an identity
(conservation, exact reconstruction).  A dropped term, a wrong sign or index,
or a transposed operand anywhere in the oracle fails at least one of them.
"""
import cmath
import math

import numpy as np
import pytest

import oracle
from workloads import make_chirp, make_tone


def relf(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


# ---------------------------------------------------------------------------
# O1 windows
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sigma", [4.0, 8.0, 32.0, 128.0])
def test_window_unit_energy(sigma):
    """Sec. 2.1: the Gaussian (pi sigma^2)^(-1/4) exp(-t^2/2sigma^2) has unit energy."""
    L = 2 * int(8 * sigma) + 1
    g, _ = oracle.gaussian_windows(L, sigma)
    assert abs(np.sum(g * g) - 1.0) < 1e-12


@pytest.mark.parametrize("sigma", [8.0, 32.0, 128.0])
def test_window_eq22_sqrt2(sigma, golden):
    """Sec. 2.3, Eq. 22: integral of g(0) g(t) dt = sqrt(2) (sampled: the sum over j)."""
    L = 2 * int(8 * sigma) + 1
    g, _ = oracle.gaussian_windows(L, sigma)
    M = (L - 1) // 2
    val = g[M] * np.sum(g)
    ref = golden["eq22_int_g0_g"]
    assert abs(val - ref["value"]) < ref["tol"]


def test_window_derivative_is_derivative():
    """Sec. 2.2: g' is the derivative of g -- checked by a central difference of g(t)."""
    sigma, L = 16.0, 129
    g, gd = oracle.gaussian_windows(L, sigma)
    M = (L - 1) // 2
    amp = (math.pi * sigma * sigma) ** -0.25
    h = 1e-5
    for j in range(-M, M + 1, 7):
        fd = (amp * math.exp(-((j + h) ** 2) / (2 * sigma ** 2))
              - amp * math.exp(-((j - h) ** 2) / (2 * sigma ** 2))) / (2 * h)
        assert abs(gd[j + M] - fd) < 1e-8 * amp
        assert abs(g[j + M] - amp * math.exp(-j * j / (2 * sigma ** 2))) < 1e-15


def test_window_rejects_even_length():
    with pytest.raises(ValueError):
        oracle.gaussian_windows(64, 8.0)


# ---------------------------------------------------------------------------
# O2 band and destination grid
# ---------------------------------------------------------------------------

def test_band_configs():
    # full band, z = 1 reproduces the one-sided grid N_f/2 + 1
    assert oracle.band(1024.0, 4096, 0.0, 512.0, 1) == oracle.Band(0, 2048, 2049, 2049)
    # [0, 6.4 kHz] at fs = 25.6 kHz, N_f = 4096, z = 4
    assert oracle.band(25600.0, 4096, 0.0, 6400.0, 4) == oracle.Band(0, 1024, 1025, 4097)
    # [0, 5 kHz] at N_f = 8192, z = 8
    assert oracle.band(25600.0, 8192, 0.0, 5000.0, 8) == oracle.Band(0, 1600, 1601, 12801)


def test_band_snaps_outward():
    """Sec. 5.1's band [6900, 9500] Hz is not on the 44.1 kHz / 8192 grid: snap outward."""
    b = oracle.band(44100.0, 8192, 6900.0, 9500.0, 8)
    df = 44100.0 / 8192
    assert b.k1 * df <= 6900.0 < (b.k1 + 1) * df
    assert (b.k2 - 1) * df < 9500.0 <= b.k2 * df
    assert b.n_dst == 8 * (b.k2 - b.k1) + 1


# ---------------------------------------------------------------------------
# O4 STFT pair
# ---------------------------------------------------------------------------

def _numpy_eq9(x, g, gd, hop, nfft, k1, k2):
    """Eq. 9 by library FFT: zero-padded windowed frame, FFT, times exp(i 2 pi k M / N_f)."""
    L = g.shape[0]
    M = (L - 1) // 2
    n = x.shape[0]
    nfr = -(-n // hop)
    xp = np.concatenate([np.zeros(M), x, np.zeros(M + hop)])
    k = np.arange(k1, k2 + 1)
    ph = np.exp(1j * 2 * np.pi * k * M / nfft)
    S = np.empty((nfr, k.shape[0]), dtype=np.complex128)
    Sd = np.empty_like(S)
    for m in range(nfr):
        seg = xp[m * hop: m * hop + L]   # samples c_m - M .. c_m + M
        buf = np.zeros(nfft)
        buf[:L] = seg * g
        S[m] = np.fft.fft(buf)[k1:k2 + 1] * ph
        buf[:L] = seg * gd
        Sd[m] = np.fft.fft(buf)[k1:k2 + 1] * ph
    return S, Sd


@pytest.mark.parametrize("L,sigma,hop,nfft,k1,k2", [
    (63, 8.0, 4, 64, 0, 32),
    (101, 12.0, 7, 128, 10, 50),
    (255, 32.0, 16, 256, 0, 128),
    (31, 4.0, 1, 32, 3, 16),
])
def test_stft_matches_numpy_fft(L, sigma, hop, nfft, k1, k2):
    rng = np.random.default_rng(11)
    x = rng.standard_normal(700)
    g, gd = oracle.gaussian_windows(L, sigma)
    S, Sd = oracle.stft(x, g, gd, hop, nfft, k1, k2)
    Sr, Sdr = _numpy_eq9(x, g, gd, hop, nfft, k1, k2)
    assert relf(S, Sr) < 1e-13
    assert relf(Sd, Sdr) < 1e-13


def test_stft_brute_force_eq7():
    """Eq. 7 literally: sum over all integers n of x[n] g[n - mH] e^{-i 2 pi k (n - mH)/N_f}."""
    rng = np.random.default_rng(3)
    N, L, sigma, hop, nfft = 40, 9, 2.0, 3, 16
    x = rng.standard_normal(N)
    g, gd = oracle.gaussian_windows(L, sigma)
    M = (L - 1) // 2

    def gw(j, w):
        return w[j + M] if -M <= j <= M else 0.0

    nfr = -(-N // hop)
    S, Sd = oracle.stft(x, g, gd, hop, nfft, 0, nfft // 2)
    for m in range(nfr):
        for k in range(nfft // 2 + 1):
            a = 0j
            b = 0j
            for nn in range(-20, N + 20):
                xv = x[nn] if 0 <= nn < N else 0.0
                e = cmath.exp(-2j * math.pi * k * (nn - m * hop) / nfft)
                a += xv * gw(nn - m * hop, g) * e
                b += xv * gw(nn - m * hop, gd) * e
            assert abs(S[m, k] - a) < 1e-13
            assert abs(Sd[m, k] - b) < 1e-13


def test_stft_chunked_equals_full():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(1000)
    g, gd = oracle.gaussian_windows(63, 8.0)
    S, Sd = oracle.stft(x, g, gd, 5, 64, 2, 20)
    S2, Sd2 = oracle.stft(x, g, gd, 5, 64, 2, 20, frame0=37, nframes=50)
    assert np.array_equal(S[37:87], S2) and np.array_equal(Sd[37:87], Sd2)


def test_maxabs_equals_max_of_stft():
    rng = np.random.default_rng(6)
    x = rng.standard_normal(900)
    g, gd = oracle.gaussian_windows(63, 8.0)
    S, _ = _numpy_eq9(x, g, gd, 3, 128, 5, 40)
    assert abs(oracle.stft_maxabs(x, g, 3, 128, 5, 40) - np.abs(S).max()) < 1e-12 * np.abs(S).max()


# ---------------------------------------------------------------------------
# O6 reassignment
# ---------------------------------------------------------------------------

def _eq28_literal(S, Sd, fs, nfft, k1, k2, z, gamma):
    """Eqs. 13 and 28-29 as printed, scanning every destination l for every k.

    omega-hat = |xi[k] - Im(S'/S)| in rad/s (Im(S'/S) is rad/sample, times fs);
    xi*[l] = 2 pi (f1 + l (f2 - f1)/(z N_r)) with f1 = k1 df, f2 = k2 df;
    coefficient k goes to l when -dxi*/2 <= omega-hat - xi*[l] < dxi*/2
    (the half-open reading of the paper's two-sided <=, one bin per coefficient).
    """
    df = fs / nfft
    nr = k2 - k1
    f1, f2 = k1 * df, k2 * df
    n_dst = z * nr + 1
    dxi = 2 * np.pi * df / z
    xi_star = 2 * np.pi * (f1 + np.arange(n_dst) * (f2 - f1) / (z * nr))
    T = np.zeros((S.shape[0], n_dst), dtype=np.complex128)
    for m in range(S.shape[0]):
        for i in range(S.shape[1]):
            s = S[m, i]
            if not abs(s) > gamma:
                continue
            k = k1 + i
            w_hat = abs(2 * np.pi * k * df - fs * (Sd[m, i] / s).imag)
            d = w_hat - xi_star
            hit = np.nonzero((d >= -dxi / 2) & (d < dxi / 2))[0]
            assert hit.shape[0] <= 1
            if hit.shape[0]:
                T[m, hit[0]] += s
    return T


@pytest.mark.parametrize("z,k1,k2", [(1, 0, 32), (3, 4, 28), (4, 0, 32)])
def test_reassign_equals_literal_eq28(z, k1, k2):
    rng = np.random.default_rng(21 + z)
    fs, nfft = 800.0, 64
    n = 600
    x = make_tone(n, 9.3 * fs / nfft, fs) + 0.5 * make_chirp(n, 60.0, 100.0, fs) \
        + 0.3 * rng.standard_normal(n)
    g, gd = oracle.gaussian_windows(41, 5.0)
    S, Sd = oracle.stft(x, g, gd, 3, nfft, k1, k2)
    gamma = 1e-3 * np.abs(S).max()
    b = oracle.band(fs, nfft, k1 * fs / nfft, k2 * fs / nfft, z)
    assert (b.k1, b.k2) == (k1, k2)
    T, idx, frac = oracle.reassign(S, Sd, nfft, k1, z, b.n_dst, gamma)
    Tref = _eq28_literal(S, Sd, fs, nfft, k1, k2, z, gamma)
    assert np.abs(T - Tref).max() <= 1e-12 * np.abs(S).max()
    # idx codes agree with the mask and the retained set
    assert np.all((idx == -1) == ~(np.abs(S) > gamma))


def test_reassign_conservation():
    """Each column of T sums to the sum of its retained in-range coefficients."""
    rng = np.random.default_rng(7)
    x = rng.standard_normal(2000)
    g, gd = oracle.gaussian_windows(127, 16.0)
    b = oracle.band(1000.0, 256, 50.0, 300.0, 4)
    S, Sd = oracle.stft(x, g, gd, 8, 256, b.k1, b.k2)
    gamma = 1e-2 * np.abs(S).max()
    T, idx, _ = oracle.reassign(S, Sd, 256, b.k1, 4, b.n_dst, gamma)
    kept = np.where(idx >= 0, S, 0)
    col = T.sum(axis=1)
    ref = kept.sum(axis=1)
    assert np.abs(col - ref).max() <= 1e-13 * np.abs(S).sum(axis=1).max()
    # every retained coefficient lands at the recorded l
    m, i = np.nonzero(idx >= 0)
    assert np.all(idx[m, i] < b.n_dst)
    # out-of-band destinations are flagged -2 and excluded
    assert np.any(idx == -2) and np.any(idx >= 0)


def test_tone_concentrates_in_one_bin():
    """Eq. 17: a stationary tone reassigns into the destination bin of its frequency.

    Tone at the centre of destination bin l0 (subdivided grid), L = 12 sigma + 1,
    relative threshold 1e-6: every retained coefficient of every interior frame
    lands in l0.
    """
    fs, nfft, z, sigma, hop = 1000.0, 256, 2, 8.0, 4
    L = int(12 * sigma) + 1
    b = oracle.band(fs, nfft, 0.0, fs / 2, z)
    l0 = 81
    f0 = (b.k1 + l0 / z) * fs / nfft
    n = 2048
    x = make_tone(n, f0, fs, phase=0.3)
    g, gd = oracle.gaussian_windows(L, sigma)
    S, Sd = oracle.stft(x, g, gd, hop, nfft, b.k1, b.k2)
    gamma = 1e-6 * np.abs(S).max()
    T, idx, frac = oracle.reassign(S, Sd, nfft, b.k1, z, b.n_dst, gamma)
    M = (L - 1) // 2
    interior = np.arange(-(-M // hop), (n - 1 - M) // hop + 1)
    sel = idx[interior]
    assert np.all(sel[sel != -1] == l0)
    assert np.abs(frac[interior][sel == l0] - l0).max() < 0.25
    # the whole frame energy of the positive-frequency lobe sits in T[:, l0]
    Ti = T[interior]
    assert np.all(np.abs(Ti[:, l0]) > 0.999 * np.abs(Ti).sum(axis=1))


def test_linear_chirp_closed_form():
    """Eq. 13 with Eq. 39: for a linear chirp and a Gaussian window,
    omega-hat(u, xi) = w(u) + (xi - w(u)) c^2 s^4 / (1 + c^2 s^4)   (c: rad/sample^2).
    Checked per coefficient on interior frames where |S| >= 1e-2 max |S|.
    """
    fs, nfft, sigma, hop, z = 1.0, 512, 16.0, 8, 1
    L = int(12 * sigma) + 1
    c = 0.3 / sigma ** 2
    n = 2048
    w0 = 0.3
    nn = np.arange(n, dtype=np.float64)
    x = np.cos(w0 * nn + 0.5 * c * nn * nn)
    g, gd = oracle.gaussian_windows(L, sigma)
    b = oracle.band(fs, nfft, 0.0, 0.5, z)
    S, Sd = oracle.stft(x, g, gd, hop, nfft, b.k1, b.k2)
    T, idx, frac = oracle.reassign(S, Sd, nfft, b.k1, z, b.n_dst, 0.0)
    M = (L - 1) // 2
    rho = (c * sigma ** 2) ** 2 / (1 + (c * sigma ** 2) ** 2)
    worst = 0.0
    checked = 0
    for m in range(-(-M // hop), (n - 1 - M) // hop + 1):
        u = m * hop
        wu = w0 + c * u
        if not (0.5 < wu < np.pi - 0.5):
            continue
        mag = np.abs(S[m])
        keep = mag >= 1e-2 * np.abs(S).max()
        k = np.arange(b.k1, b.k2 + 1)[keep]
        xi = 2 * np.pi * k / nfft
        pred_bins = (wu + (xi - wu) * rho) * nfft / (2 * np.pi)
        worst = max(worst, float(np.abs(frac[m][keep] - pred_bins).max()))
        checked += int(keep.sum())
    assert checked > 1000
    assert worst < 0.05


# ---------------------------------------------------------------------------
# O7 ridge
# ---------------------------------------------------------------------------

def test_ridge_is_first_argmax():
    rng = np.random.default_rng(9)
    T = rng.standard_normal((50, 40)) + 1j * rng.standard_normal((50, 40))
    T[3, 10] = T[3, 12] = 100.0      # tie: smallest l wins
    T[4, :] = 0.0                    # empty range: -1
    r = oracle.ridge(T, 5, 30)
    ref = 5 + np.argmax(np.abs(T[:, 5:31]) ** 2, axis=1)
    ref[4] = -1
    assert np.array_equal(r, ref)
    assert r[3] == 10


# ---------------------------------------------------------------------------
# O8 inverse
# ---------------------------------------------------------------------------

def _ideal_tone_T(nframes, hop, nfft, n_dst, l0, w0, g0, amp=1.0, phase=0.0):
    """Perfectly concentrated SST of amp*cos(w0 n + phase): N_f g[0] amp/2 e^{i(w0 c_m + phase)} at l0."""
    T = np.zeros((nframes, n_dst), dtype=np.complex128)
    c = np.arange(nframes) * hop
    T[:, l0] = nfft * g0 * amp / 2 * np.exp(1j * (w0 * c + phase))
    return T


@pytest.mark.parametrize("hop,z,k1,l0", [(1, 1, 0, 37), (8, 4, 0, 150), (5, 3, 12, 61),
                                         (16, 2, 7, 1)])
def test_inverse_ideal_tone_is_exact(hop, z, k1, l0):
    """Eqs. 25-26 on the SST of Eq. 17 (all of a tone's mass on its own bin) give the tone back
    at every sample, edges included."""
    nfft, sigma, n = 128, 10.0, 1500
    L = 81
    g, _ = oracle.gaussian_windows(L, sigma)
    M = (L - 1) // 2
    n_dst = z * 40 + 1
    nfr = -(-n // hop)
    w0 = 2 * np.pi * (z * k1 + l0) / (z * nfft)
    T = _ideal_tone_T(nfr, hop, nfft, n_dst, l0, w0, g[M], amp=0.7, phase=0.4)
    ridge = np.full(nfr, l0, dtype=np.int32)
    xh = oracle.inverse(T, ridge, 3, g, hop, nfft, k1, z, n)
    ref = 0.7 * np.cos(w0 * np.arange(n) + 0.4)
    assert np.abs(xh - ref).max() < 1e-12
    if hop == 1:
        xh15 = oracle.inverse_eq15(T, ridge, 3, g[M], nfft, k1, z)
        assert np.abs(xh15 - ref).max() < 1e-12


def test_inverse_dc_weight_is_one():
    """At DC the one-sided weight is 1: a constant comes back with unit gain."""
    nfft, hop, n, L = 64, 4, 400, 41
    g, _ = oracle.gaussian_windows(L, 6.0)
    M = (L - 1) // 2
    nfr = -(-n // hop)
    T = np.zeros((nfr, 33), dtype=np.complex128)
    T[:, 0] = nfft * g[M] * 1.25
    xh = oracle.inverse(T, np.zeros(nfr, np.int32), 2, g, hop, nfft, 0, 1, n)
    assert np.abs(xh - 1.25).max() < 1e-12


def test_inverse_ridge_minus_one_contributes_nothing():
    nfft, hop, n, L = 64, 4, 400, 41
    g, _ = oracle.gaussian_windows(L, 6.0)
    nfr = -(-n // hop)
    rng = np.random.default_rng(1)
    T = rng.standard_normal((nfr, 33)) + 1j * rng.standard_normal((nfr, 33))
    xh = oracle.inverse(T, np.full(nfr, -1, np.int32), 2, g, hop, nfft, 0, 1, n)
    assert np.all(xh == 0.0)


def test_ola_denominator_interior_sqrt2_over_h():
    """Eq. 22 with hop H: sum_m g[0] g[n - mH] = sqrt(2)/H in the interior (unit-energy g)."""
    for sigma, hop in [(32.0, 1), (128.0, 16), (256.0, 32)]:
        L = 2 * int(4 * sigma) - 1
        g, _ = oracle.gaussian_windows(L, sigma)
        M = (L - 1) // 2
        for s in range(5000, 5000 + hop):
            js = np.arange(-M, M + 1)
            mask = ((s - js) % hop) == 0
            den = g[M] * g[mask].sum()
            assert abs(den * hop - math.sqrt(2)) < 2e-3


def test_stft_synthesis_identity():
    """Eqs. 10-11: STFT synthesis over all one-sided bins reconstructs the signal exactly."""
    rng = np.random.default_rng(4)
    n, L, sigma, hop, nfft = 700, 63, 8.0, 5, 64
    x = rng.standard_normal(n)
    g, gd = oracle.gaussian_windows(L, sigma)
    S, _ = oracle.stft(x, g, gd, hop, nfft, 0, nfft // 2, want_sd=False)
    xh = oracle.stft_synthesis(S, g, hop, nfft, n)
    assert np.abs(xh - x).max() < 1e-12


def test_tone_pipeline_reconstruction_snr():
    """A clean tone at a destination-bin centre, SST + direct inverse (Eqs. 25-26):
    unit gain, >= 60 dB in the interior."""
    fs, nfft, z, sigma, hop = 25600.0, 1024, 4, 32.0, 8
    L = 255
    b = oracle.band(fs, nfft, 0.0, 6400.0, z)
    l0 = 4 * 30 + 2
    f0 = (b.k1 + l0 / z) * fs / nfft
    n = 8192
    x = make_tone(n, f0, fs, amp=0.9, phase=1.1)
    g, gd = oracle.gaussian_windows(L, sigma)
    S, Sd = oracle.stft(x, g, gd, hop, nfft, b.k1, b.k2)
    T, idx, _ = oracle.reassign(S, Sd, nfft, b.k1, z, b.n_dst, 1e-3 * np.abs(S).max())
    nfr = S.shape[0]
    xh = oracle.inverse(T, np.full(nfr, l0, np.int32), 6, g, hop, nfft, b.k1, z, n)
    M = (L - 1) // 2
    sl = slice(M, n - M)
    snr = 10 * np.log10(np.sum(x[sl] ** 2) / np.sum((x[sl] - xh[sl]) ** 2))
    assert snr > 60.0


def test_eq15_and_eq26_agree_on_tone_at_hop1():
    fs, nfft, sigma = 1024.0, 512, 16.0
    L = 129
    n = 2048
    b = oracle.band(fs, nfft, 0.0, fs / 2, 1)
    l0 = 50
    x = make_tone(n, l0 * fs / nfft, fs, phase=0.2)
    g, gd = oracle.gaussian_windows(L, sigma)
    S, Sd = oracle.stft(x, g, gd, 1, nfft, b.k1, b.k2)
    T, _, _ = oracle.reassign(S, Sd, nfft, b.k1, 1, b.n_dst, 1e-4 * np.abs(S).max())
    ridge = np.full(n, l0, np.int32)
    x26 = oracle.inverse(T, ridge, 10, g, 1, nfft, b.k1, 1, n)
    x15 = oracle.inverse_eq15(T, ridge, 10, g[(L - 1) // 2], nfft, b.k1, 1)
    M = (L - 1) // 2
    sl = slice(M, n - M)
    for xh in (x26, x15):
        snr = 10 * np.log10(np.sum(x[sl] ** 2) / np.sum((x[sl] - xh[sl]) ** 2))
        assert snr > 50.0


# ---------------------------------------------------------------------------
# Renyi entropy (Sec. 3, Eq. 32), P = |C|^2, discrete form
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha", [2.0, 3.0, 0.5])
def test_renyi_closed_forms(alpha):
    """One occupied cell gives 0; K equal cells give log2 K (for every alpha);
    two levels give the closed form; scaling C changes nothing."""
    rng = np.random.default_rng(3)
    C = np.zeros((7, 11), dtype=np.complex128)
    C[3, 4] = 2.0 - 1.5j
    assert abs(oracle.renyi(C, alpha)) < 1e-12
    for K in (2, 5, 77):
        C = np.zeros(77, dtype=np.complex128)
        idx = rng.choice(77, size=K, replace=False)
        C[idx] = 0.3 * np.exp(1j * rng.uniform(0, 2 * np.pi, K))   # equal |C|, any phase
        assert abs(oracle.renyi(C, alpha) - math.log2(K)) < 1e-12
    # K1 cells of energy e1 and K2 of e2
    K1, K2, e1, e2 = 3, 10, 4.0, 0.25
    C = np.concatenate([np.full(K1, math.sqrt(e1)), np.full(K2, math.sqrt(e2) * 1j),
                        np.zeros(5)])
    tot = K1 * e1 + K2 * e2
    want = math.log2(K1 * (e1 / tot) ** alpha + K2 * (e2 / tot) ** alpha) / (1 - alpha)
    assert abs(oracle.renyi(C, alpha) - want) < 1e-12
    C = rng.standard_normal((13, 9)) + 1j * rng.standard_normal((13, 9))
    assert abs(oracle.renyi(C, alpha) - oracle.renyi(17.5 * C, alpha)) < 1e-12


def test_renyi_orders_concentration():
    """A wider Gaussian ridge (less concentrated) has a larger entropy, and the
    entropy of a separable product of two grids is the sum of their entropies."""
    f = np.arange(64)
    vals = []
    for width in (1.0, 2.0, 4.0, 8.0):
        row = np.exp(-0.5 * ((f - 32) / width) ** 2)
        vals.append(oracle.renyi(np.tile(row, (20, 1)), 3.0))
    assert all(a < b for a, b in zip(vals, vals[1:]))
    a = np.exp(-0.5 * ((np.arange(40) - 20) / 3.0) ** 2)
    b = np.exp(-0.5 * ((np.arange(30) - 10) / 5.0) ** 2)
    prod = np.sqrt(np.outer(a, b))        # P = |C|^2 = outer(a, b)
    ra = oracle.renyi(np.sqrt(a), 3.0)
    rb = oracle.renyi(np.sqrt(b), 3.0)
    assert abs(oracle.renyi(prod, 3.0) - (ra + rb)) < 1e-10


def test_renyi_rejects_degenerate_input():
    assert math.isnan(oracle.renyi(np.zeros((3, 3)), 3.0))
    assert math.isnan(oracle.renyi(np.ones((3, 3)), 1.0))
