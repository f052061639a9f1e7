"""Comparison rules between the GPU library and the float64 oracle.

Tolerances:
  * STFT pair S, S' and the SST matrix T: relative Frobenius error <= 1e-5
    (T after reconciling the index decisions below; the raw value is reported);
  * threshold gamma: relative 1e-5;
  * destination indices: bit-exact, except
      - a coefficient whose |S| lies within 1e-5 gamma of gamma (or within the
        tier's own error bound of |S|) may be retained by one side only, and
      - a coefficient may land in the bin next to the oracle's when the
        oracle's fractional destination u lies within max(1e-4, 4 e_u) of the
        rounding boundary between them (the 1e-4 zone of the acceptance rule,
        widened to where FP32 cannot decide), e_u = z N_f / (2 pi) 2^-24 ||y||
        (1/(s|S|) + |S'|/|S|^2) being the first-order effect on u of one unit
        2^-24 ||y|| of error in S and in S' (||y||: norm of the packed windowed
        frame g x + i s g' x);
      - and the number of differences stays within a budget E + 4 sqrt(E) + 4,
        E = sum over retained coefficients of P(|N(0, e_u^2)| > distance to
        the boundary): the expected count if u carried a Gaussian error of
        one e_u (the measured spread of the FP32 FFT path is about 0.7 e_u);
    any other difference fails.  The matrix-core tiers pass their own worst-
    case bound of |dS| and |dS'| instead; their zone is the exact (not
    linearised) reach of that bound and no count budget applies.
  * inverse: relative Frobenius error of xhat <= 1e-5 on identical T, and
    reconstruction SNR within 0.1 dB of the oracle pipeline's.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def relf(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def snr_db(ref, est, lo: int, hi: int) -> float:
    r = np.asarray(ref, dtype=np.float64)[lo:hi]
    e = np.asarray(est, dtype=np.float64)[lo:hi]
    return float(10.0 * np.log10(np.sum(r * r) / np.sum((r - e) ** 2)))


def packed_norms(x, g, gd, s_pack, hop, frames):
    """||y_m|| = sqrt(||g x_m||^2 + ||s g' x_m||^2) for the given frames (float64)."""
    x = np.asarray(x, dtype=np.float64)
    L = g.shape[0]
    M = (L - 1) // 2
    n = x.shape[0]
    out = np.empty(len(frames))
    for i, m in enumerate(frames):
        lo = int(m) * hop - M
        seg = np.zeros(L)
        a, b = max(lo, 0), min(lo + L - 1, n - 1)
        if b >= a:
            seg[a - lo:b - lo + 1] = x[a:b + 1]
        out[i] = math.sqrt(np.sum((seg * g) ** 2) + np.sum((seg * gd * s_pack) ** 2))
    return out


@dataclass
class IndexReport:
    n_coeff: int
    n_retained: int
    literal_mismatch: int      # any difference at all
    literal_outside_1e4: int   # differences not within 1e-4 of a boundary
    membership_near_gamma: int
    boundary_flips: int
    unexplained: int
    worst_flip_ratio: float    # max of (distance to the boundary) / e_u over accepted flips
    expected_flips: float = 0.0
    budget: float = float("inf")

    def ok(self) -> bool:
        flips = self.literal_mismatch - self.membership_near_gamma
        return self.unexplained == 0 and flips <= self.budget


ZONE_MULT = 4.0   # D24(ii): flips accepted within max(1e-4, 4 e_u) of the boundary


def classify_indices(idx_g, idx_o, frac_o, S_o, Sd_o, gamma_o, nfft, z, s_pack, ny, n_dst=None,
                     err_s=None, err_sd=None, gamma_g=None):
    """Compare destination indices (see module doc).  ny[m] = ||y_m|| per frame.

    gamma_g: the GPU's threshold when it comes from a different arithmetic
    (the matrix-core tiers).

    err_s / err_sd (per frame) replace the FP32 FFT error model by the caller's
    worst-case bound on the absolute error of S and S' (the matrix-core tiers):
    u may then move by up to z N_f/(2 pi) (|S'| es + |S| ed) / (|S| (|S| - es)),
    and by any amount when es >= |S|.

    A GPU destination l is accepted for oracle position u when
    |l - u| <= 1/2 + tol: l is a bin that u rounds to once u moves by at most
    tol.  A GPU "outside the band" (-2) is accepted when u lies within tol of
    the band edges.
    """
    idx_g = np.asarray(idx_g)
    idx_o = np.asarray(idx_o)
    mag = np.abs(S_o)
    n_coeff = idx_o.size
    mem_o = idx_o != -1
    mem_g = idx_g != -1
    diff = idx_g != idx_o
    literal = int(diff.sum())
    both = mem_o & mem_g
    u = frac_o
    c = z * nfft / (2 * math.pi)
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        dist = np.abs((u + 0.5) - np.round(u + 0.5))
        if err_s is not None:
            es = np.asarray(err_s)[:, None]
            ed = np.asarray(err_sd)[:, None]
            e_u = c * (np.abs(Sd_o) * es + mag * ed) / (mag * (mag - es))
            e_u = np.where(mag > es, e_u, np.inf)
            near = np.abs(mag - gamma_o) <= np.maximum(1e-5 * gamma_o, es)
            tol = np.maximum(1e-4, e_u)
        else:
            e_u = c * 2.0 ** -24 * ny[:, None] * (1.0 / (s_pack * mag) + np.abs(Sd_o) / (mag * mag))
            near = np.abs(mag - gamma_o) <= 1e-5 * gamma_o
            tol = np.maximum(1e-4, ZONE_MULT * e_u)
    if gamma_g is not None:
        # a tier whose gamma comes from its own arithmetic: coefficients whose
        # |S| lies between the two thresholds may be retained by one side only
        near = near | ((mag - gamma_o) * (mag - gamma_g) <= 0.0)
    flip = diff & both
    gi = idx_g.astype(np.float64)
    with np.errstate(invalid="ignore"):
        ok_in = (idx_g >= 0) & (np.abs(gi - u) <= 0.5 + tol)
        if n_dst is None:
            n_dst = int(max(idx_o.max(), idx_g.max())) + 1
        ok_out = (idx_g == -2) & ((u < -0.5 + tol) | (u >= n_dst - 0.5 - tol))
    accepted_flip = flip & (ok_in | ok_out)
    mem_diff = mem_o != mem_g
    accepted_mem = mem_diff & near
    bad = diff & ~(accepted_flip | accepted_mem)
    unexplained = int(bad.sum())
    outside_1e4 = int((diff & ~(both & (dist < 1e-4))).sum())
    with np.errstate(invalid="ignore", divide="ignore"):
        ratios = np.abs(np.where(idx_g >= 0, np.abs(gi - u) - 0.5, 0.0))[accepted_flip] / e_u[accepted_flip]
    expected, budget = 0.0, float("inf")
    if err_s is None:
        from scipy.special import erfc
        with np.errstate(invalid="ignore", divide="ignore"):
            p = 0.5 * erfc(dist[mem_o] / (e_u[mem_o] * math.sqrt(2.0)))
        expected = float(np.nansum(p))
        budget = expected + 4.0 * math.sqrt(expected) + 4.0
    details = []
    for m, i in zip(*np.nonzero(bad)):
        details.append(dict(m=int(m), i=int(i), idx_g=int(idx_g[m, i]), idx_o=int(idx_o[m, i]),
                            u=float(u[m, i]), e_u=float(e_u[m, i]),
                            mag_rel=float(mag[m, i] / max(mag.max(), 1e-300)),
                            near_gamma=bool(near[m, i])))
        if len(details) >= 8:
            break
    rep = IndexReport(n_coeff, int(mem_o.sum()), literal, outside_1e4, int(accepted_mem.sum()),
                      int(accepted_flip.sum()), unexplained,
                      float(np.nanmax(ratios)) if ratios.size else 0.0, round(expected, 2),
                      round(budget, 2))
    rep.details = details
    return rep, None


def reconciled_T(S_o, idx_g, n_dst):
    """Oracle coefficients scattered with the GPU's destination decisions."""
    nfr, n_src = S_o.shape
    T = np.zeros((nfr, n_dst), dtype=np.complex128)
    m, i = np.nonzero(idx_g >= 0)
    np.add.at(T, (m, idx_g[m, i]), S_o[m, i])
    return T
