/*
 * sst_oracle.c -- plain float64 CPU oracle of the downsampled STFT-based
 * synchrosqueezing transform (SST) and its direct inverse.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library: every table below is built
 * here, from the paper's formulas, in float64.
 *
 * Reference: D. He, H. Cao, "Fast implementation of synchrosqueezing transform
 * based on downsampling for large-scale vibration signal analysis"
 * (arXiv 2003.07065).  Each function names the passage it follows.
 *
 * Deliberately slow and obvious: direct band-limited DFTs (no FFT), scalar
 * reassignment, and a direct per-sample inverse.  OpenMP only parallelises
 * independent outer loops (frames, output samples); no result depends on the
 * thread count.
 *
 * Conventions (readings of the paper, each justified in the design notes):
 *   - sigma and window positions are in samples; window index j in [-M, M];
 *   - frames are centred at c_m = m*H, m = 0 .. ceil(N/H)-1, and x[n] = 0
 *     outside [0, N);
 *   - complex arrays are interleaved (re, im) doubles;
 *   - the band [f1, f2] is snapped outward to source bins k1..k2 and the
 *     destination grid is f*_l = (k1 + l/z) * fs/N_f, l = 0 .. z*(k2-k1);
 *   - reassignment rounds half up: l = floor(u + 1/2);
 *   - a coefficient is retained when |S| > gamma (strict).
 *
 * Parity pins: see tests/test_oracle_pins.py.  Every exported function is
 * pinned there against something other than itself.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define SSO_TWO_PI 6.283185307179586476925286766559

/* Exact integer reduction of a (possibly negative) product into [0, mod). */
static int64_t sso_mod(int64_t a, int64_t mod)
{
    int64_t r = a % mod;
    return r < 0 ? r + mod : r;
}

/* ---------------------------------------------------------------------------
 * O1. Windows (Sec. 2.1, Gaussian g; Sec. 2.2, its derivative g').
 *   g(t)  = (pi sigma^2)^(-1/4) exp(-t^2 / (2 sigma^2))
 *   g'(t) = -(t / sigma^2) g(t)
 * sampled at t = j, j in [-M, M], M = (L-1)/2.  Returns 0, or -1 for bad L.
 * ------------------------------------------------------------------------- */
int sso_gaussian_windows(int L, double sigma, double *g, double *gd)
{
    if (L < 1 || (L % 2) == 0 || !(sigma > 0.0))
        return -1;
    int M = (L - 1) / 2;
    double amp = pow(M_PI * sigma * sigma, -0.25);
    for (int j = -M; j <= M; ++j) {
        double t = (double)j;
        double gj = amp * exp(-t * t / (2.0 * sigma * sigma));
        g[j + M] = gj;
        if (gd)
            gd[j + M] = -(t / (sigma * sigma)) * gj;
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * O2. Band of interest and destination grid (Sec. 2.4, Eqs. 27-29).
 *   df = fs/N_f; k1 = floor(f1/df + 1e-9); k2 = min(ceil(f2/df - 1e-9), N_f/2)
 *   N_r = k2 - k1; n_src = N_r + 1; n_dst = z N_r + 1.
 * Returns 0, or -1 for an empty/invalid band.
 * ------------------------------------------------------------------------- */
int sso_band(double fs, int nfft, double f_lo, double f_hi, int z,
             int *k1, int *k2, int *n_src, int *n_dst)
{
    if (!(fs > 0.0) || nfft < 2 || z < 1 || !(f_lo >= 0.0) || !(f_hi > f_lo))
        return -1;
    double df = fs / (double)nfft;
    int a = (int)floor(f_lo / df + 1e-9);
    int b = (int)ceil(f_hi / df - 1e-9);
    if (b > nfft / 2)
        b = nfft / 2;
    if (a < 0 || a >= b)
        return -1;
    *k1 = a;
    *k2 = b;
    *n_src = b - a + 1;
    *n_dst = z * (b - a) + 1;
    return 0;
}

/* ---------------------------------------------------------------------------
 * O4. Downsampled STFT pair (Sec. 2.1, Eqs. 7-9; Sec. 2.2 for g').
 *   S[m,k]  = sum_{j=-M}^{M} x[mH + j] g[j]  exp(-i 2 pi k j / N_f)
 *   S'[m,k] = sum_{j=-M}^{M} x[mH + j] g'[j] exp(-i 2 pi k j / N_f)
 * for frames m in [frame0, frame0 + nframes) and bins k in [k1, k2].  The
 * exponent index (k*j) mod N_f is reduced exactly in integers and looked up in
 * a float64 table W[r] = exp(-i 2 pi r / N_f).  This is Eq. 9 (zero-padded
 * N_f-point DFT times the centre phase exp(i 2 pi k M / N_f)) written directly.
 * Outputs S, Sd: interleaved complex [nframes][k2-k1+1]; Sd may be NULL.
 * ------------------------------------------------------------------------- */
static void sso_twiddles(int nfft, double **wre, double **wim)
{
    *wre = (double *)malloc(sizeof(double) * (size_t)nfft);
    *wim = (double *)malloc(sizeof(double) * (size_t)nfft);
    for (int r = 0; r < nfft; ++r) {
        double a = SSO_TWO_PI * (double)r / (double)nfft;
        (*wre)[r] = cos(a);
        (*wim)[r] = -sin(a);
    }
}

/* Direct DFT of one frame centred at c, bins k1..k2, into S (and Sd). */
static void sso_stft_frame(const double *x, int64_t n, const double *g, const double *gd,
                           int M, int64_t c, int nfft, int k1, int k2,
                           const double *wre, const double *wim, double *S, double *Sd)
{
    for (int k = k1; k <= k2; ++k) {
        double sr = 0.0, si = 0.0, dr = 0.0, di = 0.0;
        /* r = (k j) mod N_f, stepped exactly in integers as j increases */
        int64_t r = sso_mod((int64_t)k * (-M), nfft);
        for (int j = -M; j <= M; ++j, r = (r + k >= nfft) ? r + k - nfft : r + k) {
            int64_t idx = c + j;
            if (idx < 0 || idx >= n)
                continue;
            double xv = x[idx];
            double a = xv * g[j + M];
            sr += a * wre[r];
            si += a * wim[r];
            if (Sd) {
                double b = xv * gd[j + M];
                dr += b * wre[r];
                di += b * wim[r];
            }
        }
        S[2 * (k - k1)] = sr;
        S[2 * (k - k1) + 1] = si;
        if (Sd) {
            Sd[2 * (k - k1)] = dr;
            Sd[2 * (k - k1) + 1] = di;
        }
    }
}

void sso_stft(const double *x, int64_t n, const double *g, const double *gd, int L,
              int hop, int nfft, int k1, int k2, int64_t frame0, int64_t nframes,
              double *S, double *Sd)
{
    int M = (L - 1) / 2;
    int n_src = k2 - k1 + 1;
    double *wre, *wim;
    sso_twiddles(nfft, &wre, &wim);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t f = 0; f < nframes; ++f) {
        size_t o = 2 * (size_t)f * (size_t)n_src;
        sso_stft_frame(x, n, g, gd, M, (frame0 + f) * (int64_t)hop, nfft, k1, k2, wre, wim,
                       S + o, Sd ? Sd + o : NULL);
    }
    free(wre);
    free(wim);
}

/* ---------------------------------------------------------------------------
 * O5. Global magnitude maximum for a relative threshold (Sec. 2.2, Eq. 13:
 * gamma = rho * max |S| over the in-band bins of the frames given).  Computes S
 * frame by frame with the same direct sum as sso_stft and keeps the maximum.
 * Frames m in [frame0, frame0 + nframes).
 * ------------------------------------------------------------------------- */
double sso_stft_maxabs(const double *x, int64_t n, const double *g, int L, int hop,
                       int nfft, int k1, int k2, int64_t frame0, int64_t nframes)
{
    int M = (L - 1) / 2;
    int n_src = k2 - k1 + 1;
    double *wre, *wim;
    sso_twiddles(nfft, &wre, &wim);
    double best = 0.0;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 2 * (size_t)n_src);
        double local = 0.0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t f = 0; f < nframes; ++f) {
            sso_stft_frame(x, n, g, NULL, M, (frame0 + f) * (int64_t)hop, nfft, k1, k2,
                           wre, wim, buf, NULL);
            for (int i = 0; i < n_src; ++i) {
                double mag = sqrt(buf[2 * i] * buf[2 * i] + buf[2 * i + 1] * buf[2 * i + 1]);
                if (mag > local)
                    local = mag;
            }
        }
        free(buf);
#pragma omp critical
        {
            if (local > best)
                best = local;
        }
    }
    free(wre);
    free(wim);
    return best;
}

/* ---------------------------------------------------------------------------
 * O6. IF estimate and selective, subdivided reassignment
 * (Sec. 2.2, Eqs. 12-14; Sec. 2.4, Eqs. 27-29).
 * For every frame and in-band source bin k with |S| > gamma:
 *   omega-hat = | xi[k] - Im(S'/S) |                         (Eq. 13)
 *   in source-bin units: kappa = | k - N_f Im(S' conj(S)) / (2 pi |S|^2) |
 *   destination position u = z (kappa - k1)                  (Eqs. 28-29)
 *   l = floor(u + 1/2); if 0 <= l < n_dst: T[m,l] += S[m,k]  (Eq. 28)
 * idx receives l for a contributing coefficient, -1 below threshold and -2
 * for a destination outside the band; frac receives u (NaN below threshold).
 * T (interleaved complex [nframes][n_dst]) is overwritten.  idx/frac may be
 * NULL.
 * ------------------------------------------------------------------------- */
void sso_reassign(const double *S, const double *Sd, int64_t nframes, int n_src,
                  int nfft, int k1, int z, int n_dst, double gamma,
                  double *T, int32_t *idx, double *frac)
{
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < nframes; ++f) {
        double *row = T + 2 * (size_t)f * (size_t)n_dst;
        memset(row, 0, sizeof(double) * 2 * (size_t)n_dst);
        for (int i = 0; i < n_src; ++i) {
            size_t o = 2 * ((size_t)f * n_src + (size_t)i);
            double sr = S[o], si = S[o + 1];
            double dr = Sd[o], di = Sd[o + 1];
            double mag2 = sr * sr + si * si;
            size_t oi = (size_t)f * n_src + (size_t)i;
            if (!(sqrt(mag2) > gamma)) {
                if (idx)
                    idx[oi] = -1;
                if (frac)
                    frac[oi] = NAN;
                continue;
            }
            /* Im(S' * conj(S)) / |S|^2 = Im(S'/S), radians per sample */
            double q = (di * sr - dr * si) / mag2;
            int k = k1 + i;
            double kappa = fabs((double)k - (double)nfft * q / SSO_TWO_PI);
            double u = (double)z * (kappa - (double)k1);
            double lf = floor(u + 0.5);
            if (frac)
                frac[oi] = u;
            if (lf < 0.0 || lf >= (double)n_dst) {
                if (idx)
                    idx[oi] = -2;
                continue;
            }
            int l = (int)lf;
            row[2 * l] += sr;
            row[2 * l + 1] += si;
            if (idx)
                idx[oi] = l;
        }
    }
}

/* ---------------------------------------------------------------------------
 * O7. Ridge of one component (Sec. 2.2, the zone M_q[m] around an extracted
 * ridge; the extraction rule is not specified by the paper).  Reading used:
 * per frame, the destination bin of largest |T| inside [la, lb]; ties go to the
 * smallest l.  ridge[f] = -1 when the whole range is zero.
 * ------------------------------------------------------------------------- */
void sso_ridge(const double *T, int64_t nframes, int n_dst, int la, int lb,
               int32_t *ridge)
{
    if (la < 0)
        la = 0;
    if (lb > n_dst - 1)
        lb = n_dst - 1;
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < nframes; ++f) {
        const double *row = T + 2 * (size_t)f * (size_t)n_dst;
        double best = 0.0;
        int arg = -1;
        for (int l = la; l <= lb; ++l) {
            double m2 = row[2 * l] * row[2 * l] + row[2 * l + 1] * row[2 * l + 1];
            if (m2 > best) {
                best = m2;
                arg = l;
            }
        }
        ridge[f] = arg;
    }
}

/* One-sided spectrum weight: 2 for interior bins, 1 at DC and at Nyquist. */
static double sso_side_weight(int64_t abs_bin, int64_t grid)
{
    return (abs_bin == 0 || 2 * abs_bin == grid) ? 1.0 : 2.0;
}

/* ---------------------------------------------------------------------------
 * O8. Direct inverse of the downsampled SST (Sec. 2.3, Eqs. 25-26, and the
 * band / subdivision remark at the end of Sec. 2.5).
 *   r[m,j] = (1/N_f) sum_{l in zone(m)} a_l Re( T[m,l] exp(+i 2 pi ((z k1 + l) j mod z N_f) / (z N_f)) )
 *   xhat[n] = sum_m g[n - mH] r[m, n - mH] / sum_m g[0] g[n - mH]
 * zone(m) = [ridge[m] - hw, ridge[m] + hw] intersected with [0, n_dst);
 * ridge[m] < 0 means the frame contributes nothing to the numerator.  The
 * denominator runs over every frame whose window covers n.  a_l = 2 except 1
 * when the destination frequency is 0 or fs/2 (one-sided spectrum).
 * T holds all nframes = ceil(N/H) frames (interleaved complex [nframes][n_dst]).
 * ------------------------------------------------------------------------- */
void sso_inverse(const double *T, int64_t nframes, int n_dst, const int32_t *ridge,
                 int hw, const double *g, int L, int hop, int nfft, int k1, int z,
                 int64_t n, double *xhat)
{
    int M = (L - 1) / 2;
    int64_t grid = (int64_t)z * nfft;
    double *cre = (double *)malloc(sizeof(double) * (size_t)grid);
    double *cim = (double *)malloc(sizeof(double) * (size_t)grid);
    for (int64_t r = 0; r < grid; ++r) {
        double a = SSO_TWO_PI * (double)r / (double)grid;
        cre[r] = cos(a);
        cim[r] = sin(a);
    }
    double g0 = g[M];
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        /* frames whose window [c_m - M, c_m + M] contains s */
        int64_t mlo = (s - M + hop - 1 >= 0) ? (s - M + hop - 1) / hop : 0;
        int64_t mhi = (s + M) / hop;
        if (mhi > nframes - 1)
            mhi = nframes - 1;
        double num = 0.0, den = 0.0;
        for (int64_t m = mlo; m <= mhi; ++m) {
            int64_t j = s - m * (int64_t)hop;
            if (j < -M || j > M)
                continue;
            double gj = g[j + M];
            den += g0 * gj;
            int r0 = ridge[m];
            if (r0 < 0)
                continue;
            int la = r0 - hw < 0 ? 0 : r0 - hw;
            int lb = r0 + hw > n_dst - 1 ? n_dst - 1 : r0 + hw;
            const double *row = T + 2 * (size_t)m * (size_t)n_dst;
            double acc = 0.0;
            for (int l = la; l <= lb; ++l) {
                int64_t b = (int64_t)z * k1 + l;
                int64_t r = sso_mod(b * j, grid);
                double a = sso_side_weight(b, grid);
                acc += a * (row[2 * l] * cre[r] - row[2 * l + 1] * cim[r]);
            }
            num += gj * acc / (double)nfft;
        }
        xhat[s] = den > 0.0 ? num / den : 0.0;
    }
    free(cre);
    free(cim);
}

/* ---------------------------------------------------------------------------
 * Standard inverse SST for H_t = 1 (Sec. 2.2, Eq. 15, discrete constant).
 *   xhat[m] = (1 / (N_f g[0])) sum_{l in zone(m)} a_l Re T[m,l]
 * The continuous constant 1/(2 pi g(0)) becomes 1/(N_f g[0]) for an N_f-point
 * DFT; a_l doubles the one-sided sum as in sso_inverse.
 * ------------------------------------------------------------------------- */
void sso_inverse_eq15(const double *T, int64_t nframes, int n_dst, const int32_t *ridge,
                      int hw, double g0, int nfft, int k1, int z, double *xhat)
{
    int64_t grid = (int64_t)z * nfft;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < nframes; ++m) {
        int r0 = ridge[m];
        double acc = 0.0;
        if (r0 >= 0) {
            int la = r0 - hw < 0 ? 0 : r0 - hw;
            int lb = r0 + hw > n_dst - 1 ? n_dst - 1 : r0 + hw;
            const double *row = T + 2 * (size_t)m * (size_t)n_dst;
            for (int l = la; l <= lb; ++l) {
                int64_t b = (int64_t)z * k1 + l;
                acc += sso_side_weight(b, grid) * row[2 * l];
            }
        }
        xhat[m] = acc / ((double)nfft * g0);
    }
}

/* ---------------------------------------------------------------------------
 * Discrete STFT synthesis (Sec. 2.1, Eqs. 10-11) over the one-sided bins
 * k = 0 .. N_f/2, used as the exact-reconstruction identity: phase-undone
 * inverse DFT, real part with the one-sided weight, overlap-add with g, and the
 * per-sample normaliser sum_m g[n - mH]^2.
 *   xhat[n] = sum_m g[j] Re((1/N_f) sum_k a_k S[m,k] e^{i 2 pi k j / N_f}) / sum_m g[j]^2,
 *   j = n - mH.
 * S holds all frames over all one-sided bins: interleaved [nframes][N_f/2+1].
 * ------------------------------------------------------------------------- */
void sso_stft_synthesis(const double *S, int64_t nframes, const double *g, int L, int hop,
                        int nfft, int64_t n, double *xhat)
{
    int M = (L - 1) / 2;
    int nb = nfft / 2 + 1;
    double *cre = (double *)malloc(sizeof(double) * (size_t)nfft);
    double *cim = (double *)malloc(sizeof(double) * (size_t)nfft);
    for (int r = 0; r < nfft; ++r) {
        double a = SSO_TWO_PI * (double)r / (double)nfft;
        cre[r] = cos(a);
        cim[r] = sin(a);
    }
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        int64_t mlo = (s - M + hop - 1 >= 0) ? (s - M + hop - 1) / hop : 0;
        int64_t mhi = (s + M) / hop;
        if (mhi > nframes - 1)
            mhi = nframes - 1;
        double num = 0.0, den = 0.0;
        for (int64_t m = mlo; m <= mhi; ++m) {
            int64_t j = s - m * (int64_t)hop;
            if (j < -M || j > M)
                continue;
            double gj = g[j + M];
            den += gj * gj;
            const double *row = S + 2 * (size_t)m * (size_t)nb;
            double acc = 0.0;
            for (int k = 0; k < nb; ++k) {
                int64_t r = sso_mod((int64_t)k * j, nfft);
                acc += sso_side_weight(k, nfft) * (row[2 * k] * cre[r] - row[2 * k + 1] * cim[r]);
            }
            num += gj * acc / (double)nfft;
        }
        xhat[s] = den > 0.0 ? num / den : 0.0;
    }
    free(cre);
    free(cim);
}

/* ---------------------------------------------------------------------------
 * Renyi entropy of a time-frequency representation (Sec. 3, Eq. 32), used by
 * the paper to measure the concentration of SST and STFT.  Discrete form over
 * the rows x cols grid of complex coefficients C with P = |C|^2 (the paper does
 * not define P; reading: the energy of each coefficient):
 *   R = 1/(1 - alpha) log2( sum_cells (P / sum_cells P)^alpha ),
 * alpha > 0, alpha != 1.  The integral of Eq. 32 over a grid of cells would add
 * the constant log2 of the cell area; the discrete form leaves it out, so one
 * occupied cell gives 0 and K equal cells give log2 K.  Returns NaN for an
 * all-zero C or an invalid alpha.
 * ------------------------------------------------------------------------- */
double sso_renyi(const double *C, int64_t rows, int64_t cols, double alpha)
{
    if (!(alpha > 0.0) || alpha == 1.0)
        return NAN;
    int64_t n = rows * cols;
    double tot = 0.0;
#pragma omp parallel for reduction(+ : tot) schedule(static)
    for (int64_t i = 0; i < n; ++i)
        tot += C[2 * i] * C[2 * i] + C[2 * i + 1] * C[2 * i + 1];
    if (!(tot > 0.0))
        return NAN;
    double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double p = (C[2 * i] * C[2 * i] + C[2 * i + 1] * C[2 * i + 1]) / tot;
        if (p > 0.0)
            acc += pow(p, alpha);
    }
    return log2(acc) / (1.0 - alpha);
}

/* Number of OpenMP threads a parallel region of this library uses. */
int sso_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
