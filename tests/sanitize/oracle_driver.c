/* Exercises the float64 oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer on a small signal: windows, band, STFT pair,
 * maximum, reassignment, ridge, both inverses, the STFT synthesis and the
 * Renyi entropy, including frames that reach past both ends of the signal;
 * then the mirror ABI (sst_oracle_abi.c): plan, chunked forward, ridge,
 * chunked inverse, and rejected arguments.  Test infrastructure only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "sst_oracle.h"

int sso_gaussian_windows(int L, double sigma, double *g, double *gd);
int sso_band(double fs, int nfft, double f_lo, double f_hi, int z, int *k1, int *k2, int *n_src,
             int *n_dst);
void sso_stft(const double *x, int64_t n, const double *g, const double *gd, int L, int hop,
              int nfft, int k1, int k2, int64_t frame0, int64_t nframes, double *S, double *Sd);
double sso_stft_maxabs(const double *x, int64_t n, const double *g, int L, int hop, int nfft,
                       int k1, int k2, int64_t frame0, int64_t nframes);
void sso_reassign(const double *S, const double *Sd, int64_t nframes, int n_src, int nfft, int k1,
                  int z, int n_dst, double gamma, double *T, int32_t *idx, double *frac);
void sso_ridge(const double *T, int64_t nframes, int n_dst, int la, int lb, int32_t *ridge);
void sso_inverse(const double *T, int64_t nframes, int n_dst, const int32_t *ridge, int hw,
                 const double *g, int L, int hop, int nfft, int k1, int z, int64_t n, double *xhat);
void sso_inverse_eq15(const double *T, int64_t nframes, int n_dst, const int32_t *ridge, int hw,
                      double g0, int nfft, int k1, int z, double *xhat);
void sso_stft_synthesis(const double *S, int64_t nframes, const double *g, int L, int hop,
                        int nfft, int64_t n, double *xhat);
double sso_renyi(const double *C, int64_t rows, int64_t cols, double alpha);

int main(void)
{
    const int n = 3000, L = 255, hop = 7, nfft = 512, z = 3;
    double *x = malloc(sizeof(double) * n), *g = malloc(sizeof(double) * L),
           *gd = malloc(sizeof(double) * L);
    for (int i = 0; i < n; ++i)
        x[i] = cos(0.3 * i + 1e-4 * i * i) + 0.1 * sin(1.7 * i);
    if (sso_gaussian_windows(L, 32.0, g, gd) != 0)
        return 1;
    int k1, k2, n_src, n_dst;
    if (sso_band(1000.0, nfft, 20.0, 400.0, z, &k1, &k2, &n_src, &n_dst) != 0)
        return 1;
    int64_t nfr = (n + hop - 1) / hop;
    double *S = malloc(sizeof(double) * 2 * nfr * n_src), *Sd = malloc(sizeof(double) * 2 * nfr * n_src);
    sso_stft(x, n, g, gd, L, hop, nfft, k1, k2, 0, nfr, S, Sd);
    double mx = sso_stft_maxabs(x, n, g, L, hop, nfft, k1, k2, 0, nfr);
    double *T = malloc(sizeof(double) * 2 * nfr * n_dst), *frac = malloc(sizeof(double) * nfr * n_src);
    int32_t *idx = malloc(sizeof(int32_t) * nfr * n_src), *ridge = malloc(sizeof(int32_t) * nfr);
    sso_reassign(S, Sd, nfr, n_src, nfft, k1, z, n_dst, 1e-3 * mx, T, idx, frac);
    sso_ridge(T, nfr, n_dst, 0, n_dst - 1, ridge);
    double *xh = malloc(sizeof(double) * n);
    sso_inverse(T, nfr, n_dst, ridge, 5, g, L, hop, nfft, k1, z, n, xh);
    sso_inverse_eq15(T, nfr, n_dst, ridge, 5, g[L / 2], nfft, k1, z, xh);
    int nb = nfft / 2 + 1;
    double *Sf = calloc((size_t)2 * nfr * nb, sizeof(double));
    sso_stft(x, n, g, gd, L, hop, nfft, 0, nfft / 2, 0, nfr, Sf, NULL);
    sso_stft_synthesis(Sf, nfr, g, L, hop, nfft, n, xh);
    double err = 0.0;
    for (int i = 0; i < n; ++i)
        err = fmax(err, fabs(xh[i] - x[i]));
    double r = sso_renyi(T, nfr, n_dst, 3.0);
    printf("oracle driver: synthesis max err %.3e, renyi %.4f\n", err, r);

    /* mirror ABI */
    int bad = 0;
    sst_oracle_params p = {sizeof(sst_oracle_params), n, 1000.0, L, 32.0, NULL, NULL, hop, nfft,
                           20.0, 400.0, z, SST_ORACLE_THR_REL_MAX, 1e-3, 0, 0};
    sst_oracle_plan_t pl = NULL;
    bad |= sst_oracle_plan(&p, &pl) != SST_ORACLE_OK;
    sst_oracle_shape sh;
    bad |= sst_oracle_plan_query(pl, &sh) != SST_ORACLE_OK;
    float *xf = malloc(sizeof(float) * n), *Tf = malloc(sizeof(float) * 2 * nfr * n_dst);
    float *Sf32 = malloc(sizeof(float) * 2 * nfr * n_src), *xhf = calloc((size_t)2 * n, sizeof(float));
    double *cs = malloc(sizeof(double) * 3 * nfr), errs[4];
    int32_t *rr = malloc(sizeof(int32_t) * 2 * nfr), band[4] = {0, n_dst / 2, n_dst / 2, n_dst - 1};
    for (int i = 0; i < n; ++i)
        xf[i] = (float)x[i];
    const int64_t a = nfr / 3;
    float gam = 0.f;
    bad |= sst_oracle_forward(pl, xf, 0, a, Tf, Sf32, NULL, idx, cs, &gam) != SST_ORACLE_OK;
    bad |= sst_oracle_forward(pl, xf, a, nfr - a, Tf + 2 * a * n_dst, NULL, NULL, NULL, NULL,
                              NULL) != SST_ORACLE_OK;
    bad |= sst_oracle_ridge(pl, Tf, nfr, band, 2, rr) != SST_ORACLE_OK;
    bad |= sst_oracle_inverse(pl, Tf, 0, nfr, rr, 2, 5, xhf, xhf, errs, 0) != SST_ORACLE_OK;
    bad |= sst_oracle_inverse(pl, Tf, 0, a, rr, 1, 5, xhf, NULL, NULL,
                              SST_ORACLE_INV_ACCUMULATE) != SST_ORACLE_OK;
    bad |= sst_oracle_forward(pl, xf, 0, nfr + 1, Tf, NULL, NULL, NULL, NULL, NULL) !=
           SST_ORACLE_E_ARG;
    bad |= sst_oracle_inverse(pl, Tf, 0, nfr, rr, 2, 5, xhf, NULL, NULL, SST_ORACLE_INV_EQ15) !=
           SST_ORACLE_E_ARG;
    p.win_len = 2 * nfft;
    sst_oracle_plan_t bad_pl = NULL;
    bad |= sst_oracle_plan(&p, &bad_pl) != SST_ORACLE_E_ARG || bad_pl != NULL;
    sst_oracle_destroy(pl);
    printf("oracle driver: mirror ABI %s\n", bad ? "FAILED" : "ok");
    free(xf); free(Tf); free(Sf32); free(xhf); free(cs); free(rr);

    free(x); free(g); free(gd); free(S); free(Sd); free(T); free(frac); free(idx); free(ridge);
    free(xh); free(Sf);
    return (err < 1e-9 && isfinite(r) && !bad) ? 0 : 1;
}
