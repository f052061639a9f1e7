/*
 * sst_oracle_abi.c -- the oracle's mirror of the GPU library's C ABI
 * (declared in sst_oracle.h), over host pointers.
 *
 * TEST INFRASTRUCTURE ONLY, like sst_oracle.c, whose float64 functions do all
 * of the arithmetic: this file only validates arguments, widens the float
 * inputs, calls them in the order of the method and rounds the outputs once.
 *   forward: gamma (Sec. 2.2, Eq. 13; relative: rho max |S| over every frame,
 *            sso_stft_maxabs), STFT pair of the chunk (Sec. 2.1, Eqs. 7-9,
 *            sso_stft), reassignment (Eqs. 12-14, 27-29, sso_reassign);
 *   ridge:   sso_ridge per component (Sec. 2.2, zone M_q[m]);
 *   inverse: sso_inverse (Sec. 2.3, Eqs. 25-26) over a float64 copy of the
 *            whole T grid with the chunk's rows in place (the denominator runs
 *            over every frame, so chunks add up), or sso_inverse_eq15 (Eq. 15).
 */
#include "sst_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int sso_gaussian_windows(int L, double sigma, double *g, double *gd);
int sso_band(double fs, int nfft, double f_lo, double f_hi, int z, int *k1, int *k2,
             int *n_src, int *n_dst);
void sso_stft(const double *x, int64_t n, const double *g, const double *gd, int L, int hop,
              int nfft, int k1, int k2, int64_t frame0, int64_t nframes, double *S, double *Sd);
double sso_stft_maxabs(const double *x, int64_t n, const double *g, int L, int hop, int nfft,
                       int k1, int k2, int64_t frame0, int64_t nframes);
void sso_reassign(const double *S, const double *Sd, int64_t nframes, int n_src, int nfft,
                  int k1, int z, int n_dst, double gamma, double *T, int32_t *idx,
                  double *frac);
void sso_ridge(const double *T, int64_t nframes, int n_dst, int la, int lb, int32_t *ridge);
void sso_inverse(const double *T, int64_t nframes, int n_dst, const int32_t *ridge, int hw,
                 const double *g, int L, int hop, int nfft, int k1, int z, int64_t n,
                 double *xhat);
void sso_inverse_eq15(const double *T, int64_t nframes, int n_dst, const int32_t *ridge,
                      int hw, double g0, int nfft, int k1, int z, double *xhat);

struct sst_oracle_plan_s {
    sst_oracle_params p;
    sst_oracle_shape sh;
    double *g, *gd;   /* window pair, L taps each */
};

int32_t sst_oracle_plan(const sst_oracle_params *params, sst_oracle_plan_t *out)
{
    if (!params || !out)
        return SST_ORACLE_E_ARG;
    *out = NULL;
    const sst_oracle_params *p = params;
    if (p->struct_size != sizeof(sst_oracle_params) || p->n_samples < 1 || !(p->fs > 0.0) ||
        p->win_len < 1 || (p->win_len % 2) == 0 || p->nfft < 2 || p->win_len > p->nfft ||
        p->hop < 1 || p->subdiv < 1 || (p->thr_mode != SST_ORACLE_THR_ABS &&
                                          p->thr_mode != SST_ORACLE_THR_REL_MAX) ||
        !(p->thr >= 0.0) || ((p->window == NULL) != (p->dwindow == NULL)) ||
        (!p->window && !(p->sigma > 0.0)) || !(p->f_hi <= p->fs / 2.0))
        return SST_ORACLE_E_ARG;
    int k1, k2, n_src, n_dst;
    if (sso_band(p->fs, p->nfft, p->f_lo, p->f_hi, p->subdiv, &k1, &k2, &n_src, &n_dst) != 0)
        return SST_ORACLE_E_ARG;
    struct sst_oracle_plan_s *pl = (struct sst_oracle_plan_s *)calloc(1, sizeof(*pl));
    if (!pl)
        return SST_ORACLE_E_NOMEM;
    pl->p = *p;
    pl->p.window = pl->p.dwindow = NULL;   /* the copies below outlive the caller's */
    pl->g = (double *)malloc(sizeof(double) * (size_t)p->win_len);
    pl->gd = (double *)malloc(sizeof(double) * (size_t)p->win_len);
    if (!pl->g || !pl->gd) {
        sst_oracle_destroy(pl);
        return SST_ORACLE_E_NOMEM;
    }
    if (p->window) {
        memcpy(pl->g, p->window, sizeof(double) * (size_t)p->win_len);
        memcpy(pl->gd, p->dwindow, sizeof(double) * (size_t)p->win_len);
    } else if (sso_gaussian_windows(p->win_len, p->sigma, pl->g, pl->gd) != 0) {
        sst_oracle_destroy(pl);
        return SST_ORACLE_E_ARG;
    }
    sst_oracle_shape *s = &pl->sh;
    s->n_samples = p->n_samples;
    s->n_frames = (p->n_samples + p->hop - 1) / p->hop;
    s->win_len = p->win_len;
    s->hop = p->hop;
    s->nfft = p->nfft;
    s->subdiv = p->subdiv;
    s->k1 = k1;
    s->k2 = k2;
    s->n_src = n_src;
    s->n_dst = n_dst;
    s->workspace_bytes = 0;
    s->t_row_bytes = 8 * (size_t)n_dst;
    *out = pl;
    return SST_ORACLE_OK;
}

int32_t sst_oracle_plan_query(sst_oracle_plan_t pl, sst_oracle_shape *out)
{
    if (!pl || !out)
        return SST_ORACLE_E_ARG;
    *out = pl->sh;
    return SST_ORACLE_OK;
}

static double *widen(const float *v, size_t n)
{
    double *d = (double *)malloc(sizeof(double) * (n ? n : 1));
    if (d)
        for (size_t i = 0; i < n; ++i)
            d[i] = (double)v[i];
    return d;
}

int32_t sst_oracle_forward(sst_oracle_plan_t pl, const float *x, int64_t frame0,
                           int64_t nframes, float *T, float *S, float *Sd, int32_t *idx,
                           double *colstats, float *gamma_out)
{
    if (!pl || !x || !T || frame0 < 0 || nframes < 0 || frame0 + nframes > pl->sh.n_frames)
        return SST_ORACLE_E_ARG;
    const sst_oracle_params *p = &pl->p;
    const sst_oracle_shape *s = &pl->sh;
    const size_t n = (size_t)s->n_samples;
    double *xd = widen(x, n);
    const size_t ns = (size_t)nframes * (size_t)s->n_src;
    const size_t nt = (size_t)nframes * (size_t)s->n_dst;
    double *Sdb = (double *)malloc(sizeof(double) * 2 * (ns ? ns : 1));
    double *Sddb = (double *)malloc(sizeof(double) * 2 * (ns ? ns : 1));
    double *Tdb = (double *)malloc(sizeof(double) * 2 * (nt ? nt : 1));
    int32_t rc = SST_ORACLE_OK;
    if (!xd || !Sdb || !Sddb || !Tdb) {
        rc = SST_ORACLE_E_NOMEM;
        goto done;
    }
    double gamma = p->thr;
    if (p->thr_mode == SST_ORACLE_THR_REL_MAX)
        gamma = p->thr * sso_stft_maxabs(xd, s->n_samples, pl->g, p->win_len, p->hop, p->nfft,
                                         s->k1, s->k2, 0, s->n_frames);
    if (gamma_out)
        *gamma_out = (float)gamma;
    sso_stft(xd, s->n_samples, pl->g, pl->gd, p->win_len, p->hop, p->nfft, s->k1, s->k2,
             frame0, nframes, Sdb, Sddb);
    sso_reassign(Sdb, Sddb, nframes, s->n_src, p->nfft, s->k1, p->subdiv, s->n_dst, gamma, Tdb,
                 idx, NULL);
    for (size_t i = 0; i < 2 * nt; ++i)
        T[i] = (float)Tdb[i];
    for (size_t i = 0; i < 2 * ns; ++i) {
        if (S)
            S[i] = (float)Sdb[i];
        if (Sd)
            Sd[i] = (float)Sddb[i];
    }
    if (colstats) {
        for (int64_t f = 0; f < nframes; ++f) {
            const double *row = Tdb + 2 * (size_t)f * (size_t)s->n_dst;
            double re = 0.0, im = 0.0, e2 = 0.0;
            for (int l = 0; l < s->n_dst; ++l) {
                re += row[2 * l];
                im += row[2 * l + 1];
                e2 += row[2 * l] * row[2 * l] + row[2 * l + 1] * row[2 * l + 1];
            }
            colstats[3 * f] = re;
            colstats[3 * f + 1] = im;
            colstats[3 * f + 2] = e2;
        }
    }
done:
    free(xd);
    free(Sdb);
    free(Sddb);
    free(Tdb);
    return rc;
}

int32_t sst_oracle_ridge(sst_oracle_plan_t pl, const float *T, int64_t nframes,
                         const int32_t *band, int32_t n_comp, int32_t *ridge)
{
    if (!pl || !T || !band || !ridge || n_comp < 1 || n_comp > 16 || nframes < 0 ||
        nframes > pl->sh.n_frames)
        return SST_ORACLE_E_ARG;
    const size_t nt = (size_t)nframes * (size_t)pl->sh.n_dst;
    double *Tdb = widen(T, 2 * nt);
    if (!Tdb)
        return SST_ORACLE_E_NOMEM;
    for (int q = 0; q < n_comp; ++q)
        sso_ridge(Tdb, nframes, pl->sh.n_dst, band[2 * q], band[2 * q + 1],
                  ridge + (size_t)q * (size_t)nframes);
    free(Tdb);
    return SST_ORACLE_OK;
}

int32_t sst_oracle_inverse(sst_oracle_plan_t pl, const float *T, int64_t frame0,
                           int64_t nframes, const int32_t *ridge, int32_t n_comp, int32_t hw,
                           float *xhat, const float *xref, double *err, uint32_t flags)
{
    if (!pl || !T || !ridge || !xhat || n_comp < 1 || n_comp > 65535 || hw < 0 || hw > 512 ||
        frame0 < 0 || nframes < 1 || frame0 + nframes > pl->sh.n_frames ||
        (flags & ~(SST_ORACLE_INV_ACCUMULATE | SST_ORACLE_INV_EQ15)))
        return SST_ORACLE_E_ARG;
    const sst_oracle_params *p = &pl->p;
    const sst_oracle_shape *s = &pl->sh;
    const int eq15 = (flags & SST_ORACLE_INV_EQ15) != 0;
    const int accumulate = (flags & SST_ORACLE_INV_ACCUMULATE) != 0;
    const int whole = frame0 == 0 && nframes == s->n_frames;
    if ((err && (!xref || !whole || accumulate)) || (eq15 && p->hop != 1))
        return SST_ORACLE_E_ARG;
    const int M = (p->win_len - 1) / 2;
    const int64_t N = s->n_samples, nf = s->n_frames, nd = s->n_dst;
    /* the chunk's rows in a float64 copy of the whole grid; other frames are
       absent from the numerator (ridge -1) and present in the denominator */
    double *Tall = (double *)calloc(2 * (size_t)nf * (size_t)nd, sizeof(double));
    int32_t *rall = (int32_t *)malloc(sizeof(int32_t) * (size_t)nf);
    double *xd = (double *)malloc(sizeof(double) * (size_t)N);
    if (!Tall || !rall || !xd) {
        free(Tall);
        free(rall);
        free(xd);
        return SST_ORACLE_E_NOMEM;
    }
    for (size_t i = 0; i < 2 * (size_t)nframes * (size_t)nd; ++i)
        Tall[2 * (size_t)frame0 * (size_t)nd + i] = (double)T[i];
    /* samples the chunk reaches */
    int64_t lo = eq15 ? frame0 : frame0 * p->hop - M;
    int64_t hi = eq15 ? frame0 + nframes - 1 : (frame0 + nframes - 1) * p->hop + M;
    lo = lo < 0 ? 0 : lo;
    hi = hi > N - 1 ? N - 1 : hi;
    for (int q = 0; q < n_comp; ++q) {
        for (int64_t m = 0; m < nf; ++m)
            rall[m] = (m >= frame0 && m < frame0 + nframes)
                          ? ridge[(size_t)q * (size_t)nframes + (size_t)(m - frame0)]
                          : -1;
        if (eq15)
            sso_inverse_eq15(Tall, nf, (int)nd, rall, hw, pl->g[M], p->nfft, s->k1, p->subdiv,
                             xd);
        else
            sso_inverse(Tall, nf, (int)nd, rall, hw, pl->g, p->win_len, p->hop, p->nfft,
                        s->k1, p->subdiv, N, xd);
        float *out = xhat + (size_t)q * (size_t)N;
        for (int64_t i = lo; i <= hi; ++i)
            out[i] = accumulate ? (float)((double)out[i] + xd[i]) : (float)xd[i];
        if (err) {
            const float *r = xref + (size_t)q * (size_t)N;
            double d2 = 0.0, r2 = 0.0;
            for (int64_t i = M; i < N - M; ++i) {
                const double d = (double)r[i] - (double)out[i];
                d2 += d * d;
                r2 += (double)r[i] * (double)r[i];
            }
            err[2 * q] = d2;
            err[2 * q + 1] = r2;
        }
    }
    free(Tall);
    free(rall);
    free(xd);
    return SST_ORACLE_OK;
}

void sst_oracle_destroy(sst_oracle_plan_t pl)
{
    if (!pl)
        return;
    free(pl->g);
    free(pl->gd);
    free(pl);
}
