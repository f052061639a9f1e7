/*
 * sst_oracle.h -- the oracle's mirror of the GPU library's C ABI, over host
 * pointers.
 *
 * TEST INFRASTRUCTURE ONLY (see sst_oracle.c).  Every type and constant here
 * is declared anew for the oracle: it includes nothing of the GPU library.
 * The calls take the same arguments, in the same order and layout, as the
 * GPU library's plan / query / forward / ridge / inverse calls, with host
 * memory in place of device memory and no workspace, binding or stream, so
 * that a test can drive one pipeline through either library.  Arithmetic is
 * float64 throughout (sst_oracle.c); float arrays are only the ABI's storage:
 * x is widened on entry, T / S / S' are rounded once on exit.
 *
 * Method: D. He, H. Cao, arXiv 2003.07065 -- framing and STFT pair (Sec. 2.1,
 * Eqs. 7-9), IF estimate and selective subdivided reassignment (Sec. 2.2,
 * Eqs. 12-14; Sec. 2.4, Eqs. 27-29), ridge zones (Sec. 2.2), direct inverse
 * (Sec. 2.3, Eqs. 25-26) and the hop-1 inverse (Sec. 2.2, Eq. 15).
 */
#ifndef SST_ORACLE_H
#define SST_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes: 0 = OK, negative = error (same values as the GPU library's) */
#define SST_ORACLE_OK 0
#define SST_ORACLE_E_ARG (-1)
#define SST_ORACLE_E_UNSUPPORTED (-2)
#define SST_ORACLE_E_NOMEM (-6)

#define SST_ORACLE_THR_ABS 0      /* gamma = thr */
#define SST_ORACLE_THR_REL_MAX 1  /* gamma = thr * max |S| over all frames, in-band bins */

#define SST_ORACLE_INV_ACCUMULATE 1u
#define SST_ORACLE_INV_EQ15 2u

/*
 * Parameters: the same fields, order and meaning as the GPU library's
 * parameter block (N, fs, L, sigma, optional window pair, H, N_f, band, z,
 * threshold).  precision and flags are accepted and ignored (the oracle is
 * float64 only).
 */
typedef struct {
    uint32_t struct_size;
    int64_t n_samples;
    double fs;
    int32_t win_len;
    double sigma;
    const double *window;
    const double *dwindow;
    int32_t hop;
    int32_t nfft;
    double f_lo;
    double f_hi;
    int32_t subdiv;
    int32_t thr_mode;
    double thr;
    int32_t precision;
    uint32_t flags;
} sst_oracle_params;

typedef struct {
    int64_t n_samples;
    int64_t n_frames;         /* ceil(N / hop) */
    int32_t win_len, hop, nfft, subdiv;
    int32_t k1, k2;
    int32_t n_src;            /* k2 - k1 + 1 */
    int32_t n_dst;            /* z (k2 - k1) + 1 */
    size_t workspace_bytes;   /* 0: the oracle needs none */
    size_t t_row_bytes;       /* 8 n_dst */
} sst_oracle_shape;

typedef struct sst_oracle_plan_s *sst_oracle_plan_t;

/* Validate and build the float64 windows and band.  Errors: E_ARG, E_NOMEM. */
int32_t sst_oracle_plan(const sst_oracle_params *params, sst_oracle_plan_t *out);
int32_t sst_oracle_plan_query(sst_oracle_plan_t plan, sst_oracle_shape *out);

/*
 * Forward SST of frames [frame0, frame0 + nframes): T float complex
 * [nframes][n_dst] (every element written); optional S, Sd float complex
 * [nframes][n_src], idx int32 [nframes][n_src] (l, -1 below threshold, -2
 * outside the band), colstats double [nframes][3] (sum Re T, sum Im T,
 * sum |T|^2 of the float64 row), gamma_out float [1].  With the relative
 * threshold, gamma comes from every frame of x.  Errors: E_ARG, E_NOMEM.
 */
int32_t sst_oracle_forward(sst_oracle_plan_t plan, const float *x, int64_t frame0,
                           int64_t nframes, float *T, float *S, float *Sd, int32_t *idx,
                           double *colstats, float *gamma_out);

/*
 * Ridge of each component: per frame the first largest |T| in
 * [band[2q], band[2q+1]] (clipped), -1 when that range is all zero.
 * T float complex [nframes][n_dst]; ridge int32 [n_comp][nframes].
 */
int32_t sst_oracle_ridge(sst_oracle_plan_t plan, const float *T, int64_t nframes,
                         const int32_t *band, int32_t n_comp, int32_t *ridge);

/*
 * Direct inverse of n_comp components from T rows of frames
 * [frame0, frame0 + nframes): xhat float [n_comp][N] (accumulated with
 * SST_ORACLE_INV_ACCUMULATE, else the samples the chunk reaches are
 * overwritten); optional xref / err as the GPU library's (sum (xref-xhat)^2
 * and sum xref^2 over [M, N - M), whole-signal calls).  SST_ORACLE_INV_EQ15:
 * the hop-1 inverse.  Errors: E_ARG, E_NOMEM.
 */
int32_t sst_oracle_inverse(sst_oracle_plan_t plan, const float *T, int64_t frame0,
                           int64_t nframes, const int32_t *ridge, int32_t n_comp, int32_t hw,
                           float *xhat, const float *xref, double *err, uint32_t flags);

void sst_oracle_destroy(sst_oracle_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif
