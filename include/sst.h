/*
 * sst.h -- C ABI of the MI355X (gfx950) downsampled synchrosqueezing
 * transform library.
 *
 * Method: D. He, H. Cao, "Fast implementation of synchrosqueezing transform
 * based on downsampling for large-scale vibration signal analysis",
 * arXiv 2003.07065.  The library computes
 *   - the downsampled STFT pair S, S' with a Gaussian window g and its
 *     derivative g' (Sec. 2.1, Eqs. 7-9; Sec. 2.2),
 *   - the IF estimate and the selective, subdivided reassignment into the SST
 *     matrix T (Sec. 2.2, Eqs. 12-14; Sec. 2.4, Eqs. 27-29),
 *   - ridges per component (Sec. 2.2, the zone M_q[m]),
 *   - the direct downsampled inverse (Sec. 2.3, Eqs. 25-26, with the band /
 *     subdivision remark closing Sec. 2.5) and the standard hop-1 inverse
 *     (Sec. 2.2, Eq. 15).
 *
 * Conventions used by every call:
 *   - sigma, window taps and hops are in samples; window index j in [-M, M],
 *     M = (L-1)/2; frame m is centred at sample m*H, m = 0 .. ceil(N/H)-1;
 *     x[n] = 0 outside [0, N);
 *   - the band [f_lo, f_hi] is snapped outward to source bins k1..k2:
 *     k1 = floor(f_lo/df + 1e-9), k2 = min(ceil(f_hi/df - 1e-9), N_f/2),
 *     df = fs/N_f; n_src = k2-k1+1 source bins, n_dst = z*(k2-k1)+1
 *     destination bins at f*_l = (k1 + l/z) df;
 *   - a coefficient is retained when |S| > gamma and lands in destination
 *     l = floor(z(|k - delta| - k1) + 1/2), delta = N_f Im(S'/S)/(2 pi);
 *     destinations outside [0, n_dst) are dropped;
 *   - complex arrays are interleaved float pairs (re, im), row-major;
 *   - all device pointers are caller-owned HIP device memory on the device
 *     that was current at sst_plan_bind; "stream" is a hipStream_t (NULL =
 *     the default stream); every call is asynchronous on that stream unless
 *     stated otherwise and never blocks the host;
 *   - every function returns an sst_status; nothing throws or aborts across
 *     the ABI.  On error, sst_last_error() returns a thread-local message.
 *
 * The library never allocates device memory: the caller binds one workspace
 * buffer per plan (size from sst_plan_query).
 */
#ifndef SST_H
#define SST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sst_status;

#define SST_OK 0
#define SST_E_ARG (-1)          /* invalid argument; see sst_last_error() */
#define SST_E_UNSUPPORTED (-2)  /* valid for the method, not built here (e.g. N_f > 8192) */
#define SST_E_WORKSPACE (-3)    /* workspace missing, misaligned or too small */
#define SST_E_DEVICE (-4)       /* a HIP call failed; sst_last_error() names it */
#define SST_E_STATE (-5)        /* plan not bound */
#define SST_E_NOMEM (-6)        /* host allocation failed */

/* Threshold modes (Sec. 2.2, Eq. 13: |S| > gamma). */
#define SST_THR_ABS 0           /* gamma = thr */
#define SST_THR_REL_MAX 1       /* gamma = thr * max |S| over every frame and in-band bin */

/* STFT arithmetic of the forward transform. */
#define SST_PREC_FP32_FFT 0     /* FP32 LDS FFT pair */
#define SST_PREC_GEMM_BF16 1    /* STFT as a DFT-matrix product on the matrix cores, BF16
                                   operands, FP32 accumulation */
#define SST_PREC_GEMM_F16X3 2   /* the same with FP16 hi/lo split operands, three products
                                   (hi*hi + hi*lo + lo*hi), FP32 accumulation */

/* sst_forward flags */
#define SST_FWD_REUSE_GAMMA 1u  /* keep the gamma computed by the previous forward call
                                   on this plan (chunked calls after the first) */
#define SST_FWD_OUT_MAG_F32 2u  /* compressed output: T holds float |T| [nframes][n_dst]
                                   (half the bytes of the complex rows) */
#define SST_FWD_OUT_MAG_F16 4u  /* compressed output: T holds half |T| [nframes][n_dst]
                                   (a quarter of the bytes); both FP32 FFT tier only */

/* sst_inverse flags */
#define SST_INV_ACCUMULATE 1u   /* add into xhat instead of overwriting it */
#define SST_INV_EQ15 2u         /* standard inverse of Eq. 15 (hop must be 1) */

/*
 * Transform parameters, copied at plan time (Sec. 2.1, 2.2, 2.4).
 *   struct_size  sizeof(sst_params), for forward compatibility
 *   n_samples    N, signal length, 1 <= N < 2^30
 *   fs           sampling rate in Hz, > 0
 *   win_len      L = 2M+1, odd, 1 <= L <= nfft
 *   sigma        Gaussian width in samples, > 0 (ignored when window given)
 *   window       optional host array of L doubles g[-M..M]; NULL = Gaussian
 *   dwindow      optional host array of L doubles g'[-M..M]; required iff window
 *   hop          H_t >= 1
 *   nfft         N_f, power of two, 512 <= N_f <= 8192, L <= N_f
 *   f_lo, f_hi   band of interest in Hz, 0 <= f_lo < f_hi <= fs/2
 *   subdiv       z >= 1, z*N_f <= 2^20
 *   thr_mode     SST_THR_ABS or SST_THR_REL_MAX
 *   thr          gamma (ABS, >= 0) or rho (REL_MAX, >= 0)
 *   precision    SST_PREC_FP32_FFT, or a DFT-as-GEMM tier (SST_PREC_GEMM_BF16,
 *                SST_PREC_GEMM_F16X3) for hop a multiple of 8 and a DFT-matrix table
 *                (4 n_src rows x L taps, 2 bytes each) of at most 64 MiB -- narrow
 *                bands, where 4 n_src L products per frame undercut the FFT;
 *                the relative threshold is taken on the tier's own arithmetic
 *                (as for the FFT tier, see sst_forward); the GEMM tiers are not
 *                supported by the batched calls
 *   flags        reserved, 0
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
} sst_params;

/* Shapes derived at plan time (sst_plan_query). */
typedef struct {
    int64_t n_samples;        /* N */
    int64_t n_frames;         /* ceil(N / hop) */
    int32_t win_len, hop, nfft, subdiv;
    int32_t k1, k2;           /* source-bin band */
    int32_t n_src;            /* k2 - k1 + 1 */
    int32_t n_dst;            /* z (k2 - k1) + 1 */
    size_t workspace_bytes;   /* device workspace the caller must bind */
    size_t t_row_bytes;       /* 8 * n_dst: bytes of one T row (frame) */
} sst_shape;

typedef struct sst_plan_s *sst_plan_t;

/*
 * sst_plan -- validate parameters, build the float64 host tables (windows,
 * centre-phase factors exp(i 2 pi (k M mod N_f)/N_f) of Eq. 9, inverse
 * phasor tables) and choose kernel shapes.  Host only: no HIP call, no device
 * allocation.  *out receives a plan owned by the caller (sst_destroy).
 * Errors: SST_E_ARG (reason in sst_last_error), SST_E_UNSUPPORTED, SST_E_NOMEM.
 */
sst_status sst_plan(const sst_params *params, sst_plan_t *out);

/* sst_plan_query -- fill *out (host only). */
sst_status sst_plan_query(sst_plan_t plan, sst_shape *out);

/*
 * sst_plan_bind -- attach a caller-owned device workspace of at least
 * workspace_bytes bytes (256-byte aligned) and upload the plan's tables with
 * one asynchronous host-to-device copy on `stream`.  The plan keeps the host
 * tables alive, so the call returns at once.  Binding again replaces the
 * workspace.  Errors: SST_E_WORKSPACE, SST_E_DEVICE.
 */
sst_status sst_plan_bind(sst_plan_t plan, void *workspace_dev, size_t bytes, void *stream);

/*
 * Optional per-coefficient / per-frame outputs of sst_forward (debug and
 * parity).  Every pointer may be NULL.  Rows cover the frames of the call.
 *   S        complex float [nframes][n_src]: S[m, k1 + i] of Eq. 9
 *   Sd       complex float [nframes][n_src]: S'[m, k1 + i] (g' window)
 *   idx      int32 [nframes][n_src]: destination l, -1 below threshold,
 *            -2 destination outside [0, n_dst)
 *   colstats double [nframes][3]: sum_l Re T, sum_l Im T, sum_l |T|^2,
 *            accumulated in FP64 from the FP32 row of T by an epilogue of the
 *            forward kernel (it needs none of the per-coefficient outputs;
 *            complex rows only, SST_E_UNSUPPORTED with SST_FWD_OUT_MAG_*)
 *   gamma    float [1]: the threshold gamma used by the call
 *   kernel_events  two hipEvent_t handles (created by the caller), recorded
 *            on the call's stream right before and right after the launch of
 *            the fused forward kernel (or of the GEMM-tier kernel), so that
 *            the caller can time that kernel alone; NULL entries are skipped
 */
typedef struct {
    float *S;
    float *Sd;
    int32_t *idx;
    double *colstats;
    float *gamma;
    void *kernel_events[2];
} sst_fwd_aux;

/*
 * sst_forward -- forward SST of frames [frame0, frame0 + nframes) of x
 * (Eqs. 7-9, 12-14, 27-29): framing with g and g', FP32 FFT pair of size N_f,
 * IF estimate, threshold, selective subdivided reassignment into T.
 *   x        device float [n_samples]; read only
 *   T        device complex float [nframes][n_dst], row r = frame frame0 + r;
 *            every element of the rows is written (zeros included); with
 *            SST_FWD_OUT_MAG_F32 / _F16 it holds float / half |T| instead (the
 *            norm of the complex value, rounded once; not an input of the
 *            inverse, which needs the phase)
 *   aux      optional outputs, may be NULL
 *   flags    0, or SST_FWD_REUSE_GAMMA and at most one SST_FWD_OUT_MAG_*
 * With SST_THR_REL_MAX and no SST_FWD_REUSE_GAMMA, gamma comes from max |S|
 * over ALL frames of x (not only the chunk), on the forward kernel's own
 * arithmetic (FP32 FFT, or the GEMM tier's products).  A call over the whole
 * signal (frame0 = 0, nframes = n_frames, no per-coefficient outputs)
 * computes it speculatively: the maximum over every k-th frame group (or GEMM
 * tile; k from sst_tuning.seed_step) and the running maximum give a lower
 * bound of gamma, each group records the least |S| it kept, and the groups
 * that kept a coefficient at or below the final gamma are transformed again
 * -- T is the same, bit for bit, as with the final gamma given.  Other calls
 * run a maximum pre-pass over all frames first.  Calls on one plan share the
 * workspace: calls that overlap in time on different streams race.
 * Errors: SST_E_ARG (range, NULL x/T), SST_E_STATE, SST_E_DEVICE.
 */
sst_status sst_forward(sst_plan_t plan, const float *x, int64_t frame0, int64_t nframes,
                       float *T, const sst_fwd_aux *aux, uint32_t flags, void *stream);

/*
 * sst_forward_static -- sst_forward for callers that cannot allocate device
 * memory at all: code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The plan needs no sst_plan_bind: its workspace is a
 * fixed array of SST_STATIC_SCRATCH_BYTES inside the library, one per device,
 * held from the library's first use on that device until the process ends.
 * The call allocates nothing (no hipMalloc / hipFree, no allocating library
 * routine); the caller still passes x, T and the optional aux buffers, with
 * the same layout and meaning as for sst_forward.  The first call of a plan
 * on a device (or after another plan used that device's scratch) uploads the
 * plan's tables into the scratch with one asynchronous host-to-device copy
 * on `stream`.
 *   Shared state: every sst_forward_static call on a device uses that
 * device's one scratch array, which keeps the last call's contents (the
 * kernels clear the counters they need).  Calls that overlap in time on one
 * device race, whatever their plans and streams; SST_FWD_REUSE_GAMMA needs
 * the previous static call on the device to have been a thresholding call of
 * the same plan.
 * Errors: as sst_forward; SST_E_UNSUPPORTED when the plan's workspace_bytes
 * exceed SST_STATIC_SCRATCH_BYTES (checked before any device call).
 */
#define SST_STATIC_SCRATCH_BYTES (32u << 20)
sst_status sst_forward_static(sst_plan_t plan, const float *x, int64_t frame0, int64_t nframes,
                              float *T, const sst_fwd_aux *aux, uint32_t flags, void *stream);

/*
 * sst_ridge -- ridge of each component (Sec. 2.2, zone M_q[m]): for every
 * frame of the chunk and component q, the destination bin of largest |T| in
 * [band[2q], band[2q+1]] (clipped to [0, n_dst)); ties go to the smallest l;
 * -1 when the range is all zero.
 *   T        device complex float [nframes][n_dst]
 *   band     host int32 [2 n_comp]: inclusive destination-bin ranges
 *   ridge    device int32 [n_comp][nframes]
 * Errors: SST_E_ARG, SST_E_STATE, SST_E_DEVICE.
 */
sst_status sst_ridge(sst_plan_t plan, const float *T, int64_t nframes, const int32_t *band,
                     int32_t n_comp, int32_t *ridge, void *stream);

/*
 * sst_ridge_guided -- sst_ridge with a search band that follows a guide per
 * frame (e.g. a harmonic order of a measured shaft speed): for frame m and
 * component q the ridge is the first largest |T| in
 * [centre[q][m] + band[2q], centre[q][m] + band[2q+1]] (clipped to [0, n_dst)),
 * -1 when centre[q][m] < 0 or the range is all zero.
 *   centre   device int32 [n_comp][nframes]: guide destination bins
 *   band     host int32 [2 n_comp]: offsets relative to the guide, each in
 *            [-n_dst, n_dst]
 * Errors: as sst_ridge.
 */
sst_status sst_ridge_guided(sst_plan_t plan, const float *T, int64_t nframes,
                            const int32_t *centre, const int32_t *band, int32_t n_comp,
                            int32_t *ridge, void *stream);

/*
 * sst_inverse -- direct downsampled inverse (Eqs. 25-26; zN_f grid for z > 1)
 * of n_comp components from the T rows of frames [frame0, frame0 + nframes):
 *   r[m,j] = (1/N_f) sum_{l in zone} a_l Re(T[m,l] e^{i 2 pi ((z k1 + l) j mod z N_f)/(z N_f)})
 *   xhat_q[n] += sum_{m in chunk} g[n - mH] r[m, n - mH] / sum_{all m} g[0] g[n - mH]
 * zone = [ridge - hw, ridge + hw] intersected with [0, n_dst); a_l = 2 except 1 at
 * DC and at fs/2.  The denominator runs over every frame of the signal, so
 * chunked calls with SST_INV_ACCUMULATE sum to the whole-signal result.
 * Without SST_INV_ACCUMULATE the samples the chunk reaches are overwritten.
 * With SST_INV_EQ15 (hop 1 only): xhat_q[m] = (1/(N_f g[0])) sum_zone a_l Re T[m,l].
 * Arithmetic: the sum over frames runs on the matrix cores with both operands
 * split into FP16 hi + lo parts (22 significant bits each, power-of-two scaled)
 * and FP32 accumulation; phases, weights and the denominator are FP32/FP64 as
 * above.  Measured against an FP64 evaluation: about 3e-7 relative.
 *   T        device complex float [nframes][n_dst]
 *   ridge    device int32 [n_comp][nframes]; -1 = no contribution from that frame
 *   hw       zone half-width in destination bins, >= 0
 *   xhat     device float [n_comp][n_samples]
 *   xref     optional device float [n_comp][n_samples] (noise-free components)
 *   err      optional device double [n_comp][2]: sum (xref - xhat)^2 and sum xref^2
 *            over n in [M, N - M), FP64 (Eq. 33); needs xref and a whole-signal call
 * Errors: SST_E_ARG, SST_E_STATE, SST_E_DEVICE, SST_E_UNSUPPORTED (n_comp * ceil(span / 256)
 * >= 2^31, or a window too long for the hop to fit the per-tile tables).
 */
sst_status sst_inverse(sst_plan_t plan, const float *T, int64_t frame0, int64_t nframes,
                       const int32_t *ridge, int32_t n_comp, int32_t hw, float *xhat,
                       const float *xref, double *err, uint32_t flags, void *stream);

/*
 * Batched form: many channels, each with its own parameters (length, hop,
 * N_f, window, band, subdivision, threshold), processed by one persistent
 * launch per group of channels that share N_f and the pass-1 tap-row count
 * (so a mixed batch of three DFT sizes is three launches, which a caller
 * may capture in one hipGraph).  Work items are (channel, group of frames);
 * every item computes exactly what sst_forward computes for that channel,
 * with the same kernels, so a channel's T is bit-identical to a
 * single-channel sst_forward of it.  Calls follow the single-channel rules:
 * asynchronous on `stream`, caller-owned device memory, no device allocation.
 */
typedef struct sst_batch_s *sst_batch_t;

/*
 * sst_batch_plan -- validate and plan n_channels channels (params[c] as for
 * sst_plan).  Host only.  Errors as sst_plan (the message names the channel).
 */
sst_status sst_batch_plan(const sst_params *params, int32_t n_channels, sst_batch_t *out);

/*
 * sst_batch_query -- shape of channel c (as sst_plan_query; its
 * workspace_bytes is the whole batch's workspace).
 */
sst_status sst_batch_query(sst_batch_t batch, int32_t c, sst_shape *out);

/*
 * sst_batch_bind -- attach one caller-owned workspace (256-byte aligned, at
 * least workspace_bytes) and upload every channel's tables on `stream`.
 */
sst_status sst_batch_bind(sst_batch_t batch, void *workspace_dev, size_t bytes, void *stream);

/*
 * sst_batch_set_io -- record channel c's device buffers (host only):
 *   x      float [n_samples of c]
 *   T      complex float [n_frames of c][n_dst of c], whole signal; channels
 *          processed by different forward calls may share T memory
 *   ridge  int32 [n_comp][n_frames] (inverse; may be NULL for forward-only use)
 *   n_comp components, hw zone half-width (inverse)
 *   xhat   float [n_comp][n_samples] (inverse)
 *   xref, err  optional, as for sst_inverse
 * Takes effect at the next sst_batch_commit.
 */
sst_status sst_batch_set_io(sst_batch_t batch, int32_t c, const float *x, float *T,
                            const int32_t *ridge, int32_t n_comp, int32_t hw, float *xhat,
                            const float *xref, double *err);

/*
 * sst_batch_commit -- upload the per-channel descriptors built from the
 * recorded buffers.  Blocks until the upload is done (setup call; not for
 * graph capture).  Errors: SST_E_STATE (not bound), SST_E_DEVICE.
 */
sst_status sst_batch_commit(sst_batch_t batch, void *stream);

/*
 * sst_batch_forward -- forward SST (as sst_forward over every frame) of
 * channels [c_begin, c_end): relative thresholds are computed per channel
 * unless SST_FWD_REUSE_GAMMA.  Kernel launches only, so it can be captured.
 * Errors: SST_E_ARG (range, a channel without x or T), SST_E_STATE, SST_E_DEVICE.
 */
sst_status sst_batch_forward(sst_batch_t batch, int32_t c_begin, int32_t c_end, uint32_t flags,
                             void *stream);

/*
 * sst_batch_inverse -- direct inverse (as sst_inverse over every frame, no
 * flags) of every component of channels [c_begin, c_end) in one launch.
 * Kernel launches only.  Errors: SST_E_ARG (a channel without ridge/xhat),
 * SST_E_STATE, SST_E_UNSUPPORTED (z N_f > 65536), SST_E_DEVICE.
 */
sst_status sst_batch_inverse(sst_batch_t batch, int32_t c_begin, int32_t c_end, void *stream);

/* sst_batch_destroy -- release the batch's host memory. */
void sst_batch_destroy(sst_batch_t batch);

/*
 * Launch choices of a plan.  None of them changes T (every forward variant
 * computes each row with the same arithmetic); the inverse tile width changes
 * xhat only at the rounding level (about 1e-7 relative).  0 = the library's
 * default.
 *   fwd_wg_per_cu  forward workgroups kept resident per CU (1 .. what fits;
 *                  larger values are capped)
 *   seed_step      speculative relative threshold: seed the running maximum
 *                  with every seed_step-th frame group (>= 1)
 *   inv_tf         inverse: groups of 256 output samples per workgroup, 1, 4
 *                  or 8 (4 only when the frames 1024 samples meet fit the
 *                  staged block; 8 when the frames 2048 samples meet fit it
 *                  and the hop-decimated window table fits; SST_E_UNSUPPORTED
 *                  otherwise); 0 = the widest that fits (or 4 when inv_groups
 *                  asks for 2 or 4)
 *   inv_groups     inverse with inv_tf 4: destination groups of 16 bins staged
 *                  together, 1 (one at a time), 2 or 4 (groups of the tile's
 *                  zones together, sharing each window operand read and each
 *                  sample's phasors; needs the hop-decimated window table and
 *                  the staged groups within a third (2) or half (4) of the
 *                  CU's LDS, SST_E_UNSUPPORTED otherwise); 0 = 1
 */
typedef struct {
    int32_t fwd_wg_per_cu;
    int32_t seed_step;
    int32_t inv_tf;
    int32_t inv_groups;
} sst_tuning;

/* sst_plan_get_tuning -- the choices in effect (defaults resolved where known:
 * fwd_wg_per_cu after bind, inv_tf and inv_groups always; seed_step 0 =
 * automatic). */
sst_status sst_plan_get_tuning(sst_plan_t plan, sst_tuning *out);

/* sst_plan_set_tuning -- set the launch choices (before or after bind).
 * Errors: SST_E_ARG (negative values, inv_tf not 0/1/4/8, inv_groups not
 * 0/1/2/4), SST_E_UNSUPPORTED. */
sst_status sst_plan_set_tuning(sst_plan_t plan, const sst_tuning *tuning);

/*
 * sst_autotune -- search the launch choices of a bound plan on the caller's
 * buffers and keep the fastest: every forward choice (workgroups per CU,
 * threshold seed step) is timed over the whole signal with HIP events, then,
 * when ridge and xhat are given, every inverse tile width.  Each candidate
 * runs once untimed and `reps` times timed (reps >= 1); when those take under
 * 20 ms in all, it is timed again over as many calls as fill about 20 ms (at
 * most 1000) and that mean is used.  Blocks until done
 * (a set-up call); T and xhat hold the last candidate's results.
 *   x, T           as for sst_forward over all frames
 *   ridge, n_comp, hw, xhat   as for sst_inverse (optional: NULL ridge skips
 *                  the inverse choices)
 *   best           optional: receives the chosen values
 * Errors: SST_E_ARG, SST_E_STATE (not bound), SST_E_DEVICE.
 */
sst_status sst_autotune(sst_plan_t plan, const float *x, float *T, const int32_t *ridge,
                        int32_t n_comp, int32_t hw, float *xhat, int32_t reps, void *stream,
                        sst_tuning *best);

/*
 * sst_tuning_save / sst_tuning_load -- a JSON cache of tuned choices keyed by
 * the device architecture and the plan's shape ("gfx950 nfft=.. L=.. H=..
 * n_src=.. n_dst=.. prec=.."), one entry per line.  save inserts or replaces
 * the plan's entry with its current choices; load applies the plan's entry
 * (SST_E_ARG when the file or the entry is missing).  sst_plan and
 * sst_batch_plan apply the entry of each plan from the file named by the
 * environment variable SST_TUNE_CACHE, when it holds one.  Host only.
 */
sst_status sst_tuning_save(sst_plan_t plan, const char *path);
sst_status sst_tuning_load(sst_plan_t plan, const char *path);

/*
 * sst_stft -- the STFT product alone (Sec. 2.1, Eqs. 7-9): S (and, when Sd is
 * not NULL, S' with the window g') of frames [frame0, frame0 + nframes), in-band
 * bins k1..k2, with the centre phase of Eq. 9 -- the values sst_forward's
 * debug output S holds, on the same FP32 FFT pair.
 *   S, Sd    device complex float [nframes][n_src], row r = frame frame0 + r
 * Errors: SST_E_ARG, SST_E_STATE, SST_E_DEVICE.
 */
sst_status sst_stft(sst_plan_t plan, const float *x, int64_t frame0, int64_t nframes, float *S,
                    float *Sd, void *stream);

/*
 * sst_stft_inverse -- STFT synthesis (Sec. 2.1, Eqs. 10-11) of the whole signal
 * from in-band rows: per frame, the centre phase removed and an N_f-point
 * inverse DFT of the one-sided spectrum (bins k1..k2; 2 Re(.) for interior
 * bins, Re(.) at DC and at fs/2), windowed by g and overlap-added:
 *   xhat[n] = sum_m g[n - mH] s[m, n - mH] / sum_m g[n - mH]^2,
 *   s[m, j] = (1/N_f) sum_k a_k Re(S[m, k] e^{+i 2 pi k j / N_f}).
 * With the full band (f_lo = 0, f_hi = fs/2) it reconstructs x exactly up to
 * rounding; with a narrower band, the band-limited part.
 *   S     device complex float [n_frames][n_src] (sst_stft of every frame)
 *   xhat  device float [n_samples]
 * Errors: SST_E_ARG, SST_E_STATE, SST_E_DEVICE.
 */
sst_status sst_stft_inverse(sst_plan_t plan, const float *S, float *xhat, void *stream);

/*
 * sst_renyi -- Renyi entropy (Sec. 3, Eq. 32) of a time-frequency
 * representation, the paper's measure of TF concentration, with P = |C|^2:
 *   R = 1/(1 - alpha) log2( sum over the grid of (P / sum P)^alpha )
 * (discrete form: the constant log2 of the cell area is left out, so one
 * occupied cell gives 0 and K equal cells log2 K).  Plan-independent.
 *   C      device array [rows][ld] of kind SST_RENYI_COMPLEX64 (complex float,
 *          e.g. T or S rows), SST_RENYI_MAG_F32 (float |C|) or SST_RENYI_MAG_F16
 *          (half |C|); only the first cols of each row are read
 *   alpha  integer order, 2 <= alpha <= 4 (the paper uses 3)
 *   work   device double [SST_RENYI_WORK_DOUBLES] (per-workgroup partial sums)
 *   out    device double [3]: sum P, sum P^alpha (float64), R in bits
 *          (NaN when every P is 0)
 * The float64 sums are reduced in a fixed order: the result does not depend
 * on scheduling.  Asynchronous on `stream`.  Errors: SST_E_ARG.
 */
#define SST_RENYI_COMPLEX64 0
#define SST_RENYI_MAG_F32 1
#define SST_RENYI_MAG_F16 2
#define SST_RENYI_WORK_DOUBLES 2048
sst_status sst_renyi(const void *C, int32_t kind, int64_t rows, int32_t cols, int64_t ld,
                     int32_t alpha, double *work, double *out, void *stream);

/* sst_destroy -- release the plan's host memory (the workspace stays the caller's). */
void sst_destroy(sst_plan_t plan);

/* sst_status_string -- static text for a status code. */
const char *sst_status_string(sst_status status);

/* sst_last_error -- thread-local detail of the last failing call on this thread. */
const char *sst_last_error(void);

/*
 * sst_critical_hf -- plan-time advisory bounds on H_f = N/N_f (Sec. 4):
 *   Eq. 38: H_f < 3N / (4 pi sigma fs)           (reassignment still acts)
 *   Eq. 46: H_f < sqrt(2) N / (2 pi sigma fs)    (no global reassignment)
 * sigma_s in seconds.  Host only.  Errors: SST_E_ARG for non-positive inputs.
 */
sst_status sst_critical_hf(double n, double sigma_s, double fs, double *eq38, double *eq46);

#ifdef __cplusplus
}
#endif

#endif /* SST_H */
