// Internal interface between the host runtime (sst_host.cpp) and the gfx950
// kernels (sst_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace sst {

// Device-side control block at the start of the workspace.
struct Ctrl {
    float gamma;        // threshold |S| > gamma
    float gamma2;       // gamma^2 (the kernels compare |A|^2 > gamma^2)
    float maxabs2;      // max |S|^2 found by the threshold pre-pass
    unsigned maxbits;   // running max |S|^2 as float bits (atomicMax on non-negative floats)
    float pad[60];
};
static_assert(sizeof(Ctrl) == 256, "control block is one 256-byte slot");

// Per-channel descriptor read (through the scalar cache) by the threshold
// and forward kernels.  A launch processes a contiguous list of descriptors
// whose channels share N_f; single-channel calls use a list of one.
struct ChanDesc {
    const float *x;         // [n] signal
    int64_t n;              // signal length
    int64_t n_frames;       // frames of the whole signal: ceil(n / hop)
    int64_t frame0;         // first frame of the forward call
    int64_t nframes;        // frames of the forward call
    int64_t item0;          // forward items (F frames each) of the launch list before this channel
    int64_t item_end;       // item0 + ceil(nframes / F)
    int64_t mitem0;         // threshold items (F frame pairs each) before this channel
    int64_t mitem_end;      // mitem0 + ceil(ceil(n_frames / 2) / F) (relative threshold), else mitem0
    const float2 *win;      // [L]: (g[j], s * g'[j]), j = -M..M
    Ctrl *ctrl;             // threshold of this channel
    float2 *T;              // [nframes][n_dst]
    float2 *S;              // optional [nframes][n_src]
    float2 *Sd;             // optional [nframes][n_src]
    int32_t *idx;           // optional [nframes][n_src]
    double *colstats;       // optional [nframes][3]
    int L, M, hop, k1, n_src, n_dst, z, thr_mode;
    float thr;              // gamma (absolute) or rho (relative)
    float inv_s;            // 1/s: S' = B / s
    float cdelta;           // N_f / (2 pi s): delta (bins) = cdelta Im(B conj A) / |A|^2
    int out_fmt;            // rows of T: 0 complex float, 1 float |T|, 2 half |T|
};

// One launch of the threshold or forward kernel over descriptors ch[0 .. n_ch).
struct GroupLaunch {
    const ChanDesc *ch;     // device array
    int n_ch;
    int64_t item_begin;     // first item: ch[0].item0 (forward) or ch[0].mitem0 (threshold)
    int64_t item_stop;      // ch[n_ch-1].item_end or .mitem_end
    const float2 *twid;     // [N_f]: exp(-i 2 pi r / N_f), shared by the launch
    int step;               // max-only pre-pass: visit every step-th item (0 or 1: all)
    int spec;               // forward: threshold each item at a lower bound of gamma
    float *smin;            // spec: per item (launch numbering), least |S|^2 kept
    int32_t *list;          // forward: only the items list[0 .. *list_n) (fix-up pass)
    int32_t *list_n;        // count of list; cleared by launch_clear_max when non-null
};

// Per-channel descriptor of the direct inverse (one call's frames of one
// channel, every component).  Launches cover a contiguous list of them.
struct InvDesc {
    const float2 *T;        // [nframes][n_dst] rows of the call
    const int32_t *ridge;   // [n_comp][nframes]
    float *xhat;            // [n_comp][n]
    const float *xref;      // optional [n_comp][n]
    double *err;            // optional [n_comp][2]
    const float2 *win;      // [L]; .x = g[j]
    const float2 *ph_lo;    // [1 << lo_bits]: exp(+i 2 pi r / G), r < 2^lo_bits
    const float2 *ph_hi;    // [G >> lo_bits]: exp(+i 2 pi (h << lo_bits) / G)
    const float *den;       // [hop]: sum_m g[0] g[n - mH] for samples n = r mod hop whose
                            // frames all exist
    int64_t n;              // signal length
    int64_t n_frames;       // all frames of the signal
    int64_t frame0, nframes;
    int64_t span_lo;        // first output sample the call reaches
    int64_t span_len;       // number of output samples the call reaches
    int64_t blk0;           // workgroups of the launch list before this channel
    int64_t blk_end;        // blk0 + n_comp * tiles
    int64_t tiles;          // ceil(span_len / 256)
    int L, M, hop, nfft, k1, z, n_dst, hw, n_comp;
    int G;                  // z * N_f (phase grid of the inverse)
    int lo_bits;            // split of the phase-table index
    int g_pow2;             // G is a power of two
    float inv_G;            // 1/G
    float inv_nfft;
    float g_scale;          // 2^tg: the window's largest |g[j]| 2^tg lies in [2^13, 2^14)
    float g_unscale;        // 2^-tg
    int dec_reach;          // JL = M + 63 + 16 H: window indices of the decimated table
    int dec_row;            // (2 JL) / H + 2: words per residue row of that table
    int accumulate;         // add into xhat
    int pad_;
};

// One inverse launch over descriptors ch[0 .. n_ch).
struct InvLaunch {
    const InvDesc *ch;      // device array
    int n_ch;
    int max_k;              // most frames one output tile meets
    int64_t blk_begin;      // ch[0].blk0
    int max_tab;            // LDS float2 entries of the largest phase tables in the list
    int max_gtab;           // LDS words of the largest window table in the list
    int dec;                // window tables decimated by the hop (inv_gtab_words)
    int tf;                 // groups of kInvTileSamples per workgroup (1, kInvWideTF or
                            // kInvXWideTF; the last needs dec)
    int groups;             // groups of 16 destinations staged together (1, 2 or 4; 2 and 4
                            // need tf > 1 and dec)
};

// Words of a channel's inverse window table: decimated by the hop,
// H dec_row, when that is at most kInvDecMax; otherwise L + 2 (indices
// clamped).
constexpr int kInvDecMax = 10240;

constexpr int kInvTileSamples = 256;   // output samples per group of four inverse waves
constexpr int kInvWideTF = 4;          // groups per workgroup of the wide inverse tiles
constexpr int kInvXWideTF = 8;         // groups per workgroup of the extra-wide tiles
constexpr int kInvWideKB = 144;        // frames a wide tile may meet (one staged block)
// LDS of the grouped inverse with g groups staged: three workgroups per CU
// for two groups, two for four
constexpr size_t inv_group_lds_max(int g) { return g >= 4 ? 80 * 1024 : 53 * 1024; }

// Precision tiers of the DFT-as-GEMM forward (values of sst_params.precision).
constexpr int SST_GEMM_BF16 = 1;
constexpr int SST_GEMM_F16X3 = 2;

// Arguments of the DFT-as-GEMM forward kernel.
struct GemmArgs {
    const float *x;
    int64_t n;
    int64_t frame0, nframes;
    const void *afrag;      // [row_tiles][ksteps][64] 16-byte A fragments (BF16, or FP16 hi)
    const void *afrag_lo;   // FP16 lo fragments (F16X3)
    const float2 *win;      // [L]: .x = g[j]
    const Ctrl *ctrl;       // gamma2
    float2 *T;              // [nframes][n_dst]
    float2 *S;              // optional [nframes][n_src]
    float2 *Sd;             // optional [nframes][n_src]
    int32_t *idx;           // optional [nframes][n_src]
    int L, M, hop, k1, n_src, n_dst, z;
    int row_tiles;          // ceil(4 n_src / 32)
    int ksteps;             // K / 16, K = L rounded up to 16
    int slab;               // staged samples per tile: (FT - 1) hop + K
    float unscale_g;        // 2^-s of the g rows (FP16 split), else 1
    float unscale_gd;       // same for the g' rows
    float cdelta;           // N_f / (2 pi)
    float bound_c;          // 1.1 sqrt(2 n_src N_f)
    float gmax2;            // max_j g[j]^2
    // Threshold (relative gamma on the tier's own arithmetic):
    //   mode 0: forward of every tile; spec: gamma from the running maximum
    //     (a lower bound), recording each tile's least kept |S|^2 in smin and
    //     folding its max |S|^2 into ctrl->maxbits;
    //   mode 1: max |S|^2 only, of every tile_step-th tile, into ctrl->maxbits;
    //   mode 2: forward of the tiles listed in list[0 .. *list_n).
    int mode;
    int spec;
    int64_t tile_step;
    int thr_mode;
    float thr;
    Ctrl *ctrlw;            // the same control block, written (maxbits)
    float *smin;            // [tiles]
    const int32_t *list;
    const int32_t *list_n;
};

// Arguments of the ridge kernel.
struct RidgeArgs {
    const float2 *T;
    int64_t nframes;
    int n_dst;
    int n_comp;
    int band[2 * 16];       // inclusive [lo, hi] per component (at most 16); relative
                            // to centre[q][m] when centre is given
    const int32_t *centre;  // optional [n_comp][nframes] guide bins (-1: no ridge)
    int32_t *ridge;         // [n_comp][nframes]
};

// STFT synthesis (Eqs. 10-11) from in-band rows [n_frames][n_src].
constexpr int kSynTile = 2048;   // output samples per synthesis workgroup
struct SynArgs {
    const float2 *S;        // [n_frames][n_src], bins k1..k2, centre phase included (Eq. 9)
    const float2 *win;      // [L]: .x = g[j]
    const float *den2;      // [hop]: sum of g[j]^2 over j = r mod hop, |j| <= M
    const float2 *twid;     // [N_f]: exp(-i 2 pi r / N_f)
    float *xhat;            // [n]
    int64_t n, n_frames;
    int M, hop, k1, k2, n_src;
    float inv_nfft;
};
hipError_t launch_synthesis(int nfft, const SynArgs &a, hipStream_t s);
// STFT product: S (and S') rows of the items of g (forward numbering).
hipError_t launch_stft(int nfft, int L, const GroupLaunch &g, int grid, hipStream_t s);

// Arguments of the Renyi-entropy reduction (sst_analysis.hip).
constexpr int kRenyiParts = 1024;   // per-workgroup partial sums (work holds 2 per part)
struct RenyiArgs {
    const void *C;          // [rows][ld] complex float, float or half magnitudes
    int64_t rows;
    int64_t ld;             // row stride in elements
    int64_t rows_per;       // rows per workgroup (set by the launcher)
    int cols;
    int alpha;              // integer order >= 2
    double *work;           // [2 kRenyiParts]
    double *out;            // [3]: sum P, sum P^alpha, R in bits
};
hipError_t launch_renyi(const RenyiArgs &a, int kind, hipStream_t s);

// Launchers (sst_kernels.hip).  Each returns the hipError_t of its launch.
// Pieces of the threshold of the FFT path (launch_gamma and launch_spec_list
// serve the GEMM tiers too).  launch_clear_max zeroes maxbits of
// every channel (and *g.list_n); launch_max_prepass folds max |S|^2 of every
// g.step-th forward item of the whole signals (items numbered by mitem0, with
// the forward kernel's own arithmetic) into maxbits; launch_gamma sets gamma.
hipError_t launch_clear_max(const GroupLaunch &g, hipStream_t s);
hipError_t launch_max_prepass(int nfft, int L, const GroupLaunch &g, int grid, hipStream_t s);
hipError_t launch_gamma(const GroupLaunch &g, hipStream_t s);
// After a speculative forward: sets gamma of every channel (as launch_gamma)
// and appends to g.list the items whose least kept |S|^2 does not exceed the
// final gamma^2.
hipError_t launch_spec_list(const GroupLaunch &g, hipStream_t s);
// Forward variants: production; debug (writes S, S', idx, colstats); stats
// (production arithmetic with the colstats epilogue, single channel).
constexpr int kFwdKindPlain = 0;
constexpr int kFwdKindDebug = 1;
constexpr int kFwdKindStats = 2;
// max_n_src / max_n_dst / max_L bound the launch's channels.
hipError_t launch_forward(int nfft, int max_L, int max_n_src, int max_n_dst, int kind,
                          const GroupLaunch &g, int grid, hipStream_t s);
// DFT-as-GEMM forward (FT frames per tile: 32 or 64).
hipError_t launch_gemm_forward(int prec, int ft, bool debug, const GemmArgs &a, int grid,
                               hipStream_t s);
size_t gemm_lds_bytes(int prec, int ft, int n_dst, int slab, int L);
int gemm_occupancy(int prec, int ft, size_t lds);
// Copy one descriptor into device memory (a kernel, so it can be captured);
// with clear_max also zero d.ctrl->maxbits, and *list_n when non-null.
hipError_t launch_put_desc(const ChanDesc &d, ChanDesc *dst, bool clear_max, int32_t *list_n,
                           hipStream_t s);
// Inverse of the launch list (blocks = ch[n_ch-1].blk_end - blk_begin).
// Clears err first when `clear_err`.
hipError_t launch_inverse(const InvLaunch &l, int64_t blocks, bool clear_err, hipStream_t s);
// Eq. 15 for one descriptor (host copy `a`, device copy `dev`).
hipError_t launch_inverse_eq15(const InvDesc &a, const InvDesc *dev, float inv_nfft_g0,
                               hipStream_t s);
hipError_t launch_put_inv_desc(const InvDesc &d, InvDesc *dst, hipStream_t s);
size_t inv_lds_bytes(const InvLaunch &l);
hipError_t launch_ridge(const RidgeArgs &a, hipStream_t s);

// Static scratch of sst_forward_static: the device address of this device's
// copy of a fixed array of kStaticScratchBytes (looked up once per device,
// with `dev` current).  kMaxDevices bounds the device ordinals served.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
hipError_t static_scratch(int dev, unsigned char **out);

// Kernel geometry, shared so the host can size grids and workspaces.
int fwd_frames_per_iter(int nfft);   // F
int fwd_threads(int nfft);           // threads per workgroup
int fwd_lds_elems(int nfft);         // float2 capacity of the LDS buffer
int fwd_occupancy(int nfft, int L);  // resident workgroups per CU (forward)
int fwd_rounds(int nfft, int n_src);          // coefficient rounds per thread: 3, 5 or 9
size_t fwd_lds_bytes(int nfft);               // LDS of the forward kernel

}  // namespace sst
