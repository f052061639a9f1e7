// Internal interface between the host runtime (sst_host.cpp) and the gfx950
// kernels (sst_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace sst {

// Device-side control block at the start of the workspace.
struct Ctrl {
    float gamma;    // threshold |S| > gamma
    float gamma2;   // gamma^2 (the kernels compare |A|^2 > gamma^2)
    float maxabs2;  // max |S|^2 found by the threshold pre-pass
    float pad[61];
};
static_assert(sizeof(Ctrl) == 256, "control block is one 256-byte slot");

// Arguments of the fused forward kernel (framing, FFT pair, IF, reassignment).
struct FwdArgs {
    const float *x;         // [n]
    int64_t n;              // signal length
    int64_t frame0;         // first frame of the call
    int64_t nframes;        // frames in the call
    const float2 *win;      // [L]: (g[j], s * g'[j]), j = -M..M
    const float2 *cphase;   // [n_src]: exp(+i 2 pi ((k M) mod N_f) / N_f)
    const float2 *twid;     // [N_f]: exp(-i 2 pi r / N_f)
    const Ctrl *ctrl;       // gamma2
    float2 *T;              // [nframes][n_dst]
    float2 *S;              // optional [nframes][n_src]
    float2 *Sd;             // optional [nframes][n_src]
    int32_t *idx;           // optional [nframes][n_src]
    double *colstats;       // optional [nframes][3]
    int L, M, hop, k1, n_src, n_dst, z;
    float2 cph_step;        // exp(+i 2 pi ((NT M) mod N_f) / N_f), NT = threads per workgroup
    float inv_s;            // 1/s: S' = B / s
    float cdelta;           // N_f / (2 pi s): delta (bins) = cdelta Im(B conj A) / |A|^2
};

// Arguments of the threshold pre-pass (max |S|^2 over every frame and in-band bin).
struct MaxArgs {
    const float *x;
    int64_t n;
    int64_t n_frames;       // all frames of the signal
    const float2 *win;
    const float2 *twid;
    float *partial;         // [gridDim.x]
    int L, M, hop, k1, n_src;
};

// Arguments of the direct inverse kernel.
struct InvArgs {
    const float2 *T;        // [nframes][n_dst] rows of the chunk
    const int32_t *ridge;   // [n_comp][nframes]
    float *xhat;            // [n_comp][n]
    const float *xref;      // optional [n_comp][n]
    double *err;            // optional [n_comp][2]
    const float2 *win;      // [L]; .x = g[j]
    const float2 *ph_lo;    // [1 << lo_bits]: exp(+i 2 pi r / G), r < 2^lo_bits
    const float2 *ph_hi;    // [G >> lo_bits]: exp(+i 2 pi (h << lo_bits) / G)
    int64_t n;              // signal length
    int64_t n_frames;       // all frames of the signal
    int64_t frame0, nframes;
    int64_t span_lo;        // first output sample the chunk reaches
    int64_t span_len;       // number of output samples the chunk reaches
    int L, M, hop, nfft, k1, z, n_dst, hw, n_comp;
    int G;                  // z * N_f (phase grid of the inverse)
    int lo_bits;            // split of the phase-table index
    int g_pow2;             // G is a power of two
    float inv_G;            // 1/G
    float inv_nfft;
    int accumulate;         // add into xhat
    int fb;                 // frames staged per LDS block
};

// Arguments of the ridge kernel.
struct RidgeArgs {
    const float2 *T;
    int64_t nframes;
    int n_dst;
    int n_comp;
    int band[2 * 16];       // inclusive [lo, hi] per component (at most 16)
    int32_t *ridge;         // [n_comp][nframes]
};

// Launchers (sst_kernels.hip).  Each returns the hipError_t of its launch.
hipError_t launch_threshold(int nfft, const MaxArgs &a, Ctrl *ctrl, int mode, float thr,
                            int grid, hipStream_t s);
hipError_t launch_forward(int nfft, const FwdArgs &a, int grid, hipStream_t s);
hipError_t launch_inverse(const InvArgs &a, hipStream_t s);
hipError_t launch_inverse_eq15(const InvArgs &a, float inv_nfft_g0, hipStream_t s);
hipError_t launch_ridge(const RidgeArgs &a, hipStream_t s);

// Kernel geometry, shared so the host can size grids and workspaces.
int fwd_frames_per_iter(int nfft);   // F
int fwd_threads(int nfft);           // threads per workgroup
int fwd_lds_elems(int nfft);         // float2 capacity of the LDS buffer
int fwd_occupancy(int nfft, int L, int n_src);  // resident workgroups per CU (forward)
int max_occupancy(int nfft, int L);  // resident workgroups per CU (threshold pre-pass)
size_t inv_lds_bytes(const InvArgs &a);
size_t fwd_dyn_lds(int nfft, int n_src);      // dynamic LDS of the forward kernel
int fwd_rounds(int nfft, int n_src);          // coefficient rounds per thread: 3, 5 or 9
size_t fwd_lds_bytes(int nfft, int n_src);    // static + dynamic LDS of the forward kernel

}  // namespace sst
