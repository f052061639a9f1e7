// gfx950 DFT-as-GEMM forward kernel of the downsampled SST (precision tier).
//
// Method: He & Cao, arXiv 2003.07065.  The in-band STFT pair of Eq. 9 (with its
// centre phase) is a matrix product: for FT consecutive frames m,
//   C[r, m] = sum_j A[r, j] X[j, m],   X[j, m] = x[mH - M + j]  (j < L),
// where row r = 4 b + p of A holds, for source bin k = k1 + b and tap t = j - M,
//   p = 0: g[t] cos(2 pi (k t mod N_f) / N_f)     (Re S)
//   p = 1: -g[t] sin(...)                        (Im S)
//   p = 2, 3: the same with g' (Re S', Im S').
// A is built once on the host in float64 and rounded to BF16, or split into
// FP16 hi + lo parts (each scaled by a power of two into FP16's range); X is the
// frames' sample slab staged in LDS.  The products run on the matrix cores
// (32x32x16 MFMA, FP32 accumulation): one product for BF16, three for the
// FP16 split (hi*hi + hi*lo + lo*hi).  The epilogue works straight from the
// accumulators: each lane holds the four rows of a bin for one frame, so it
// evaluates the IF estimate and the destination (Eqs. 12-13, 27-29) and adds
// S to the frame's destination histogram in LDS (Eq. 28), which is streamed to
// HBM as rows of T once every row tile is done.
//
// Histogram arithmetic.  As in the FFT kernel the sums are 32-bit fixed-point
// integers (order independent), but the scale must be fixed before the first
// row tile: by Parseval, sum_k |S_k|^2 <= N_f sum_j x_j^2 g_j^2 over all N_f
// bins, hence sum over the n_src band bins of (|Re S| + |Im S|) is at most
// sqrt(2 n_src N_f sum_j x_j^2 g_j^2), taken with a 10 % margin for the
// rounding of the low-precision products; sum_j x_j^2 g_j^2 is bounded in turn
// by max g^2 times the sums of squares of the 8-sample groups that cover the
// frame's window (about one bit of scale lost against the exact sum).
//
// Layouts (32x32x16 MFMA, checked on the hardware): lane l holds A rows
// l mod 32 with k = 8 (l / 32) .. +7, B columns (frames) l mod 32 with the same
// k, and accumulator i holds row 8 (i / 4) + 4 (l / 32) + i mod 4, column l mod
// 32.  With rows ordered 4 b + p, accumulators 4q .. 4q+3 of a lane are the
// four parts of bin 2q + l / 32 of the row tile for frame l mod 32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sst_internal.h"

namespace sst {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

constexpr int kBufferWord3 = 0x00020000;   // raw buffer, 32-bit data format
constexpr int kNonTemporal = 2;
constexpr int NT = 256;                    // threads per workgroup (4 waves)

// Power-of-two scale 2^K with B 2^K < 2^31 (B >= 0), clamped to [2^-100, 2^100].
__device__ __forceinline__ float fixed_scale(float B)
{
    int e = 0;
    frexpf(B, &e);
    int K = B > 0.f ? 31 - e : 0;
    K = K > 100 ? 100 : (K < -100 ? -100 : K);
    return ldexpf(1.0f, K);
}

template <int PREC>
__device__ __forceinline__ f32x16 mma(u4v a, u4v b, f32x16 c)
{
    if constexpr (PREC == SST_GEMM_BF16)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// Low-precision copy of one sample: BF16 (round to nearest even), or the FP16
// hi part and the FP16 rounding of the remainder.
template <int PREC>
__device__ __forceinline__ void split(float v, unsigned short &hi, unsigned short &lo)
{
    if constexpr (PREC == SST_GEMM_BF16) {
        hi = __builtin_bit_cast(unsigned short, (__bf16)v);
        lo = 0;
    } else {
        const _Float16 h = (_Float16)v;
        hi = __builtin_bit_cast(unsigned short, h);
        lo = __builtin_bit_cast(unsigned short, (_Float16)(v - (float)h));
    }
}

template <int PREC>
__device__ __forceinline__ float widen(unsigned short hi, unsigned short lo)
{
    if constexpr (PREC == SST_GEMM_BF16)
        return (float)__builtin_bit_cast(__bf16, hi);
    else
        return (float)__builtin_bit_cast(_Float16, hi) + (float)__builtin_bit_cast(_Float16, lo);
}

__device__ __forceinline__ float gamma2_rel(int thr_mode, float thr, float max2)
{
    const float gm = thr_mode == 1 ? thr * sqrtf(max2) : thr;
    return gm * gm;
}

__device__ __forceinline__ float block_max(float v, float *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    const float r = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __syncthreads();
    return r;
}

// FT frames per tile (32 or 64: one or two 32-frame column tiles).
template <int PREC, int FT, bool DEBUG>
__global__ __launch_bounds__(NT, 2) void gemm_kernel(GemmArgs a)
{
    constexpr int CT = FT / 32;               // column tiles
    constexpr bool SPLIT = PREC == SST_GEMM_F16X3;
    extern __shared__ __align__(16) unsigned char smem[];
    const int slab = a.slab;                  // samples staged per tile (multiple of 8)
    const int ngrp = slab / 8;                // groups of 8 staged samples
    int *hist = reinterpret_cast<int *>(smem);                        // [FT][n_dst][2]
    unsigned short *xhi = reinterpret_cast<unsigned short *>(hist + 2 * FT * a.n_dst);
    unsigned short *xlo = xhi + slab;                                 // SPLIT only
    float *gsq = reinterpret_cast<float *>(xlo + (SPLIT ? slab : 0)); // [ngrp]: sum x^2
    float *scf = gsq + ((ngrp + 3) & ~3);                             // [FT]
    float *iscf = scf + FT;                                           // [FT]
    float *red = iscf + FT;                                           // [4]

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 31, half = lane >> 5;
    const int64_t n_tiles = (a.nframes + FT - 1) / FT;
    const u4v *__restrict__ afrag = reinterpret_cast<const u4v *>(a.afrag);
    const u4v *__restrict__ afrag_lo = reinterpret_cast<const u4v *>(a.afrag_lo);
    const bool maxonly = a.mode == 1;
    const bool spec = a.mode == 0 && a.spec;
    const int64_t n_visit = a.mode == 2 ? (int64_t)*a.list_n
                            : (maxonly ? (n_tiles + a.tile_step - 1) / a.tile_step : n_tiles);

    for (int64_t v = blockIdx.x; v < n_visit; v += gridDim.x) {
        const int64_t tile = a.mode == 2 ? (int64_t)a.list[v] : (maxonly ? v * a.tile_step : v);
        // Speculative relative threshold: the running maximum is at most the
        // final one, so the gamma it gives is a lower bound (a superset of the
        // coefficients is kept; the tiles that kept one at or below the final
        // gamma are redone in mode 2).
        unsigned runbits = 0u;
        float gamma2 = a.ctrl->gamma2;
        if (spec) {
            runbits = __hip_atomic_load(&a.ctrlw->maxbits, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
            gamma2 = gamma2_rel(a.thr_mode, a.thr, __uint_as_float(runbits)) * 0.999999f;
        }
        float tmax = 0.f, tmin = __builtin_huge_valf();   // max |S|^2, least kept |S|^2
        const int64_t m0 = tile * FT;   // first frame of the tile, relative to frame0
        const int nvalid = (int)((a.nframes - m0) < FT ? (a.nframes - m0) : FT);
        const int64_t s0 = (a.frame0 + m0) * (int64_t)a.hop - a.M;
        __syncthreads();   // previous tile's store phase is done with the LDS

        // slab of samples in groups of 8, zero outside the signal; FP16 split:
        // scaled by 2^sx.  The sums of squares per group feed the scale bound.
        auto load8 = [&](int gi, float (&v)[8]) {
            const int64_t n = s0 + 8 * gi;
#pragma unroll
            for (int t = 0; t < 8; ++t)
                v[t] = (n + t >= 0 && n + t < a.n) ? a.x[n + t] : 0.f;
        };
        float sxs = 1.f, sxu = 1.f;
        if constexpr (SPLIT) {
            float vmax = 0.f;
            for (int gi = threadIdx.x; gi < ngrp; gi += NT) {
                float v[8];
                load8(gi, v);
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    vmax = fmaxf(vmax, fabsf(v[t]));
            }
            const float mx = block_max(vmax, red);
            int e = 0;
            frexpf(mx, &e);                       // mx < 2^e
            const int sx = mx > 0.f ? 14 - e : 0;   // mx 2^sx < 2^14
            sxs = ldexpf(1.f, sx);
            sxu = ldexpf(1.f, -sx);
        }
        for (int gi = threadIdx.x; gi < ngrp; gi += NT) {
            float v[8];
            load8(gi, v);
            float sq = 0.f;
            unsigned short hi[8], lo[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                sq += v[t] * v[t];
                split<PREC>(v[t] * sxs, hi[t], lo[t]);
            }
            gsq[gi] = sq;
            u4v ph, pl;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                ph[t] = (unsigned)hi[2 * t] | ((unsigned)hi[2 * t + 1] << 16);
                pl[t] = (unsigned)lo[2 * t] | ((unsigned)lo[2 * t + 1] << 16);
            }
            *reinterpret_cast<u4v *>(xhi + 8 * gi) = ph;
            if constexpr (SPLIT)
                *reinterpret_cast<u4v *>(xlo + 8 * gi) = pl;
        }
        if (!maxonly)
            for (int e = threadIdx.x; e < 2 * FT * a.n_dst; e += NT)
                hist[e] = 0;
        __syncthreads();

        // per-frame fixed-point scale: Parseval bound with sum_j x_j^2 g_j^2 <=
        // max g^2 times the sums of squares of the groups covering the window
        if (!maxonly) {
            constexpr int TPF = NT / FT;          // threads per frame
            const int f = threadIdx.x / TPF, part = threadIdx.x % TPF;
            const int g0 = f * (a.hop / 8), gn = (a.L + 7) / 8;
            float en = 0.f;
            for (int gi = part; gi < gn; gi += TPF)
                en += gsq[g0 + gi];
#pragma unroll
            for (int o = TPF / 2; o > 0; o >>= 1)
                en += __shfl_xor(en, o, 64);
            if (part == 0) {
                const float sc = fixed_scale(a.bound_c * sqrtf(a.gmax2 * en));
                scf[f] = sc;
                iscf[f] = 1.0f / sc;   // exact: a power of two
            }
        }
        __syncthreads();

        const float ug = a.unscale_g * sxu, ugd = a.unscale_gd * sxu;
        for (int rt = wave; rt < a.row_tiles; rt += 4) {
            f32x16 acc[CT];
#pragma unroll
            for (int c = 0; c < CT; ++c)
                acc[c] = f32x16{};
            const int64_t abase = (int64_t)rt * a.ksteps * 64 + lane;
            const u4v *ap = afrag + abase, *apl = afrag_lo + abase;
            const unsigned short *bp = xhi + col * a.hop + 8 * half;   // k = 0, column tile 0
            const int cstride = 32 * a.hop;                             // next column tile
            // The A fragments (from L2) are loaded AD steps ahead into a ring of
            // registers, so that later steps' loads are in flight while this
            // one's products run.  The main loop covers whole blocks of AD steps
            // without branches (a load past the last step takes the last
            // fragment again); the remaining steps use what the ring holds.
            constexpr int AD = 4;
            const int klast = a.ksteps - 1;
            u4v ring[AD], ringl[AD];
#pragma unroll
            for (int u = 0; u < AD; ++u) {
                ring[u] = ap[min(u, klast) * 64];
                ringl[u] = SPLIT ? apl[min(u, klast) * 64] : u4v{};
            }
            auto step = [&](int ks, u4v ac, u4v acl) {
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    const unsigned short *q = bp + c * cstride + ks * 16;
                    const u4v b = *reinterpret_cast<const u4v *>(q);
                    acc[c] = mma<PREC>(ac, b, acc[c]);
                    if constexpr (SPLIT) {
                        const u4v bl = *reinterpret_cast<const u4v *>(q + slab);
                        acc[c] = mma<PREC>(ac, bl, acc[c]);
                        acc[c] = mma<PREC>(acl, b, acc[c]);
                    }
                }
            };
            const int kmain = a.ksteps - a.ksteps % AD;
            for (int k0 = 0; k0 < kmain; k0 += AD) {
#pragma unroll
                for (int u = 0; u < AD; ++u) {
                    const u4v ac = ring[u], acl = ringl[u];
                    ring[u] = ap[min(k0 + u + AD, klast) * 64];
                    if constexpr (SPLIT)
                        ringl[u] = apl[min(k0 + u + AD, klast) * 64];
                    step(k0 + u, ac, acl);
                }
            }
#pragma unroll
            for (int u = 0; u < AD - 1; ++u)
                if (kmain + u < a.ksteps)
                    step(kmain + u, ring[u], ringl[u]);
            // epilogue: IF estimate, destination, histogram (Eqs. 12-13, 27-29)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int f = c * 32 + col;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int b = rt * 8 + 2 * q + half;
                    if (b >= a.n_src || f >= nvalid)
                        continue;
                    const float sr = acc[c][4 * q] * ug, si = acc[c][4 * q + 1] * ug;
                    const float dr = acc[c][4 * q + 2] * ugd, di = acc[c][4 * q + 3] * ugd;
                    const float mag2 = sr * sr + si * si;
                    tmax = fmaxf(tmax, mag2);
                    if (maxonly)
                        continue;
                    const int k = a.k1 + b;
                    int code = -1;
                    if (mag2 > gamma2) {
                        const float im = di * sr - dr * si;   // Im(S' conj S)
                        const float delta = a.cdelta * im / mag2;
                        const float zd = (float)a.z * delta;
                        const float hi = delta <= (float)k ? 0.5f - zd : zd + 0.5f;
                        const int ibase = delta <= (float)k ? a.z * (k - a.k1) : -a.z * (k + a.k1);
                        const int l = ibase + (int)floorf(fminf(fmaxf(hi, -1.0e8f), 1.0e8f));
                        code = (fabsf(zd) < 1.0e8f && l >= 0 && l < a.n_dst) ? l : -2;
                    }
                    if (code >= 0) {
                        tmin = fminf(tmin, mag2);
                        const float sc = scf[f];
                        int *h = hist + 2 * (f * a.n_dst + code);
                        atomicAdd(h, (int)rintf(sr * sc));
                        atomicAdd(h + 1, (int)rintf(si * sc));
                    }
                    if constexpr (DEBUG) {
                        const int64_t o = (m0 + f) * (int64_t)a.n_src + b;
                        if (a.S)
                            a.S[o] = make_float2(sr, si);
                        if (a.Sd)
                            a.Sd[o] = make_float2(dr, di);
                        if (a.idx)
                            a.idx[o] = code;
                    }
                }
            }
        }
        __syncthreads();
        if (maxonly || spec) {
            // the tile's maximum into the running one; its least kept |S|^2
            const float bm = block_max(tmax, red);
            const float bn = -block_max(-tmin, red);
            if (threadIdx.x == 0) {
                if (bm > __uint_as_float(runbits))
                    atomicMax(&a.ctrlw->maxbits, __float_as_uint(bm));
                if (spec)
                    a.smin[tile] = bn;
            }
        }
        if (maxonly)
            continue;

        // store phase: the tile's rows of T are contiguous; a buffer resource
        // bounded to the valid rows drops the rest
        const int cnt = nvalid * a.n_dst;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            a.T + m0 * a.n_dst, (short)0, cnt * 8, kBufferWord3);
        const float inv_ndst = 1.0f / (float)a.n_dst;
        for (int e = threadIdx.x; e < FT * a.n_dst; e += NT) {
            int f = (int)(((float)e + 0.5f) * inv_ndst);
            f = f < FT ? f : FT - 1;
            const float isc = iscf[f];
            const f2v v = {(float)hist[2 * e] * isc, (float)hist[2 * e + 1] * isc};
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, v), rs, (unsigned)e * 8u,
                                                  0, kNonTemporal);
        }
    }
}

template <int PREC, int FT>
hipError_t launch_prec_ft(bool debug, const GemmArgs &a, int grid, hipStream_t s)
{
    const size_t lds = gemm_lds_bytes(PREC, FT, a.n_dst, a.slab, a.L);
    if (debug)
        hipLaunchKernelGGL((gemm_kernel<PREC, FT, true>), dim3(grid), dim3(NT), lds, s, a);
    else
        hipLaunchKernelGGL((gemm_kernel<PREC, FT, false>), dim3(grid), dim3(NT), lds, s, a);
    return hipGetLastError();
}

template <int PREC, int FT>
int occ_prec_ft(size_t lds)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_kernel<PREC, FT, false>, NT, lds) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

}  // namespace

size_t gemm_lds_bytes(int prec, int ft, int n_dst, int slab, int L)
{
    const size_t xs = (size_t)slab * 2 * (prec == SST_GEMM_F16X3 ? 2 : 1);
    const size_t ngrp = (size_t)(slab / 8);
    (void)L;
    return (size_t)ft * n_dst * 8 + xs + 4 * ((ngrp + 3) & ~(size_t)3) + 8 * (size_t)ft + 16;
}

hipError_t launch_gemm_forward(int prec, int ft, bool debug, const GemmArgs &a, int grid,
                               hipStream_t s)
{
    if (prec == SST_GEMM_BF16)
        return ft == 64 ? launch_prec_ft<SST_GEMM_BF16, 64>(debug, a, grid, s)
                        : launch_prec_ft<SST_GEMM_BF16, 32>(debug, a, grid, s);
    return ft == 64 ? launch_prec_ft<SST_GEMM_F16X3, 64>(debug, a, grid, s)
                    : launch_prec_ft<SST_GEMM_F16X3, 32>(debug, a, grid, s);
}

int gemm_occupancy(int prec, int ft, size_t lds)
{
    if (prec == SST_GEMM_BF16)
        return ft == 64 ? occ_prec_ft<SST_GEMM_BF16, 64>(lds) : occ_prec_ft<SST_GEMM_BF16, 32>(lds);
    return ft == 64 ? occ_prec_ft<SST_GEMM_F16X3, 64>(lds) : occ_prec_ft<SST_GEMM_F16X3, 32>(lds);
}

}  // namespace sst
