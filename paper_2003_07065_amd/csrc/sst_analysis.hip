// gfx950 kernels of the analysis measures of the transform.
//
// Method: He & Cao, arXiv 2003.07065.
//   renyi_partial_kernel / renyi_final_kernel -- the Renyi entropy of a
//       time-frequency representation (Sec. 3, Eq. 32) with P = |C|^2, the
//       paper's measure of TF concentration: R = 1/(1 - alpha) log2 of the sum
//       over the grid of (P / sum P)^alpha, in the discrete form (no cell-area
//       term).  Two float64 sums, sum P and sum P^alpha, are reduced in a fixed
//       order (per-workgroup partials, then one workgroup), so the result does
//       not depend on scheduling.  Bound: HBM, one read of C.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sst_internal.h"

namespace sst {
namespace {

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// P of element (r, c) of the input, as float.
template <int KIND>
__device__ __forceinline__ float energy_at(const void *C, int64_t r, int64_t ld, int c)
{
    const int64_t i = r * ld + c;
    if constexpr (KIND == 0) {
        const float2 v = reinterpret_cast<const float2 *>(C)[i];
        return __builtin_fmaf(v.x, v.x, v.y * v.y);
    } else if constexpr (KIND == 1) {
        const float a = reinterpret_cast<const float *>(C)[i];
        return a * a;
    } else {
        const float a = (float)reinterpret_cast<const _Float16 *>(C)[i];
        return a * a;
    }
}

__device__ __forceinline__ double ipow(double p, int alpha)
{
    double r = p;
    for (int k = 1; k < alpha; ++k)
        r *= p;
    return r;
}

// Workgroup b sums rows [b rows_per, (b + 1) rows_per) into work[2b], work[2b + 1].
template <int KIND>
__global__ __launch_bounds__(256) void renyi_partial_kernel(RenyiArgs a)
{
    __shared__ double red[2][4];
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per;
    int64_t r1 = r0 + a.rows_per;
    if (r1 > a.rows)
        r1 = a.rows;
    double s1 = 0.0, sa = 0.0;
    for (int64_t r = r0; r < r1; ++r)
        for (int c = threadIdx.x; c < a.cols; c += 256) {
            const double p = (double)energy_at<KIND>(a.C, r, a.ld, c);
            s1 += p;
            sa += ipow(p, a.alpha);
        }
    s1 = wave_sum_f64(s1);
    sa = wave_sum_f64(sa);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = s1;
        red[1][w] = sa;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.work[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        a.work[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

// One workgroup: the partials in a fixed tree order, then R.
__global__ __launch_bounds__(1024) void renyi_final_kernel(RenyiArgs a, int nparts)
{
    __shared__ double s[2][1024];
    const int t = threadIdx.x;
    s[0][t] = t < nparts ? a.work[2 * t] : 0.0;
    s[1][t] = t < nparts ? a.work[2 * t + 1] : 0.0;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (t < h) {
            s[0][t] += s[0][t + h];
            s[1][t] += s[1][t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double s1 = s[0][0], sa = s[1][0];
        a.out[0] = s1;
        a.out[1] = sa;
        // sum (P / s1)^alpha = sa / s1^alpha
        a.out[2] = (s1 > 0.0 && sa > 0.0)
                       ? (log2(sa) - (double)a.alpha * log2(s1)) / (1.0 - (double)a.alpha)
                       : __builtin_nan("");
    }
}

}  // namespace

hipError_t launch_renyi(const RenyiArgs &a0, int kind, hipStream_t s)
{
    RenyiArgs a = a0;
    const int64_t parts = a.rows < kRenyiParts ? a.rows : kRenyiParts;
    a.rows_per = (a.rows + parts - 1) / parts;
    const int nparts = (int)((a.rows + a.rows_per - 1) / a.rows_per);
    if (nparts > 0) {
        if (kind == 0)
            hipLaunchKernelGGL(renyi_partial_kernel<0>, dim3(nparts), dim3(256), 0, s, a);
        else if (kind == 1)
            hipLaunchKernelGGL(renyi_partial_kernel<1>, dim3(nparts), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL(renyi_partial_kernel<2>, dim3(nparts), dim3(256), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(renyi_final_kernel, dim3(1), dim3(1024), 0, s, a, nparts);
    return hipGetLastError();
}

}  // namespace sst
