// gfx950 kernels of the downsampled synchrosqueezing transform.
//
// Method: He & Cao, arXiv 2003.07065.
//   fwd_kernel   -- framing with g and g' (Sec. 2.1, Eqs. 7-8), the N_f-point
//                   FFT pair with centre phase (Eq. 9), the IF estimate and the
//                   threshold (Sec. 2.2, Eqs. 12-13), and the selective,
//                   subdivided reassignment (Eq. 14; Sec. 2.4, Eqs. 27-29)
//                   into an LDS histogram that is streamed to HBM as rows of T.
//                   Modes: the plain forward (optionally at a speculative lower
//                   bound of the relative threshold), the max-only pre-pass
//                   for that threshold, and the fix-up pass over a list of
//                   frame groups.
//   spec_list_kernel -- gamma after a speculative forward and the list of
//                   frame groups that the final gamma changes.
//   inv_kernel   -- the direct downsampled inverse (Sec. 2.3, Eqs. 25-26, zN_f
//                   phase grid of the band / subdivision remark of Sec. 2.5),
//                   its window contraction on the FP16 matrix cores with
//                   hi/lo split operands.
//   eq15_kernel  -- the standard hop-1 inverse (Sec. 2.2, Eq. 15).
//   ridge_kernel -- per-frame argmax of |T| inside a band (zone M_q[m]).
//
// FFT layout.  A workgroup transforms V = max(N_f, 4096) complex points per
// iteration: F = V / N_f frames of N_f points, NT = V / 16 threads.  Stockham
// autosort passes of radix 16 (the last pass radix N_f / 256 or 16, plus a
// radix-2 pass at N_f = 8192) run in place in LDS with two barriers per pass.
// Every thread owns one radix-16 butterfly (or 16/R radix-R butterflies) per
// pass.  The LDS index a is padded to a + a/16 so that the stride-16 writes of
// the first pass and the contiguous reads of later passes are free of bank
// conflicts.  Pass 1 reads the signal straight from HBM (coalesced: adjacent
// lanes read adjacent samples) and skips the zero padding of Eq. 9: when the
// window is at most N_f/4 (or N_f/2) long, only 4 (or 8) of each butterfly's 16
// inputs can be non-zero and a pruned radix-16 is used.
//
// Packed pair.  g x and s g' x are transformed together as one complex signal
// y = g x + i s g' x, s = ||g|| / ||g'||, which keeps both halves at the same
// scale so that neither loses precision in the shared FFT.  With Y = FFT(y):
//   A[k] = (Y[k] + conj Y[N-k]) / 2 = FFT(g x)[k],
//   B[k] = (Y[k] - conj Y[N-k]) / 2i = s FFT(g' x)[k].
// The centre phase of Eq. 9 multiplies A and B alike, so it cancels in
// Im(S' conj S) and is applied only to the values written out.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "sst_internal.h"

namespace sst {
namespace {

typedef float v2 __attribute__((ext_vector_type(2)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));

// Word 3 of a raw (untyped, stride 0) buffer resource on the gfx9 family:
// 32-bit data format, everything else zero.
constexpr int kBufferWord3 = 0x00020000;
// Cache policy of the T stream-out: non-temporal.
constexpr int kNonTemporal = 2;

__device__ __forceinline__ v2 mk(float a, float b)
{
    v2 r;
    r.x = a;
    r.y = b;
    return r;
}
__device__ __forceinline__ v2 cmul(v2 a, v2 b)
{
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ v2 mul_mi(v2 a) { return mk(a.y, -a.x); }   // -i a
__device__ __forceinline__ v2 conjv(v2 a) { return mk(a.x, -a.y); }
__device__ __forceinline__ int pad16(int a) { return a + (a >> 4); }
// pad16(a + 16 u) = pad16(a) + 17 u for a >= 0: strided accesses take one padded
// base and constant offsets, which the LDS instructions encode as immediates.
constexpr int padded_stride(int s) { return s + s / 16; }

// ---------------------------------------------------------------------------
// Register DFTs (forward, exp(-i ...)), natural order in and out.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void bf4(v2 &a0, v2 &a1, v2 &a2, v2 &a3)
{
    v2 t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = a1 - a3;
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + mul_mi(t3);
    a3 = t1 - mul_mi(t3);
}

constexpr float kC1 = 0.92387953251128674f;  // cos(pi/8)
constexpr float kS1 = 0.38268343236508978f;  // sin(pi/8)
constexpr float kR2 = 0.70710678118654752f;  // sqrt(1/2)

// Inner twiddles of the 4 x 4 radix-16: a[n2 + 4 k1] *= W16^(n2 k1).
__device__ __forceinline__ void tw16(v2 *a)
{
    a[5] = cmul(a[5], mk(kC1, -kS1));    // W^1
    a[9] = cmul(a[9], mk(kR2, -kR2));    // W^2
    a[13] = cmul(a[13], mk(kS1, -kC1));  // W^3
    a[6] = cmul(a[6], mk(kR2, -kR2));    // W^2
    a[10] = mul_mi(a[10]);               // W^4
    a[14] = cmul(a[14], mk(-kR2, -kR2)); // W^6
    a[7] = cmul(a[7], mk(kS1, -kC1));    // W^3
    a[11] = cmul(a[11], mk(-kR2, -kR2)); // W^6
    a[15] = cmul(a[15], mk(-kC1, kS1));  // W^9
}

// Outer radix-4 over n2 for every k1, then the transposition to natural order.
__device__ __forceinline__ void outer16(v2 *a)
{
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
        bf4(a[4 * k1], a[4 * k1 + 1], a[4 * k1 + 2], a[4 * k1 + 3]);
    v2 b[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2)
            b[k1 + 4 * k2] = a[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        a[i] = b[i];
}

// Full radix-16: n = 4 n1 + n2, k = k1 + 4 k2.
__device__ __forceinline__ void dft16(v2 *a)
{
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2)
        bf4(a[n2], a[n2 + 4], a[n2 + 8], a[n2 + 12]);
    tw16(a);
    outer16(a);
}

// Radix-16 whose inputs 4..15 are zero (n1 = 0 only).
__device__ __forceinline__ void dft16_nz4(v2 *a)
{
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        a[n2 + 4] = a[n2];
        a[n2 + 8] = a[n2];
        a[n2 + 12] = a[n2];
    }
    tw16(a);
    outer16(a);
}

// Radix-16 whose inputs 8..15 are zero (n1 in {0, 1}).
__device__ __forceinline__ void dft16_nz8(v2 *a)
{
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        v2 p = a[n2], q = a[n2 + 4];
        a[n2] = p + q;
        a[n2 + 4] = p + mul_mi(q);
        a[n2 + 8] = p - q;
        a[n2 + 12] = p - mul_mi(q);
    }
    tw16(a);
    outer16(a);
}

__device__ __forceinline__ void dft8(v2 *a)
{
    v2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    v2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    bf4(e0, e1, e2, e3);
    bf4(o0, o1, o2, o3);
    o1 = mk(kR2 * (o1.x + o1.y), kR2 * (o1.y - o1.x));    // * W8^1
    o2 = mul_mi(o2);                                      // * W8^2
    o3 = mk(kR2 * (o3.y - o3.x), -kR2 * (o3.x + o3.y));   // * W8^3
    a[0] = e0 + o0;
    a[4] = e0 - o0;
    a[1] = e1 + o1;
    a[5] = e1 - o1;
    a[2] = e2 + o2;
    a[6] = e2 - o2;
    a[3] = e3 + o3;
    a[7] = e3 - o3;
}

template <int R>
__device__ __forceinline__ void dftR(v2 *a);
template <>
__device__ __forceinline__ void dftR<2>(v2 *a)
{
    v2 t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
}
template <>
__device__ __forceinline__ void dftR<4>(v2 *a) { bf4(a[0], a[1], a[2], a[3]); }
template <>
__device__ __forceinline__ void dftR<8>(v2 *a) { dft8(a); }
template <>
__device__ __forceinline__ void dftR<16>(v2 *a) { dft16(a); }

// Pointer to memory the kernels only read and index uniformly (descriptors,
// control blocks): loads through it use the scalar unit.
#define CA __attribute__((address_space(4)))

// ---------------------------------------------------------------------------
// Geometry per DFT size.
// ---------------------------------------------------------------------------

template <int NF>
struct Geo {
    static constexpr int V = NF > 4096 ? NF : 4096;   // points per iteration
    static constexpr int F = V / NF;                  // frames per iteration
    static constexpr int NT = V / 16;                 // threads per workgroup
    static constexpr int LDS = V + V / 16;            // padded float2 capacity
    static constexpr int R3 = NF >= 4096 ? 16 : NF / 256;  // radix of pass 3
    static constexpr bool P4 = NF == 8192;            // radix-2 pass 4
};

template <int R>
constexpr int log2i() { return R <= 1 ? 0 : 1 + log2i<R / 2>(); }

// A compile-time integer passed as a value (selects a specialised lambda body).
template <int V>
struct IntC {
    static constexpr int value = V;
};

// One Stockham pass of radix R and stride NS over the F frames in LDS.  Every
// butterfly of a thread has the same twiddle index k = (j mod N_f/R) mod NS =
// tid mod NS (NS divides both N_f/R and the thread count), so the caller
// supplies the thread's R twiddles W_{NS R}^{k r}, r = 0 .. R-1 (w[0] = 1),
// each the correctly rounded value of a float64 table entry.
template <int NF, int R, int NS>
struct Pass {
    using G = Geo<NF>;
    static constexpr int NR = NF / R;
    static constexpr int NB = (NF * G::F / R) / G::NT;   // butterflies per thread
    static_assert(NS == 1 || (G::NT % NS == 0 && NR % NS == 0), "one twiddle set per thread");

    static __device__ __forceinline__ void run(v2 *lds, const v2 (&w)[R])
    {
        // LDS addresses depend only on the thread index; an opaque copy per
        // call keeps them from being hoisted out of the frame loop and spilled
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        v2 v[NB][R];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = tid + b * G::NT;
            const int f = j / NR, jj = j % NR;
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[b][r] = lds[pad16(f * NF + jj) + r * padded_stride(NR)];
        }
        if constexpr (NS > 1) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 1; r < R; ++r)
                    v[b][r] = cmul(v[b][r], w[r]);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b)
            dftR<R>(v[b]);
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = tid + b * G::NT;
            const int f = j / NR, jj = j % NR;
            const int k = jj % NS;
            const int base_i = f * NF + (jj / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r)
                lds[pad16(base_i) + r * padded_stride(NS)] = v[b][r];
        }
        __syncthreads();
    }
};

// Twiddles of the passes after the first, every one read from the float64-
// built table W_{N_f}^t (correctly rounded), none formed by products:
//   pass 2 (radix 16, stride 16): W_256^{k r} = W_{N_f}^{(N_f/256) k r}, k < 16,
//     staged once in LDS as tbl[(r - 1) 16 + k] (TW entries; a wave's lanes
//     read 16 distinct words, broadcast to the others);
//   pass 3 (radix R3, stride 256): W_{256 R3}^{k r}, k = tid mod 256, held in
//     registers for the life of the workgroup;
//   pass 4 (radix 2, N_f = 8192 only): W_8192^j for the thread's butterflies,
//     read from the table (L1/L2) at the start of the pass.
template <int NF>
struct Twiddles {
    using G = Geo<NF>;
    using P2 = Pass<NF, 16, 16>;
    using P3 = Pass<NF, G::R3, 256>;
    static constexpr int TW = 15 * 16;
    static constexpr int NB4 = G::P4 ? (NF / 2) / G::NT : 1;   // pass-4 butterflies per thread
    v2 t3[G::R3];
    const v2 *tw4;   // the table, for pass 4

    // Stage the pass-2 table into tbl (visible after the next barrier) and
    // load the pass-3 and pass-4 twiddles.
    __device__ __forceinline__ void load(v2 *tbl, const v2 *__restrict__ twid)
    {
        for (int e = threadIdx.x; e < TW; e += G::NT) {
            const int r = e / 16 + 1, k = e % 16;
            tbl[e] = twid[(unsigned)((NF / 256) * k * r)];
        }
        const int k3 = threadIdx.x % 256;
        t3[0] = mk(1.f, 0.f);
#pragma unroll
        for (int r = 1; r < G::R3; ++r)
            t3[r] = twid[(unsigned)((NF / (256 * G::R3)) * k3 * r)];
        tw4 = twid;
    }
    // LAST = false leaves out the radix-2 pass 4 (N_f = 8192): its outputs
    // are then formed where they are read (out4)
    template <bool LAST = true>
    __device__ __forceinline__ void passes(v2 *lds, const v2 *tbl) const
    {
        v2 w2[16];
        w2[0] = mk(1.f, 0.f);
        const int k2 = threadIdx.x % 16;
#pragma unroll
        for (int r = 1; r < 16; ++r)
            w2[r] = tbl[(r - 1) * 16 + k2];
        P2::run(lds, w2);
        P3::run(lds, t3);
        if constexpr (G::P4 && LAST)
            pass4(lds);
    }
    // Output k of pass 4 from its inputs (pass 4 left out): butterfly
    // j = k mod 4096 of elements u = j and v = j + 4096 gives u + W v at j and
    // u - W v at j + 4096, W = W_8192^j (wj), the products of pass4 itself.
    __device__ __forceinline__ v2 out4(const v2 *lds, int k, v2 wj) const
    {
        const int j = k & (NF / 2 - 1);
        const v2 u = lds[pad16(j)];
        const v2 t = cmul(lds[pad16(j) + padded_stride(NF / 2)], wj);
        return (k & (NF / 2)) ? u - t : u + t;
    }
    __device__ __forceinline__ v2 w4_of(int j) const { return tw4[(unsigned)j]; }
    // Radix-2 pass of stride 4096 (N_f = 8192, one frame): butterfly j pairs
    // elements j and j + 4096 with twiddle W_8192^j.
    __device__ __forceinline__ void pass4(v2 *lds) const
    {
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        v2 t4[NB4];
#pragma unroll
        for (int b = 0; b < NB4; ++b)
            t4[b] = tw4[(unsigned)(tid + b * G::NT)];
        v2 v[NB4][2];
#pragma unroll
        for (int b = 0; b < NB4; ++b) {
            const int j = tid + b * G::NT;
            v[b][0] = lds[pad16(j)];
            v[b][1] = cmul(lds[pad16(j) + padded_stride(4096)], t4[b]);
            const v2 u = v[b][0];
            v[b][0] = u + v[b][1];
            v[b][1] = u - v[b][1];
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB4; ++b) {
            const int j = tid + b * G::NT;
            lds[pad16(j)] = v[b][0];
            lds[pad16(j) + padded_stride(4096)] = v[b][1];
        }
        __syncthreads();
    }
};

// Pass 1 (radix 16, stride 1): each thread's 16 inputs come from HBM through
// `load(f, n)`; the outputs go to LDS.  Only the first NZ of the 16 inputs can
// be non-zero (NZ = 4, 8 or 16 covers ceil(L / (N_f/16)) rows of taps).
template <int NF, int NZ, typename Loader>
__device__ __forceinline__ void pass1(v2 *lds, const Loader &load)
{
    constexpr int Q = NF / 16;
    const int f = threadIdx.x / Q, jj = threadIdx.x % Q;
    v2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r)
        v[r] = (r < NZ) ? load(f, jj + r * Q) : mk(0.f, 0.f);
    if constexpr (NZ == 4)
        dft16_nz4(v);
    else if constexpr (NZ == 8)
        dft16_nz8(v);
    else
        dft16(v);
    const int base = f * NF + jj * 16;
#pragma unroll
    for (int r = 0; r < 16; ++r)
        lds[pad16(base) + r] = v[r];   // base: a multiple of 16
    __syncthreads();
}

// Flat coefficient e of an iteration -> (frame f, in-band offset ik).
__device__ __forceinline__ void split_flat(int e, int n_src, float inv_nsrc, int &f, int &ik)
{
    int q = (int)(((float)e + 0.5f) * inv_nsrc);
    if (q * n_src > e)
        --q;
    else if ((q + 1) * n_src <= e)
        ++q;
    f = q;
    ik = e - q * n_src;
}

// ---------------------------------------------------------------------------
// Forward kernel: framing, FFT pair, IF, threshold, reassignment, T rows.
//
// Phases of one iteration (F frames):
//   pass 1 .. pass s  Stockham FFT of the packed pair in the LDS buffer;
//   IF phase          every thread evaluates its in-band coefficients
//                     (Eqs. 12-13, 27-29) and keeps (destination, S) in
//                     registers; per-frame sums sum_k (|Re S| + |Im S|) are
//                     reduced per wave, then summed in a fixed order;
//   scatter phase     the LDS buffer, no longer needed by the FFT, becomes
//                     the destination histogram: zeroed, then every kept
//                     coefficient is added to its bin;
//   store phase       each bin is read, converted and streamed to HBM as T.
// Reusing the FFT buffer for the histogram halves the LDS of a workgroup and
// raises the number of resident workgroups per CU.  Rows longer than the
// buffer (F n_dst > HBINS) are scattered and stored in several chunks.
//
// Histogram arithmetic.  The sums of Eq. 28 are accumulated as 32-bit
// fixed-point integers with a per-frame power-of-two scale 2^K chosen from
// B = sum_k (|Re S| + |Im S|) over the frame's kept coefficients, which bounds
// the real and the imaginary sum of every bin: B 2^K < 2^31, so no bin
// overflows.  Each term is rounded to an integer (error <= 2^-(K+1), about
// 2^-32 B) and the integer sums are exact, hence independent of the order of
// the atomics; each bin is rounded to FP32 once when it is written.  (LDS
// floating-point atomics are an order of magnitude slower than integer ones
// on this GPU.)
//
// Pipelining.  On gfx9 one counter tracks outstanding vector-memory loads and
// stores together, so a load issued after an iteration's T stores would wait
// for those stores to drain.  Each thread therefore fetches its pass-1 samples
// of the NEXT iteration right after pass 1, before this iteration's stores,
// and every store instruction is unconditional (a buffer resource bounded to
// the valid bins drops the excess), so the wait for the prefetched samples
// covers only the loads.
//
// R bounds the in-band coefficients per thread (ceil(F n_src / NT) <= R).
// CHUNKED allows rows longer than the buffer; without it the row is a single
// chunk whose store count is known at compile time.  DEBUG adds the
// per-coefficient outputs (S, S', destination index) and the FP64 column sums.
// ---------------------------------------------------------------------------

// Power-of-two scale 2^K with B 2^K < 2^31 (B >= 0), clamped to [2^-100, 2^100].
__device__ __forceinline__ float fixed_scale(float B)
{
    int e = 0;
    frexpf(B, &e);   // B < 2^e
    int K = B > 0.f ? 31 - e : 0;
    K = K > 100 ? 100 : (K < -100 ? -100 : K);
    return ldexpf(1.0f, K);
}

// Channel of item `it` for a launch whose items ascend with the channel
// index: advance c while `it` lies past channel c's items (end[] cumulative).
template <bool THRESHOLD>
__device__ __forceinline__ int chan_of(const CA ChanDesc *ch, int n_ch, int c, int64_t it)
{
    while (c < n_ch - 1 && it >= (THRESHOLD ? ch[c].mitem_end : ch[c].item_end))
        ++c;
    return c;
}

// Per-channel values a workgroup keeps in scalar registers while it works
// on that channel's items; reloaded only when the channel changes.
__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide max of v, then one atomicMax of its float bits into *dst
// (non-negative floats order like their bit patterns).  Every thread calls it.
template <int NT>
__device__ __forceinline__ void block_max_flush(float v, float *red, unsigned *dst)
{
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float b = red[0];
        for (int w = 1; w < NT / 64; ++w)
            b = fmaxf(b, red[w]);
        atomicMax(dst, __float_as_uint(b));
    }
    __syncthreads();
}

// Wave reductions on the data-parallel primitives (no LDS round trips): xor
// 1 and xor 2 within quads, rotations by 4 and 8 within rows of 16 lanes,
// then row 0 -> 1 and row 2 -> 3 and lane 31 -> rows 2, 3.  The reduction
// of all 64 lanes is left in lane 63.  `id` is the identity of `op`.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_mov(float old, float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v),
                                                      CTRL, ROWS, 0xf, false));
}

template <class Op>
__device__ __forceinline__ float wave_reduce63(float v, float id, Op op)
{
    v = op(v, dpp_mov<0xb1>(id, v));         // quad_perm [1, 0, 3, 2]
    v = op(v, dpp_mov<0x4e>(id, v));         // quad_perm [2, 3, 0, 1]
    v = op(v, dpp_mov<0x124>(id, v));        // row_ror 4
    v = op(v, dpp_mov<0x128>(id, v));        // row_ror 8
    v = op(v, dpp_mov<0x142, 0xa>(id, v));   // row_bcast 15 into rows 1, 3
    v = op(v, dpp_mov<0x143, 0xc>(id, v));   // row_bcast 31 into rows 2, 3
    return v;
}

// |A|^2 as every threshold decision of the FFT path computes it (one
// rounding order, so the pre-pass maximum and the forward agree bit for bit).
__device__ __forceinline__ float mag2_of(v2 A)
{
    return __builtin_fmaf(A.x, A.x, A.y * A.y);
}

// gamma^2 from max |S|^2: rho^2 max (relative) or the given gamma (absolute).
__device__ __forceinline__ float gamma2_of(int thr_mode, float thr, float max2)
{
    const float gm = thr_mode == 1 ? thr * sqrtf(max2) : thr;
    return gm * gm;
}

struct Chan {
    const float *x;
    const float2 *win;
    float2 *T;
    float2 *S;
    float2 *Sd;
    int32_t *idx;
    double *colstats;
    Ctrl *ctrl;
    int64_t n, n_frames, frame0, nframes, item0, item_end;
    int L, M, hop, k1, n_src, n_dst, z, thr_mode, out_fmt;
    float gamma2, thr, inv_s, cdelta, inv_nsrc, inv_ndst;
};

template <bool THRESHOLD>
__device__ __forceinline__ Chan load_chan(const CA ChanDesc *ch, int c)
{
    const CA ChanDesc &d = ch[c];
    Chan r;
    r.x = d.x;
    r.win = d.win;
    r.T = d.T;
    r.S = d.S;
    r.Sd = d.Sd;
    r.idx = d.idx;
    r.colstats = d.colstats;
    r.ctrl = d.ctrl;
    r.n = d.n;
    r.n_frames = d.n_frames;
    // threshold passes cover every frame of the signal
    r.frame0 = THRESHOLD ? 0 : d.frame0;
    r.nframes = THRESHOLD ? d.n_frames : d.nframes;
    r.item0 = THRESHOLD ? d.mitem0 : d.item0;
    r.item_end = THRESHOLD ? d.mitem_end : d.item_end;
    r.L = d.L;
    r.M = d.M;
    r.hop = d.hop;
    r.k1 = d.k1;
    r.n_src = d.n_src;
    r.n_dst = d.n_dst;
    r.z = d.z;
    r.thr_mode = d.thr_mode;
    r.out_fmt = d.out_fmt;
    r.thr = d.thr;
    r.gamma2 = THRESHOLD ? 0.f : ((const CA Ctrl *)d.ctrl)->gamma2;
    r.inv_s = d.inv_s;
    r.cdelta = d.cdelta;
    r.inv_nsrc = 1.0f / (float)d.n_src;
    r.inv_ndst = 1.0f / (float)d.n_dst;
    return r;
}

// exp(+i 2 pi t / N_f) for 0 <= t < N_f from two LDS copies of the twiddle
// table (lo[r] = W^r, r < 64; hi[h] = W^(64 h)): the conjugate of
// W^t = hi[t / 64] lo[t mod 64].
__device__ __forceinline__ v2 cphase_of(const v2 *lo, const v2 *hi, int t)
{
    return conjv(cmul(hi[t >> 6], lo[t & 63]));
}

// Modes of the forward kernel.
constexpr int kFwdPlain = 0;     // the forward over items item_begin, item_begin + 1, ...
constexpr int kFwdMaxOnly = 1;   // threshold pre-pass on the forward's arithmetic
constexpr int kFwdFixup = 2;     // the forward over the items of a fix-up list
constexpr int kFwdStft = 3;      // the STFT product only: S (and S') rows of the items

template <int NF, int NZ, int R, bool DEBUG, bool CHUNKED, bool MULTI, int MODE = kFwdPlain,
          bool STATS = false>
// Waves per SIMD: 4 for N_f = 8192 and for N_f = 4096 with at most 8 tap rows
// (two 8-wave or four 4-wave workgroups fill a CU's LDS), 3 otherwise.  MULTI: the launch may hold several channels (else
// exactly one).  STATS (and DEBUG): the per-frame FP64 sums of the stored rows
// (colstats) as an epilogue of the store phase.
__global__ __launch_bounds__(Geo<NF>::NT, DEBUG ? 2 : ((NF == 8192 || (NF == 4096 && NZ < 16)) ? 4 : 3)) void fwd_kernel(GroupLaunch g)
{
    // kFwdMaxOnly: the threshold pre-pass on the forward's own arithmetic --
    // pass 1 and the FFT passes, then max |A|^2 over the band, folded into
    // maxbits of each channel; items are numbered by mitem0 over the whole
    // signal.  kFwdFixup: the items of g.list only.
    constexpr bool MAXONLY = MODE == kFwdMaxOnly;
    constexpr bool listed = MODE == kFwdFixup;
    constexpr bool COLS = DEBUG || STATS;   // the colstats epilogue is compiled in
    if (listed && (int64_t)blockIdx.x >= (int64_t)*g.list_n)
        return;   // no entry for this workgroup (the usual case: an empty list)
    using G = Geo<NF>;
    constexpr int F = G::F, NT = G::NT, Q = NF / 16;
    constexpr int HB = G::LDS;        // histogram bins (two 32-bit integers each)
    constexpr int NST = HB / NT;      // store instructions per thread and chunk
    static_assert(HB % NT == 0, "histogram is a whole number of store rounds");
    constexpr int SEGF = 24;          // key = (frame << SEGF) | flat destination
    constexpr int NHI = NF / 64;
    __shared__ v2 lds[G::LDS];
    __shared__ float bpart[NT / 64][F];   // per-wave partial bounds, summed in fixed order
    __shared__ float spart[NT / 64][2];   // per-wave max |S|^2 and least kept |S|^2
    __shared__ double colacc[COLS ? 3 * F : 1];   // per-frame FP64 sums (colstats)
    __shared__ v2 twl[Twiddles<NF>::TW];
    __shared__ v2 clo[64], chi[NHI];   // centre-phase tables (Eq. 9)
    int *hq = reinterpret_cast<int *>(lds);   // bin b: hq[2b] = re, hq[2b + 1] = im

    const v2 *__restrict__ twid = reinterpret_cast<const v2 *>(g.twid);
    Twiddles<NF> tw;
    tw.load(twl, twid);
    for (int e = threadIdx.x; e < 64 + NHI; e += NT) {
        if (e < 64)
            clo[e] = twid[(unsigned)e];
        else
            chi[e - 64] = twid[(unsigned)(e - 64) * 64u];
    }
    // N_f = 8192: the radix-2 pass 4 is left out and only the outputs that are
    // read are formed (the in-band bins and their mirrors: 3202 of 8192 on a
    // band of 0 .. N_f / 5), each from its two inputs.
    constexpr bool FUSE4 = G::P4;
    static_assert(!FUSE4 || F == 1, "pass 4 is left out with one frame per item");
    // Y[k] and conj(Y[N_f - k]) of frame f after the FFT passes.  Left-out
    // pass 4: the mirror's butterfly is 4096 - (k mod 4096), whose twiddle is
    // -conj(W_8192^(k mod 4096)) exactly; bins 0 and 4096 are their own mirrors.
    auto ypair = [&](int f, int k, v2 &P, v2 &Qc) {
        if constexpr (FUSE4) {
            const int j = k & (NF / 2 - 1);
            const v2 wj = tw.w4_of(j);
            P = tw.out4(lds, k, wj);
            Qc = conjv(j == 0 ? P : tw.out4(lds, NF - k, mk(-wj.x, wj.y)));
        } else {
            P = lds[pad16(f * NF + k)];
            Qc = conjv(lds[pad16(f * NF + ((NF - k) & (NF - 1)))]);
        }
    };
    const CA ChanDesc *ch = (const CA ChanDesc *)g.ch;

    // Pass-1 role of this thread: frame f1 of the iteration, taps jj + r Q.
    const int f1 = threadIdx.x / Q, jj = threadIdx.x % Q;
    v2 w[NZ];   // (g, s g') of the thread's taps; zero beyond the window
    // Eq. 8: frame m covers samples mH - M .. mH + M.  Signals are limited to
    // 2^30 samples so sample indices fit 32 bits.
    float xv[NZ];
    int okb = 0;
    // Samples of item `it` of channel d; the taps too when the channel changes
    // (w is free then: it is read only by pass 1, which precedes the fetch).
    auto fetch = [&](int64_t it, const Chan &d, bool new_chan) {
        const bool iv = it < g.item_stop;
        const int64_t m = (iv ? it - d.item0 : 0) * F + f1;   // frame relative to d.frame0
        const bool fv = iv & (m < d.nframes);
        const int cm = (int)((d.frame0 + (fv ? m : 0)) * (int64_t)d.hop - d.M) + jj;
        const float *__restrict__ x = d.x;
        const unsigned n = (unsigned)d.n;
        okb = 0;
#pragma unroll
        for (int r = 0; r < NZ; ++r) {
            const int s = cm + r * Q;
            const bool ok = fv & ((unsigned)s < n);
            xv[r] = x[ok ? (unsigned)s : 0u];
            okb |= (int)ok << r;
        }
        if (new_chan) {
            const v2 *__restrict__ win = reinterpret_cast<const v2 *>(d.win);
#pragma unroll
            for (int r = 0; r < NZ; ++r) {
                const int tap = jj + r * Q;
                w[r] = tap < d.L ? win[(unsigned)tap] : mk(0.f, 0.f);
            }
        }
    };

    if (COLS && threadIdx.x < 3 * F)
        colacc[threadIdx.x] = 0.0;
    // Items of this workgroup: every gridDim.x-th entry of the fix-up list, or
    // of item_begin, item_begin + step, ...; item_stop ends the sequence.
    const int64_t n_list = listed ? (int64_t)*g.list_n : 0;
    const int64_t st = g.step > 1 ? g.step : 1;
    auto item_at = [&](int64_t li) -> int64_t {
        if (listed)
            return li < n_list ? (int64_t)g.list[li] : g.item_stop;
        const int64_t v = g.item_begin + li * st;
        return v < g.item_stop ? v : g.item_stop;
    };
    int64_t li = blockIdx.x;
    int64_t it = item_at(li);
    int c = chan_of<MAXONLY>(ch, g.n_ch, 0, it);
    Chan a = load_chan<MAXONLY>(ch, c);
    fetch(it, a, true);
    float best = 0.f;   // MAXONLY: running max |A|^2 of the current channel
    // Wait here for every load issued so far (tables, first samples), so that
    // inside the loop the samples prefetched by the previous iteration are the
    // only loads the first use has to wait for (vmcnt(0), expcnt and lgkmcnt
    // left unconstrained).
    __builtin_amdgcn_s_waitcnt(0x0f70);

    // centre phase of bin k1 + tid and the rotation step (F == 1), per channel
    v2 ph0 = mk(1.f, 0.f), ph_step = mk(1.f, 0.f);
    bool new_chan = true;
    while (it < g.item_stop) {
        const int64_t m0 = (it - a.item0) * F;   // first frame of the item, relative to frame0
        const int nvalid = (int)((a.nframes - m0) < F ? (a.nframes - m0) : F);
        float gamma2 = a.gamma2;
        // Speculative threshold (relative gamma): max |S|^2 seen so far by any
        // workgroup is at most the final maximum, so the gamma it gives is a
        // lower bound and keeps a superset of the coefficients.
        unsigned runbits = 0u;
        if (MODE == kFwdPlain && g.spec && a.thr_mode == 1)
            runbits = __hip_atomic_load(&a.ctrl->maxbits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const float inv_nsrc = a.inv_nsrc;
        const float inv_ndst = a.inv_ndst;
        // the previous iteration's store phase is done with the buffer (and,
        // on the first iteration, the staged tables are complete)
        __syncthreads();
        if (F == 1 && !MAXONLY && new_chan) {
            ph0 = cphase_of(clo, chi, ((a.k1 + (int)threadIdx.x) * a.M) & (NF - 1));
            ph_step = cphase_of(clo, chi, (NT * a.M) & (NF - 1));
        }

        // Wave priorities: the FFT passes (below) wait at a barrier after every
        // LDS round trip; the IF, scatter and store phases that follow are long
        // runs without one.  With two or more workgroups resident per CU in
        // different phases, letting the barrier-free phases issue first (and
        // the FFT waves fill the gaps) keeps the SIMDs busier: 0 for the FFT,
        // 1 for the IF phase, 2 for scatter and store.
        __builtin_amdgcn_s_setprio(0);
        {   // pass 1 from the prefetched samples
            v2 v[16];
#pragma unroll
            for (int r = 0; r < 16; ++r)
                v[r] = (r < NZ) ? (((okb >> r) & 1) ? xv[r] : 0.f) * w[r] : mk(0.f, 0.f);
            if constexpr (NZ == 4)
                dft16_nz4(v);
            else if constexpr (NZ == 8)
                dft16_nz8(v);
            else
                dft16(v);
            const int base = f1 * NF + jj * 16;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                lds[pad16(base) + r] = v[r];   // base: a multiple of 16
        }
        // next iteration's samples, issued before this one's stores
        const int64_t itn = item_at(li + gridDim.x);
        Chan an = a;
        const bool chg = MULTI && itn < g.item_stop && (itn >= a.item_end || itn < a.item0);
        if (chg) {
            c = chan_of<MAXONLY>(ch, g.n_ch, itn < a.item0 ? 0 : c, itn);
            an = load_chan<MAXONLY>(ch, c);
        }
        fetch(itn, an, chg);
        __syncthreads();
        tw.template passes<!FUSE4>(lds, twl);
        __builtin_amdgcn_s_setprio(1);

        if constexpr (MODE == kFwdStft) {
            // STFT product (Eq. 9 with its centre phase; S' with g'): every
            // in-band bin of the item's frames, rows of n_src written in order
            const int EM = nvalid * a.n_src;
            v2 *__restrict__ Sp = reinterpret_cast<v2 *>(a.S) + m0 * (int64_t)a.n_src;
            v2 *__restrict__ Sdp =
                a.Sd ? reinterpret_cast<v2 *>(a.Sd) + m0 * (int64_t)a.n_src : nullptr;
            for (int e = threadIdx.x; e < EM; e += NT) {
                int f, ik;
                if constexpr (F == 1) {
                    f = 0;
                    ik = e;
                } else {
                    split_flat(e, a.n_src, inv_nsrc, f, ik);
                }
                const int k = a.k1 + ik;
                v2 P, Qc;
                ypair(f, k, P, Qc);
                const v2 phk = cphase_of(clo, chi, (k * a.M) & (NF - 1));
                __builtin_nontemporal_store(cmul(phk, 0.5f * (P + Qc)), Sp + e);
                if (Sdp) {
                    const v2 D = P - Qc;
                    const v2 B = mk(0.5f * D.y, -0.5f * D.x);
                    __builtin_nontemporal_store(a.inv_s * cmul(phk, B), Sdp + e);
                }
            }
            a = an;
            new_chan = chg;
            it = itn;
            li += gridDim.x;
            continue;
        }
        if constexpr (MAXONLY) {
            const int EM = nvalid * a.n_src;
            for (int e = threadIdx.x; e < EM; e += NT) {
                int f, ik;
                if constexpr (F == 1) {
                    f = 0;
                    ik = e;
                } else {
                    split_flat(e, a.n_src, inv_nsrc, f, ik);
                }
                const int k = a.k1 + ik;
                v2 P, Qc;
                ypair(f, k, P, Qc);
                best = fmaxf(best, mag2_of(0.5f * (P + Qc)));
            }
            if (chg || itn >= g.item_stop) {
                // leaving this channel: fold the workgroup's maximum into it
                block_max_flush<NT>(best, &spart[0][0], &a.ctrl->maxbits);
                best = 0.f;
            }
            a = an;
            new_chan = chg;
            it = itn;
            li += gridDim.x;
            continue;
        }
        const bool spec = MODE == kFwdPlain && g.spec;
        if (spec)
            gamma2 = gamma2_of(a.thr_mode, a.thr, __uint_as_float(runbits)) * 0.999999f;

        // IF phase: Eqs. 12-13 and 27-29 for every in-band coefficient of the
        // F frames; kept coefficients stay in registers as (key, S).
        const int E = nvalid * a.n_src;
        const int EH = nvalid * a.n_dst;
        // Per-round quantities (bins, LDS addresses) depend only on the thread
        // index; an opaque copy per iteration keeps the compiler from hoisting
        // them out of the frame loop and spilling them.
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        int key[R];
        v2 sv[R];
        float part[F];
        float mx = 0.f, mn = __builtin_huge_valf();   // max |S|^2, least kept |S|^2
#pragma unroll
        for (int f = 0; f < F; ++f)
            part[f] = 0.f;
        // Centre phase of Eq. 9, exp(i 2 pi ((k M) mod N_f) / N_f).  With one
        // frame per iteration a thread visits k = k1 + tid + i NT, whose phases
        // differ by the constant factor for (NT M) mod N_f, so they are
        // generated by rotation; otherwise each is looked up.
        v2 ph_cur = ph0;
        const int pk0 = pad16(a.k1 + tid);        // F == 1: bin of round 0
        const int qk0 = pad16(NF - a.k1 - tid);   // and its mirror
#pragma unroll
        for (int i = 0; i < R; ++i) {
            // rounds are independent; keeping the scheduler from interleaving
            // them bounds the live registers to one round's temporaries
            __builtin_amdgcn_sched_barrier(0);
            const int e = tid + i * NT;
            key[i] = -1;
            sv[i] = mk(0.f, 0.f);
            int f, ik;
            v2 phk;
            if constexpr (F == 1) {
                f = 0;
                ik = e;
                phk = ph_cur;
                ph_cur = cmul(ph_cur, ph_step);
            } else {
                split_flat(e < E ? e : 0, a.n_src, inv_nsrc, f, ik);
                phk = cphase_of(clo, chi, ((a.k1 + ik) * a.M) & (NF - 1));
            }
            if (e >= E)
                continue;
            const int k = a.k1 + ik;
            v2 P, Qc;
            if constexpr (FUSE4) {
                ypair(f, k, P, Qc);
            } else if constexpr (F == 1) {
                // k = k1 + tid + i NT: P at pk0 + i (NT + NT/16), the mirror
                // bin N_f - k at qk0 - i (NT + NT/16) (bin 0 is its own mirror)
                P = lds[pk0 + i * padded_stride(NT)];
                Qc = conjv(lds[k == 0 ? 0 : qk0 - i * padded_stride(NT)]);
            } else {
                P = lds[pad16(f * NF + k)];
                Qc = conjv(lds[pad16(f * NF + ((NF - k) & (NF - 1)))]);
            }
            const v2 A = 0.5f * (P + Qc);
            const v2 D = P - Qc;
            const v2 B = mk(0.5f * D.y, -0.5f * D.x);
            const float mag2 = mag2_of(A);
            mx = fmaxf(mx, mag2);
            const v2 S = cmul(phk, A);
            int code = -1;
            if (mag2 > gamma2) {
                const float im = B.y * A.x - B.x * A.y;   // Im(B conj A)
                const float delta = a.cdelta * im * __builtin_amdgcn_rcpf(mag2);
                const float zd = (float)a.z * delta;
                // kappa = |k - delta|; l = floor(z (kappa - k1) + 1/2) with the
                // integer part kept exact
                const float hi = delta <= (float)k ? 0.5f - zd : zd + 0.5f;
                const int ibase = delta <= (float)k ? a.z * (k - a.k1) : -a.z * (k + a.k1);
                const int l = ibase + (int)floorf(fminf(fmaxf(hi, -1.0e8f), 1.0e8f));
                code = (fabsf(zd) < 1.0e8f && l >= 0 && l < a.n_dst) ? l : -2;
            }
            if (code >= 0) {
                mn = fminf(mn, mag2);
                key[i] = (f << SEGF) | (f * a.n_dst + code);
                sv[i] = S;
                const float mag1 = fabsf(S.x) + fabsf(S.y);
#pragma unroll
                for (int ff = 0; ff < F; ++ff)
                    part[ff] += ff == f ? mag1 : 0.f;
            }
            if constexpr (DEBUG) {
                if (a.S)
                    reinterpret_cast<v2 *>(a.S)[m0 * a.n_src + (unsigned)e] = S;
                if (a.Sd)
                    reinterpret_cast<v2 *>(a.Sd)[m0 * a.n_src + (unsigned)e] = a.inv_s * cmul(phk, B);
                if (a.idx)
                    a.idx[m0 * a.n_src + (unsigned)e] = code;
            }
        }
        // wave reductions (results in lane 63)
        auto add = [](float p, float q) { return p + q; };
#pragma unroll
        for (int ff = 0; ff < F; ++ff)
            part[ff] = wave_reduce63(part[ff], 0.f, add);
        if (spec) {
            mx = wave_reduce63(mx, 0.f, [](float p, float q) { return fmaxf(p, q); });
            mn = wave_reduce63(mn, __builtin_huge_valf(), [](float p, float q) { return fminf(p, q); });
            if ((threadIdx.x & 63) == 63) {
                spart[threadIdx.x >> 6][0] = mx;
                spart[threadIdx.x >> 6][1] = mn;
            }
        }
        if ((threadIdx.x & 63) == 63) {
#pragma unroll
            for (int ff = 0; ff < F; ++ff)
                bpart[threadIdx.x >> 6][ff] = part[ff];
        }
        __syncthreads();   // FFT buffer free, frame bounds complete
        __builtin_amdgcn_s_setprio(2);
        if (spec && threadIdx.x == 0) {
            // the item is final if nothing it kept lies at or below the final
            // gamma; the running maximum grows with the item's
            float imx = spart[0][0], imn = spart[0][1];
#pragma unroll
            for (int wv = 1; wv < NT / 64; ++wv) {
                imx = fmaxf(imx, spart[wv][0]);
                imn = fminf(imn, spart[wv][1]);
            }
            g.smin[it] = imn;
            if (imx > __uint_as_float(runbits))
                atomicMax(&a.ctrl->maxbits, __float_as_uint(imx));
        }

        // bytes per stored bin: complex float, or the magnitude as float or half
        const int osh = a.out_fmt == 0 ? 3 : (a.out_fmt == 1 ? 2 : 1);
        unsigned char *__restrict__ trow =
            reinterpret_cast<unsigned char *>(a.T) + ((m0 * (int64_t)a.n_dst) << osh);
        // the bound is summed in a fixed order so the scale, hence T, is
        // reproducible bit for bit
        float scf[F];
#pragma unroll
        for (int ff = 0; ff < F; ++ff) {
            float B = 0.f;
#pragma unroll
            for (int wv = 0; wv < NT / 64; ++wv)
                B += bpart[wv][ff];
            scf[ff] = fixed_scale(B * 1.001f);
        }
        // per-frame sums of the stored row (only when the call asks for them)
        double cre = 0.0, cim = 0.0, ce2 = 0.0;
        int cf = 0;   // frame of the thread's running sums
        auto flush_col = [&]() {
            if constexpr (!COLS) {
                return;
            } else if constexpr (F == 1) {
                // called where the whole workgroup is: one atomic per wave
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    cre += __shfl_xor(cre, o, 64);
                    cim += __shfl_xor(cim, o, 64);
                    ce2 += __shfl_xor(ce2, o, 64);
                }
                if ((threadIdx.x & 63) == 0) {
                    atomicAdd(&colacc[0], cre);
                    atomicAdd(&colacc[1], cim);
                    atomicAdd(&colacc[2], ce2);
                }
                cre = cim = ce2 = 0.0;
            } else {
                if (cre != 0.0 || cim != 0.0 || ce2 != 0.0) {
                    atomicAdd(&colacc[3 * cf], cre);
                    atomicAdd(&colacc[3 * cf + 1], cim);
                    atomicAdd(&colacc[3 * cf + 2], ce2);
                }
                cre = cim = ce2 = 0.0;
            }
        };
        // Rows longer than the buffer go in chunks of equal size, a multiple of
        // NT (at most HB), so that no pass clears or stores bins past the row
        // beyond the last partial round: nst rounds of NT bins per chunk.
        int CH = HB;
        if constexpr (CHUNKED) {
            const int nch = (EH + HB - 1) / HB;
            CH = ((EH + nch - 1) / nch + NT - 1) / NT * NT;
        }
        for (int c0 = 0; c0 < (CHUNKED ? EH : 1); c0 += CH) {
            const int cn = CHUNKED ? ((EH - c0) < CH ? (EH - c0) : CH) : EH;
            // rounds of NT bins that hold the row(s): the rest of the buffer
            // is neither cleared nor stored
            const int nst = (cn + NT - 1) / NT;
#pragma unroll
            for (int i = 0; i < NST; ++i)
                if (i < nst)
                    reinterpret_cast<unsigned long long *>(hq)[threadIdx.x + i * NT] = 0ull;
            __syncthreads();
            // scatter phase (Eq. 28)
#pragma unroll
            for (int i = 0; i < R; ++i) {
                if (key[i] < 0)
                    continue;
                const int f = key[i] >> SEGF;
                const int d = (key[i] & ((1 << SEGF) - 1)) - c0;
                if (d < 0 || d >= cn)
                    continue;
                float sc = scf[0];
#pragma unroll
                for (int ff = 1; ff < F; ++ff)
                    sc = ff == f ? scf[ff] : sc;
                atomicAdd(&hq[2 * d], (int)rintf(sv[i].x * sc));
                atomicAdd(&hq[2 * d + 1], (int)rintf(sv[i].y * sc));
            }
            __syncthreads();
            // store phase.  A buffer resource bounded to the cn valid bins
            // makes the hardware drop the stores past the end, so every store
            // instruction is unconditional.
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc(trow + ((int64_t)c0 << osh), (short)0, cn << osh,
                                                  kBufferWord3);
            // bins are read in groups of SG: one LDS round trip per group.  The
            // row format is uniform per call: the loop is specialised for each
            // (complex rows, or compressed |T| rows as float or half).
            constexpr int SG = 6;
            auto store_rows = [&](auto fmt) {
                constexpr int OSH = decltype(fmt)::value;   // log2 bytes per bin
#pragma unroll
                for (int g0 = 0; g0 < NST; g0 += SG) {
                    __builtin_amdgcn_sched_barrier(0);
                    if (g0 >= nst)
                        break;
                    unsigned long long hv[SG];
#pragma unroll
                    for (int i = 0; i < SG; ++i)
                        if (g0 + i < NST && g0 + i < nst)
                            hv[i] = reinterpret_cast<const unsigned long long *>(hq)[threadIdx.x + (g0 + i) * NT];
#pragma unroll
                    for (int i = 0; i < SG; ++i) {
                        if (g0 + i >= NST || g0 + i >= nst)
                            continue;
                        const int e = threadIdx.x + (g0 + i) * NT;
                        float isc = 1.0f / scf[0];   // exact: a power of two
                        if constexpr (F > 1) {
                            int f = (int)(((float)(c0 + e) + 0.5f) * inv_ndst);
                            f = f < nvalid ? f : nvalid - 1;
                            float sc = scf[0];
#pragma unroll
                            for (int ff = 1; ff < F; ++ff)
                                sc = ff == f ? scf[ff] : sc;
                            isc = 1.0f / sc;
                        }
                        const int re = (int)(unsigned)hv[i];
                        const int im = (int)(unsigned)(hv[i] >> 32);
                        const v2 v = mk((float)re * isc, (float)im * isc);
                        if constexpr (OSH == 3) {
                            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs,
                                                                  (unsigned)e * 8u, 0, kNonTemporal);
                        } else {
                            // compressed rows: |T| (one rounding of the complex value's norm)
                            const float mg = __builtin_sqrtf(__builtin_fmaf(v.x, v.x, v.y * v.y));
                            if constexpr (OSH == 2)
                                __builtin_amdgcn_raw_buffer_store_b32(
                                    __builtin_bit_cast(unsigned, mg), rs, (unsigned)e * 4u, 0,
                                    kNonTemporal);
                            else
                                __builtin_amdgcn_raw_buffer_store_b16(
                                    __builtin_bit_cast(unsigned short, (_Float16)mg), rs,
                                    (unsigned)e * 2u, 0, kNonTemporal);
                        }
                    }
                }
            };
            if (osh == 3)
                store_rows(IntC<3>{});
            else if (osh == 2)
                store_rows(IntC<2>{});
            else
                store_rows(IntC<1>{});
            if (COLS && a.colstats) {
                // Per-frame sums and energy of the stored FP32 row (a uniform
                // branch: calls that ask for them), in FP64, from the same
                // histogram values and scales as the stores above.  A
                // thread's frame index only grows over its bins, so its sums
                // go to that frame's LDS slot when the frame changes.
                for (int r = 0; r < nst; ++r) {
                    const int e = threadIdx.x + r * NT;
                    if (e >= cn)
                        break;
                    const unsigned long long h = reinterpret_cast<const unsigned long long *>(hq)[e];
                    int f = 0;
                    float sc = scf[0];
                    if constexpr (F > 1) {
                        f = (int)(((float)(c0 + e) + 0.5f) * inv_ndst);
                        f = f < nvalid ? f : nvalid - 1;
#pragma unroll
                        for (int ff = 1; ff < F; ++ff)
                            sc = ff == f ? scf[ff] : sc;
                        if (f != cf) {
                            flush_col();
                            cf = f;
                        }
                    }
                    const float isc = 1.0f / sc;
                    const double dx = (double)((float)(int)(unsigned)h * isc);
                    const double dy = (double)((float)(int)(unsigned)(h >> 32) * isc);
                    cre += dx;
                    cim += dy;
                    ce2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, ce2));
                }
            }
            if (CHUNKED && c0 + CH < EH)
                __syncthreads();   // store reads done before the next chunk is cleared
        }
        if (COLS && a.colstats) {   // uniform: the call asked for per-frame sums
            flush_col();
            __syncthreads();
            if ((int)threadIdx.x < 3 * nvalid)
                a.colstats[m0 * 3 + threadIdx.x] = colacc[threadIdx.x];
            if (threadIdx.x < 3 * F)
                colacc[threadIdx.x] = 0.0;
        }
        a = an;
        new_chan = chg;
        it = itn;
        li += gridDim.x;
    }
}

// ---------------------------------------------------------------------------
// STFT synthesis (Sec. 2.1, Eqs. 10-11) from in-band STFT rows.  Per frame m,
// s[m, j] = (1/N_f) sum_k a_k Re(S[m, k] e^{+i 2 pi k j / N_f}), j in [-M, M]
// (Eq. 10: the centre phase e^{-i 2 pi k M / N_f} times an N_f-point inverse
// DFT, read at n = j + M), then the overlap-add of Eq. 11 with the per-sample
// normalisation sum_m g[n - mH]^2 (reading D3: the paper's unit sum holds for
// no hop > 1 with its unit-energy window, and this one also covers the ends).
//
// The one-sided spectrum is extended Hermitian (conjugate mirror, DC and
// Nyquist real) so that every inverse is real, and two frames share one
// complex inverse: Z = Y_a + i Y_b gives y_a + i y_b.  The inverse runs as the
// forward FFT of conj Z (its output is conj z).  Each workgroup owns a tile of
// TS output samples and inverts every frame whose window reaches it (tiles
// overlap by the window length, so each frame is inverted about (TS + L) / TS
// times); each thread gathers its own TS / NT samples from the frames in
// registers, so the sums need no atomics and do not depend on scheduling.
// ---------------------------------------------------------------------------
template <int NF>
__global__ __launch_bounds__(Geo<NF>::NT) void syn_kernel(SynArgs a)
{
    using G = Geo<NF>;
    constexpr int F = G::F, NT = G::NT, NHI = NF / 64;
    constexpr int TS = kSynTile, PER = TS / NT;
    static_assert(TS % NT == 0, "a tile is a whole number of sample rounds");
    __shared__ v2 lds[G::LDS];
    __shared__ v2 twl[Twiddles<NF>::TW];
    __shared__ v2 clo[64], chi[NHI];   // W^t = chi[t / 64] clo[t mod 64], W = e^{-i 2 pi / N_f}
    const v2 *__restrict__ twid = reinterpret_cast<const v2 *>(a.twid);
    Twiddles<NF> tw;
    tw.load(twl, twid);
    for (int e = threadIdx.x; e < 64 + NHI; e += NT) {
        if (e < 64)
            clo[e] = twid[(unsigned)e];
        else
            chi[e - 64] = twid[(unsigned)(e - 64) * 64u];
    }
    __syncthreads();
    const int M = a.M, H = a.hop, L = 2 * a.M + 1;
    const int n = (int)a.n, nfr = (int)a.n_frames;
    const int t0 = (int)blockIdx.x * TS;
    const int t1 = t0 + TS - 1 < n - 1 ? t0 + TS - 1 : n - 1;
    const int mlo = t0 - M > 0 ? (t0 - M + H - 1) / H : 0;
    int mhi = (t1 + M) / H;
    mhi = mhi < nfr - 1 ? mhi : nfr - 1;
    const v2 *__restrict__ S = reinterpret_cast<const v2 *>(a.S);
    const v2 *__restrict__ win = reinterpret_cast<const v2 *>(a.win);
    const int k1 = a.k1, k2 = a.k2, n_src = a.n_src;
    // in-band S~[m, k] = S[m, k] W^{k M} (the centre phase removed), 0 outside
    auto spec = [&](int m, int k) -> v2 {
        if (m > mhi || k < k1 || k > k2)
            return mk(0.f, 0.f);
        const int t = (k * M) & (NF - 1);
        return cmul(S[(int64_t)m * n_src + (k - k1)], cmul(chi[t >> 6], clo[t & 63]));
    };
    float acc[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i)
        acc[i] = 0.f;
    for (int m0 = mlo; m0 <= mhi; m0 += 2 * F) {
        // pass 1 reads conj Z of slot f (frames m0 + 2f, m0 + 2f + 1) at index idx
        pass1<NF, 16>(lds, [&](int f, int idx) -> v2 {
            const int ma = m0 + 2 * f, mb = ma + 1;
            v2 ya, yb;
            if (2 * idx <= NF) {
                ya = spec(ma, idx);
                yb = spec(mb, idx);
                if (idx == 0 || 2 * idx == NF) {   // real at DC and at Nyquist
                    ya.y = 0.f;
                    yb.y = 0.f;
                }
            } else {                               // conjugate mirror
                ya = conjv(spec(ma, NF - idx));
                yb = conjv(spec(mb, NF - idx));
            }
            // conj(Y_a + i Y_b)
            return mk(ya.x - yb.y, -(ya.y + yb.x));
        });
        tw.passes(lds, twl);
        // FFT(conj Z) = conj z = y_a - i y_b; each thread gathers its samples
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const int ma = m0 + 2 * f;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int m = ma + h;
                if (m > mhi)
                    continue;
                const int base = m * H - M;   // sample of window index 0 (n = j + M)
#pragma unroll
                for (int i = 0; i < PER; ++i) {
                    const int sidx = t0 + (int)threadIdx.x + i * NT;
                    const int nn = sidx - base;
                    if (nn >= 0 && nn < L) {
                        const v2 o = lds[pad16(f * NF + nn)];
                        acc[i] += win[nn].x * (h ? -o.y : o.x);
                    }
                }
            }
        }
        __syncthreads();   // gathers done before the next pass 1 writes the buffer
    }
    // Eq. 11 with the per-sample normalisation sum_m g[n - mH]^2
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int sidx = t0 + (int)threadIdx.x + i * NT;
        if (sidx > t1)
            continue;
        const int flo = sidx - M > 0 ? (sidx - M + H - 1) / H : 0;
        const int fhi = (sidx + M) / H;
        float dv;
        if (sidx >= M && fhi <= nfr - 1) {
            dv = a.den2[sidx % H];
        } else {
            dv = 0.f;
            const int hi = fhi < nfr - 1 ? fhi : nfr - 1;
            for (int m = flo; m <= hi; ++m) {
                const float gj = win[sidx - m * H + M].x;
                dv = __builtin_fmaf(gj, gj, dv);
            }
        }
        a.xhat[sidx] = dv > 0.f ? acc[i] * a.inv_nfft / dv : 0.f;
    }
}

// Fix-up list of a speculative forward: items whose least kept |S|^2 is at or
// below the channel's final gamma^2 (one atomic per wave appends them).  The
// final gamma follows from maxbits as in gamma_kernel; workgroup 0 also writes
// it into the channels' control blocks.
__global__ __launch_bounds__(256) void spec_list_kernel(GroupLaunch g)
{
    const CA ChanDesc *ch = (const CA ChanDesc *)g.ch;
    const int lane = threadIdx.x & 63;
    if (blockIdx.x == 0) {
        for (int cc = threadIdx.x; cc < g.n_ch; cc += 256) {
            Ctrl *ctrl = g.ch[cc].ctrl;
            const float m2 = __uint_as_float(ctrl->maxbits);
            const float gm = g.ch[cc].thr_mode == 1 ? g.ch[cc].thr * sqrtf(m2) : g.ch[cc].thr;
            ctrl->maxabs2 = m2;
            ctrl->gamma = gm;
            ctrl->gamma2 = gamma2_of(g.ch[cc].thr_mode, g.ch[cc].thr, m2);
        }
    }
    int c = 0;
    for (int64_t base = g.item_begin + (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63);
         base < g.item_stop; base += (int64_t)gridDim.x * 256) {
        const int64_t it = base + lane;
        bool redo = false;
        if (it < g.item_stop) {
            while (c < g.n_ch - 1 && it >= ch[c].item_end)
                ++c;
            const float m2 = __uint_as_float(__hip_atomic_load(&g.ch[c].ctrl->maxbits, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT));
            redo = g.smin[it] <= gamma2_of(ch[c].thr_mode, ch[c].thr, m2);
        }
        const unsigned long long bal = __ballot(redo);
        if (bal == 0ull)
            continue;
        int at = 0;
        if (lane == 0)
            at = atomicAdd(g.list_n, __popcll(bal));
        at = __shfl(at, 0, 64);
        if (redo)
            g.list[at + __popcll(bal & ((1ull << lane) - 1ull))] = (int32_t)it;
    }
}

// Clear the running maxima of the launch's channels (and the fix-up count).
__global__ __launch_bounds__(256) void clear_max_kernel(GroupLaunch g)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < g.n_ch)
        g.ch[c].ctrl->maxbits = 0u;
    if (c == 0 && g.list_n)
        *g.list_n = 0;
}

// gamma of every channel: rho sqrt(max |S|^2) (relative) or the given value.
__global__ __launch_bounds__(256) void gamma_kernel(GroupLaunch g)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= g.n_ch)
        return;
    Ctrl *ctrl = g.ch[c].ctrl;
    const float m2 = __uint_as_float(ctrl->maxbits);
    const float gm = g.ch[c].thr_mode == 1 ? g.ch[c].thr * sqrtf(m2) : g.ch[c].thr;
    ctrl->maxabs2 = m2;
    ctrl->gamma = gm;
    ctrl->gamma2 = gamma2_of(g.ch[c].thr_mode, g.ch[c].thr, m2);
}

// Write one descriptor into device memory.
__global__ __launch_bounds__(64) void put_desc_kernel(ChanDesc d, ChanDesc *dst, int clear,
                                                      int32_t *list_n)
{
    if (threadIdx.x == 0) {
        *dst = d;
        if (clear)
            d.ctrl->maxbits = 0u;
        if (list_n)
            *list_n = 0;
    }
}

// ---------------------------------------------------------------------------
// Inverse (Eqs. 25-26).  One workgroup per 256 output samples and component.
// ---------------------------------------------------------------------------

// (b * j) mod G for b, j in [0, G), G <= 65536 (so the product fits 32 bits).
__device__ __forceinline__ int mulmod(uint32_t b, uint32_t j, int G, int pow2, float invG)
{
    const uint32_t p = b * j;
    if (pow2)
        return (int)(p & (uint32_t)(G - 1));
    const uint32_t q = (uint32_t)((float)p * invG);
    int r = (int)(p - q * (uint32_t)G);
    while (r < 0)
        r += G;
    while (r >= G)
        r -= G;
    return r;
}

__device__ __forceinline__ v2 phasor(const v2 *tlo, const v2 *thi, int idx, int lo_bits)
{
    return cmul(thi[idx >> lo_bits], tlo[idx & ((1 << lo_bits) - 1)]);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void err_reduce(double d2, double r2, double *err, int q)
{
    __shared__ double red[2][4];
    d2 = wave_sum(d2);
    r2 = wave_sum(r2);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = d2;
        red[1][w] = r2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&err[2 * q], red[0][0] + red[0][1] + red[0][2] + red[0][3]);
        atomicAdd(&err[2 * q + 1], red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    }
}

// Descriptor of workgroup `blk` of an inverse launch: the last channel whose
// blk0 <= blk (binary search over the list; every thread gets the same c).
__device__ __forceinline__ int inv_chan_of(const CA InvDesc *ch, int n_ch, int64_t blk)
{
    int lo = 0, hi = n_ch - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ch[mid].blk0 <= blk)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Inverse on the matrix cores.  For the output samples n of a tile and the
// frames m of the call whose windows reach them, with d = l - d_lo (l the
// destination bin, d_lo the lowest destination of the zones met) and
// b = z k1 + l the bin on the zN_f grid,
//   e^{i 2 pi b (n - mH)/G} = e^{i 2 pi b n / G} e^{-i 2 pi b m H / G},
// so the numerator of Eq. 26 is
//   sum_d Re( e^{i 2 pi b n / G} Z[d, n] ),
//   Z[d, n] = sum_m c~[m, d] g[n - mH],  c~[m, d] = (a_l / N_f) T[m, l] e^{-i 2 pi b m H / G}
// (zero outside the frame's zone).  Z is the product of the coefficient matrix
// (16 bins x real/imaginary = 32 rows, frames) with the banded window matrix
// (frames x samples), run on the 32x32x16 FP16 MFMA with both operands split:
// v 2^s = hi + lo, each an FP16 number (hi the rounding of v 2^s, lo that of
// the remainder), so hi + lo carries 22 significant bits, and the three
// products hi hi + hi lo + lo hi are exact in the FP32 accumulator (the
// dropped lo lo is below 2^-22 of the term).  The coefficients' power of two
// 2^s puts the block's largest one just under 2^14; the window's, 2^tg, is
// fixed on the host.  Frames come in blocks of KB staged in LDS as FP16 rows
// (frames contiguous, so a lane's 8 frames are one 16-byte read).  Each lane
// then holds 16 of the 32 rows of one sample column: the sum over bins is 16
// multiply-adds in registers and one exchange with the lane holding the other
// 16 rows.  Phase indices are reduced mod G in integers.  Lane layout
// (checked on the hardware): A lane l = row l mod 32, k = 8 (l / 32) .. + 7;
// B lane l = the same k, column l mod 32; accumulator i = row
// 8 (i / 4) + 4 (l / 32) + i mod 4, column l mod 32.
//
// Denominator: for samples whose frames all exist it depends on n mod H only
// and comes from a table built on the host in float64; near the ends of the
// signal it is summed here.
// Wide tiles.  A workgroup covers TF x 256 consecutive output samples (TF = 4,
// or 8 with the decimated window table; each wave TF groups of 64, two
// columns of 32 per group): the zone coefficients of the tile's frames are
// staged once per group of 16 bins and serve every sample group, and the
// tables are built once per TF x 256 samples.  Frames a tile meets grow by
// 256 TF / H, so a wide tile stages (256 TF + 2M) / H frames where TF narrow
// ones stage TF (256 + 2M) / H.
constexpr int kInvTile = 256;                  // samples per group of four waves (4 x 2 x 32)
template <int TF>
struct InvGeo {
    static constexpr int KB = TF == 1 ? 96 : 144;   // frames staged per block (multiple of 16)
    static constexpr int KBP = KB + 8;              // padded row of staged halves
    static constexpr int STAGE = KB * 16 / 256;     // staged coefficients per thread and block
};

typedef _Float16 f16x8v __attribute__((ext_vector_type(8)));

typedef unsigned u4v_t __attribute__((ext_vector_type(4)));

// v ~ hi + lo in FP16 (|v| < 2^15), as bit patterns
__device__ __forceinline__ void split_f16(float v, unsigned &hi, unsigned &lo)
{
    const _Float16 h = (_Float16)v;
    hi = __builtin_bit_cast(unsigned short, h);
    lo = __builtin_bit_cast(unsigned short, (_Float16)(v - (float)h));
}

// LDS layout of the inverse (byte offsets, each 16-byte aligned).
struct InvLds {
    size_t gpk, rid, ahi, alo, fred, red, total;
};
__host__ __device__ inline size_t inv_align16(size_t v)
{
    return (v + 15) & ~(size_t)15;
}
// ng groups of 16 destinations staged at once (1, 2 or 4): ahi and alo
// hold ng blocks of 32 rows of kbp halves each, fred ng x 4 wave maxima.
__host__ __device__ inline InvLds inv_lds_layout(int max_tab, int max_gtab, int max_k, int kbp,
                                                 int ng = 1)
{
    InvLds o;
    o.gpk = inv_align16(8 * (size_t)max_tab);
    o.rid = inv_align16(o.gpk + 4 * (size_t)max_gtab);
    o.ahi = inv_align16(o.rid + 4 * (size_t)max_k);
    o.alo = o.ahi + (size_t)ng * 2 * 32 * (size_t)kbp;
    o.fred = inv_align16(o.alo + (size_t)ng * 2 * 32 * (size_t)kbp);
    o.red = o.fred + 16 * (size_t)ng;
    o.total = o.red + 16;
    return o;
}

// Row length (halves) of the grouped inverse's staged blocks: the frames a
// tile meets rounded up to 16, plus 8; an odd multiple of 8, so that the 16
// lanes of a 16-byte read reach 16 different groups of four banks.
__host__ __device__ inline int inv_group_kbp(int max_k)
{
    return ((max_k + 15) & ~15) + 8;
}

// The frame steps of one wave's 64 samples (sample group cg of the tile) over
// the staged frames [kb, kb + kn): steps of 16 from kw0 (a multiple of 16,
// relative to kb) while k0 <= kw1, covering the frames whose windows reach
// the wave's samples (the others meet g = 0 in every column of the wave).
// Uniform over the wave, packed as kw0 | (kw1 + 1) << 16 (0 <= kw0, kw1 + 1
// < 2^15).  Then the lane's window addressing: j0 = n - m H of
// its first frame (k0 + 8 half) for column 0; with the decimated table, the
// word offsets (from the table's start) of that frame's residue row entries
// for columns 0 and 31 + 1, packed as off0 | off1 << 16.
struct WaveSteps {
    int kw;     // packed kw0, kw1
    int lane;   // DEC: packed offsets; otherwise j0
};
template <bool DEC>
__device__ __forceinline__ WaveSteps wave_steps(int tile_lo, int cg, int wave, int col, int half,
                                                int mlo, int kb, int kn, int M, int H, int JL,
                                                int TR, uint32_t hinv)
{
    WaveSteps w;
    const int w_lo = tile_lo + 256 * cg + 64 * __builtin_amdgcn_readfirstlane(wave);
    const int wm_lo = w_lo - M > 0 ? (w_lo - M + H - 1) / H : 0;
    const int wm_hi = (w_lo + 63 + M) / H;
    int kw0 = wm_lo - mlo - kb, kw1 = wm_hi - mlo - kb;
    kw0 = kw0 > 0 ? kw0 & ~15 : 0;
    kw1 = kw1 < kn - 1 ? kw1 : kn - 1;
    w.kw = kw0 | ((kw1 < 0 ? 0 : kw1 + 1) << 16);
    const int j0 = w_lo + col - mlo * H - (kb + kw0 + 8 * half) * H;
    if constexpr (DEC) {
        // The lane's 8 values g[j - i H], i = 0..7, are the words p[7 - i] of
        // its residue row; a step of 16 frames moves p by -16.  Every j a step
        // reaches lies within JL of 0: the steps start up to 15 frames before
        // the wave's first frame and end up to 15 after its last, and a wave
        // spans 64 samples, so |j| <= M + 63 + 15 H.
        // u0 = q0 H + r0 and u1 = u0 + 32 = q1 H + r1, 0 <= u0 < 2^24: the
        // high word of u m, m = floor(2^32 / H) (hinv), is the quotient or one
        // less, then corrected
        const uint32_t u0 = (uint32_t)(j0 + JL), u1 = u0 + 32;
        uint32_t q0 = __umulhi(u0, hinv), q1 = __umulhi(u1, hinv);
        uint32_t r0 = u0 - q0 * (uint32_t)H, r1 = u1 - q1 * (uint32_t)H;
        if (r0 >= (uint32_t)H) {
            ++q0;
            r0 -= H;
        }
        if (r1 >= (uint32_t)H) {
            ++q1;
            r1 -= H;
        }
        // every word read lies in the table (fewer than 2^16 words)
        w.lane = (int)((r0 * TR + q0 - 7) | ((r1 * TR + q1 - 7) << 16));
    } else {
        w.lane = j0;
    }
    return w;
}

// Window contraction of one wave's 64 samples over the steps ws: acc0 and
// acc1 (columns 0..31 and 32..63) accumulate Z 2^(sc + tg) =
// sum_m c~[m, d] g[n - mH] (the staged rows are zero past kn).  ZERO: the
// sums start here (the first step's products take a zero accumulator in
// place of acc); returns false, leaving acc untouched, when no frame reaches
// the wave's samples (the sums are zero).
template <bool DEC, int KBP, bool ZERO>
__device__ __forceinline__ bool wave_mfma(f32x16 &acc0, f32x16 &acc1, const unsigned short *aph,
                                          const unsigned short *apl, const unsigned *gpk,
                                          const WaveSteps &ws, int M, int H)
{
    int j0 = ws.lane;
    const unsigned *pc0 = gpk, *pc1 = gpk;
    if constexpr (DEC) {
        pc0 = gpk + (ws.lane & 0xffff);
        pc1 = gpk + ((unsigned)ws.lane >> 16);
    }
    // one step of 16 frames; FRESH: the first step of a fresh sum, whose
    // products take a zero accumulator operand (no register clearing)
    auto step = [&](int k0, auto fresh) {
        constexpr bool FRESH = decltype(fresh)::value != 0;
        const u4v_t a_hi = *reinterpret_cast<const u4v_t *>(aph + k0);
        const u4v_t a_lo = *reinterpret_cast<const u4v_t *>(apl + k0);
        const f16x8v ah = __builtin_bit_cast(f16x8v, a_hi), al = __builtin_bit_cast(f16x8v, a_lo);
        // B of column c: g[n + 32 c - m H] for the lane's 8 frames
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            unsigned w[8];
            if constexpr (DEC) {
                const unsigned *pc = c ? pc1 : pc0;
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    w[i] = pc[7 - i];
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int j = j0 + 32 * c - i * H;
                    w[i] = gpk[min(max(j, -M - 1), M + 1) + M + 1];
                }
            }
            u4v_t bh, bl;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bh[i] = __builtin_amdgcn_perm(w[2 * i + 1], w[2 * i], 0x05040100u);
                bl[i] = __builtin_amdgcn_perm(w[2 * i + 1], w[2 * i], 0x07060302u);
            }
            const f16x8v fh = __builtin_bit_cast(f16x8v, bh), fl = __builtin_bit_cast(f16x8v, bl);
            f32x16 &acc = c ? acc1 : acc0;
            if constexpr (FRESH)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, fh, f32x16{}, 0, 0, 0);
            else
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, fh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, fl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, fh, acc, 0, 0, 0);
        }
        j0 -= 16 * H;
        pc0 -= 16;
        pc1 -= 16;
    };
    int k0 = ws.kw & 0xffff;
    const int kw1 = (ws.kw >> 16) - 1;
    if constexpr (ZERO) {
        if (k0 > kw1)   // no frame reaches the wave's samples
            return false;
        step(k0, IntC<1>{});
        k0 += 16;
    }
    for (; k0 <= kw1; k0 += 16)
        step(k0, IntC<0>{});
    return true;
}

// ONE: every tile's frames fit one staged block (K <= KB), so the sums start
// after the staging and need no registers during it.  DEC: the window table is
// decimated by the hop, so a lane's 8 window values are consecutive words;
// otherwise they are gathered with clamped indices.  TF: sample groups of 256
// per workgroup (1, or 4 or 8 with ONE).  Waves per SIMD: the most that each
// variant fits without spilling registers (wide tiles: the bound of three
// leaves the same 119-123 registers, four waves per SIMD, and schedules the
// code for it 1.5 % faster than the bound of four).
template <bool ONE, bool DEC, int TF>
__global__ __launch_bounds__(256, TF > 1 ? 3 : (ONE ? (DEC ? 6 : 5) : 4)) void inv_kernel(InvLaunch l)
{
    using IG = InvGeo<TF>;
    constexpr int KB = IG::KB, KBP = IG::KBP, STAGE = IG::STAGE;
    static_assert(TF == 1 || ONE, "wide tiles stage every frame in one block");
    static_assert(TF == 1 || KB == kInvWideKB, "host and kernel agree on the wide block");
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t blk = l.blk_begin + (int64_t)blockIdx.x;
    const CA InvDesc *chs = (const CA InvDesc *)l.ch;
    const CA InvDesc &a = chs[inv_chan_of(chs, l.n_ch, blk)];
    const int nlo = 1 << a.lo_bits;
    const int nhi = (a.G + nlo - 1) >> a.lo_bits;
    const InvLds lay = inv_lds_layout(l.max_tab, l.max_gtab, l.max_k, KBP);
    v2 *tlo = reinterpret_cast<v2 *>(smem);
    v2 *thi = tlo + nlo;
    unsigned *gpk = reinterpret_cast<unsigned *>(smem + lay.gpk);   // window, packed
    int *rid = reinterpret_cast<int *>(smem + lay.rid);             // [max_k]
    unsigned short *ahi = reinterpret_cast<unsigned short *>(smem + lay.ahi);   // [32][KBP]
    unsigned short *alo = reinterpret_cast<unsigned short *>(smem + lay.alo);   // [32][KBP]
    float *fred = reinterpret_cast<float *>(smem + lay.fred);       // [4]
    int *red = reinterpret_cast<int *>(smem + lay.red);             // [2]

    // Signals hold fewer than 2^30 samples and n_comp * tiles < 2^31 (checked
    // by the host), so sample, frame and tile indices fit 32 bits.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 31, half = lane >> 5;
    const unsigned local = (unsigned)(blk - a.blk0);
    const unsigned tiles = (unsigned)a.tiles;
    const int q = (int)(local / tiles);
    const int span_lo = (int)a.span_lo, span_end = (int)(a.span_lo + a.span_len - 1);
    const int tile_lo = span_lo + (int)(local - (unsigned)q * tiles) * (kInvTile * TF);
    const int tile_hi = tile_lo + kInvTile * TF - 1 < span_end ? tile_lo + kInvTile * TF - 1 : span_end;
    const int M = a.M, H = a.hop, Gi = a.G;
    const uint32_t hinv = 0xffffffffu / (uint32_t)H;   // floor(2^32 / H) unless H is 1
    const int frame0 = (int)a.frame0, nfr = (int)a.nframes, nframes_all = (int)a.n_frames;
    const v2 *__restrict__ win = reinterpret_cast<const v2 *>(a.win);

#pragma unroll 2
    for (int e = threadIdx.x; e < nlo; e += 256)
        tlo[e] = reinterpret_cast<const v2 *>(a.ph_lo)[e];
#pragma unroll 2
    for (int e = threadIdx.x; e < nhi; e += 256)
        thi[e] = reinterpret_cast<const v2 *>(a.ph_hi)[e];
    // Window table, g[j] 2^tg as FP16 hi | lo << 16, zero for |j| > M.  DEC:
    // gpk[r TR + t] holds j = r + t H - JL (r = residue mod H); otherwise
    // gpk[j + M + 1] for |j| <= M + 1 (indices outside are clamped onto the
    // zero ends).
    const float gsc = a.g_scale;
    const int JL = DEC ? a.dec_reach : 0;
    const int TR = DEC ? a.dec_row : 0;
    const int n_tab = DEC ? H * TR : a.L + 2;
#pragma unroll 4
    for (int e = threadIdx.x; e < n_tab; e += 256) {
        int j;
        if constexpr (DEC) {
            const int r = e / TR;
            j = r + (e - r * TR) * H - JL;
        } else {
            j = e - M - 1;
        }
        unsigned w = 0u;
        if (j >= -M && j <= M) {
            unsigned h, lw;
            split_f16(win[j + M].x * gsc, h, lw);
            w = h | (lw << 16);
        }
        gpk[e] = w;
    }

    // Frames of this call whose window reaches the tile.
    int mlo = tile_lo - M > 0 ? (tile_lo - M + H - 1) / H : 0;
    int mhi = (tile_hi + M) / H;
    if (mlo < frame0)
        mlo = frame0;
    if (mhi > frame0 + nfr - 1)
        mhi = frame0 + nfr - 1;
    const int K = mhi >= mlo ? mhi - mlo + 1 : 0;
    const int32_t *__restrict__ ridge = a.ridge + (int64_t)q * a.nframes + (mlo - frame0);
    for (int k = threadIdx.x; k < K; k += 256)
        rid[k] = ridge[k];
    if (threadIdx.x < 2)
        red[threadIdx.x] = threadIdx.x == 0 ? 0x7fffffff : -1;
    __syncthreads();
    {   // destinations met by the zones of these frames
        int dmin = 0x7fffffff, dmax = -1;
        for (int k = threadIdx.x; k < K; k += 256) {
            const int r = rid[k];
            if (r >= 0) {
                dmin = min(dmin, max(r - a.hw, 0));
                dmax = max(dmax, min(r + a.hw, a.n_dst - 1));
            }
        }
        if (dmax >= 0) {
            atomicMin(&red[0], dmin);
            atomicMax(&red[1], dmax);
        }
    }
    __syncthreads();
    const int d_lo = red[0], d_hi = red[1];
    const int zk1 = a.z * a.k1;
    const uint32_t G = (uint32_t)Gi;
    const bool pow2 = a.g_pow2 != 0;
    // e^{i 2 pi 32 / G} and e^{i 2 pi 128 / G} (tables complete: the barrier above)
    const v2 w32 = phasor(tlo, thi, (int)(32u % G), a.lo_bits);
    const v2 w128 = phasor(tlo, thi, (int)(128u % G), a.lo_bits);
    const uint32_t mh0 = (uint32_t)(mlo * H) % G;    // (m_lo H) mod G
    const uint32_t n0g = (uint32_t)tile_lo % G;      // tile_lo mod G
    const uint32_t hg = (uint32_t)H % G;             // H mod G

    const v2 *__restrict__ Trow = reinterpret_cast<const v2 *>(a.T) + (int64_t)(mlo - frame0) * a.n_dst;
    const unsigned short *aph = ahi + col * KBP + 8 * half;   // this lane's A row and k chunk
    const unsigned short *apl = alo + col * KBP + 8 * half;
    // ONE with the decimated table and up to four sample groups: each sample
    // group's frame steps and window addressing do not depend on the
    // destination group; they are set once per tile (the other variants,
    // short of registers, set them per destination group)
    constexpr bool HOIST = ONE && DEC && TF <= 4;
    WaveSteps wst[HOIST ? TF : 1];
    if constexpr (HOIST) {
#pragma unroll
        for (int cg = 0; cg < TF; ++cg)
            wst[cg] = wave_steps<DEC>(tile_lo, cg, wave, col, half, mlo, 0, K, M, H, JL, TR, hinv);
    }
    // y[cg]: the sum for sample 256 cg + 64 wave + col + 32 half of the tile
    // (both halves of a column pair hold both sums; each keeps its own)
    float y[TF];
#pragma unroll
    for (int cg = 0; cg < TF; ++cg)
        y[cg] = 0.f;
    for (int d0 = d_lo; d0 <= d_hi; d0 += 16) {
        f32x16 acc0, acc1;
        if constexpr (!ONE) {
            acc0 = f32x16{};
            acc1 = f32x16{};
        }
        int sc = 0;   // accumulators hold Z 2^(sc + tg)
        for (int kb = 0; kb < (ONE ? 1 : K); kb += KB) {
            const int kn = K - kb < KB ? K - kb : KB;
            const int kn16 = (kn + 15) & ~15;
            // an opaque copy of the thread index keeps the compiler from
            // hoisting the staging indices out of the loops (and spilling them)
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            // c~[m, d] of this block in registers: 16 destinations per frame
            float cre[STAGE], cim[STAGE];
            float amax = 0.f;
            // rounds of 256 coefficients (16 frames) up to the staged rows
            const int nrd = kn16 / 16;
#pragma unroll
            for (int i = 0; i < STAGE; ++i) {
                cre[i] = cim[i] = 0.f;
                if (i >= nrd)
                    continue;
                const int e = tid + 256 * i;
                const int kk = e >> 4, dd = e & 15;
                const int k = kb + kk;
                const int ld = d0 + dd;
                v2 c = mk(0.f, 0.f);
                const int r = (kk < kn && k < K) ? rid[k] : -1;
                if (r >= 0 && ld <= d_hi && ld >= r - a.hw && ld <= r + a.hw) {
                    const int b = zk1 + ld;   // < z (k2 + 1) <= G
                    const float wgt = (b == 0 || 2 * b == Gi) ? 1.f : 2.f;
                    const v2 t = Trow[(int64_t)k * a.n_dst + ld];
                    // (m H) mod G = (m_lo H + k H) mod G, k H < 2^31
                    uint32_t mh = mh0 + (uint32_t)k * hg;
                    mh = pow2 ? (mh & (G - 1)) : mh % G;
                    const int bm = mulmod((uint32_t)b, mh, Gi, a.g_pow2, a.inv_G);
                    const v2 ph = phasor(tlo, thi, bm, a.lo_bits);   // e^{+i 2 pi b m H / G}
                    c = (wgt * a.inv_nfft) * cmul(t, conjv(ph));
                }
                cre[i] = c.x;
                cim[i] = c.y;
                amax = fmaxf(amax, fmaxf(fabsf(c.x), fabsf(c.y)));
            }
            // the block's power of two: largest |c~| 2^s in [2^13, 2^14)
            amax = wave_reduce63(amax, 0.f, [](float p, float r) { return fmaxf(p, r); });
            if (lane == 63)
                fred[wave] = amax;
            __syncthreads();   // maxima in; the previous block's halves consumed
            const float bmax = fmaxf(fmaxf(fred[0], fred[1]), fmaxf(fred[2], fred[3]));
            int ex = 0;
            (void)frexpf(bmax, &ex);   // bmax < 2^ex (ex = 0 for bmax = 0)
            int sb = 14 - ex;
            sb = sb > 100 ? 100 : (sb < -100 ? -100 : sb);   // 2^sb stays a normal float
            if (kb == 0) {
                sc = sb;
            } else if (sb < sc) {
                // a later block needs a smaller power: rescale the sums (exact)
                const float f = ldexpf(1.f, sb - sc);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    acc0[i] *= f;
                    acc1[i] *= f;
                }
                sc = sb;
            }
            const float scl = ldexpf(1.f, sc);
#pragma unroll
            for (int i = 0; i < STAGE; ++i) {
                const int e = tid + 256 * i;
                const int kk = e >> 4, dd = e & 15;
                if (i < nrd) {   // kk < kn16
                    unsigned h, lw;
                    split_f16(cre[i] * scl, h, lw);
                    ahi[(2 * dd) * KBP + kk] = (unsigned short)h;
                    alo[(2 * dd) * KBP + kk] = (unsigned short)lw;
                    split_f16(cim[i] * scl, h, lw);
                    ahi[(2 * dd + 1) * KBP + kk] = (unsigned short)h;
                    alo[(2 * dd + 1) * KBP + kk] = (unsigned short)lw;
                }
            }
            __syncthreads();
            if constexpr (!ONE) {
                const WaveSteps ws = wave_steps<DEC>(tile_lo, 0, wave, col, half, mlo, kb, kn, M, H,
                                                     JL, TR, hinv);
                wave_mfma<DEC, KBP, false>(acc0, acc1, aph, apl, gpk, ws, M, H);
            }
        }
        // rows 8 (i/4) + 4 half + i mod 4 = 2 dd + p: dd = 4 (i/4) + 2 half + (i mod 4) / 2
        const uint32_t bb = (uint32_t)(zk1 + d0 + 2 * half);
        const float unscale = ldexpf(a.g_unscale, -sc);
        // the second column of a pair (n + 32) takes the first's phasors
        // times these: e^{i 2 pi 32 bb / G}
        const v2 e32 = phasor(tlo, thi, mulmod(bb, 32u % G, Gi, a.g_pow2, a.inv_G), a.lo_bits);
#pragma unroll
        for (int cg = 0; cg < TF; ++cg) {
            if constexpr (ONE) {
                WaveSteps ws;
                if constexpr (HOIST)
                    ws = wst[cg];
                else
                    ws = wave_steps<DEC>(tile_lo, cg, wave, col, half, mlo, 0, K, M, H, JL, TR, hinv);
                if (!wave_mfma<DEC, KBP, true>(acc0, acc1, aph, apl, gpk, ws, M, H))
                    continue;   // no frame reaches these samples: the sums are zero
            }
            // nm = n mod G of the first column (n - tile_lo < 2048, so the
            // sum stays below 2^31)
            uint32_t nm = n0g + (uint32_t)(256 * cg + 64 * wave + col);
            nm = pow2 ? (nm & (G - 1)) : nm % G;
            v2 w = phasor(tlo, thi, (int)nm, a.lo_bits);                             // e^{i 2 pi n/G}
            v2 e = phasor(tlo, thi, mulmod(bb, nm, Gi, a.g_pow2, a.inv_G), a.lo_bits);   // bin bb
            v2 w4 = cmul(cmul(w, w), cmul(w, w));
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (c == 1) {   // n + 32: w32, w32^4 and e32 (one rounding each)
                    w = cmul(w, w32);
                    w4 = cmul(w4, w128);
                    e = cmul(e, e32);
                }
                const f32x16 &acc = c ? acc1 : acc0;
                // sum over the lane's 8 rows of Re(e w^(4 g + s) Z): with
                // V_g = Z_(g,0) + w Z_(g,1), the sum is Re(e P), P = sum_g w4^g V_g
                // (Horner in w4)
                auto vg = [&](int g4) {
                    return mk(fmaf(w.x, acc[4 * g4 + 2], fmaf(-w.y, acc[4 * g4 + 3], acc[4 * g4])),
                              fmaf(w.x, acc[4 * g4 + 3], fmaf(w.y, acc[4 * g4 + 2], acc[4 * g4 + 1])));
                };
                v2 p = vg(3);
#pragma unroll
                for (int g4 = 2; g4 >= 0; --g4) {
                    const v2 v = vg(g4);
                    p = mk(fmaf(p.x, w4.x, fmaf(-p.y, w4.y, v.x)), fmaf(p.x, w4.y, fmaf(p.y, w4.x, v.y)));
                }
                float t = fmaf(e.x, p.x, -e.y * p.y);
                t += __shfl_xor(t, 32, 64);
                if (half == c)
                    y[cg] += t * unscale;
            }
        }
    }

    // denominator and output: every lane writes its sample of each group
    double d2 = 0.0, r2 = 0.0;
#pragma unroll
    for (int cg = 0; cg < TF; ++cg) {
        const int n = tile_lo + 256 * cg + wave * 64 + col + 32 * half;
        const bool writer = n <= tile_hi;
        float xv = 0.f;
        if (writer) {
            const int flo = n - M > 0 ? (n - M + H - 1) / H : 0;
            const int fhi = (n + M) / H;
            float dv;
            if (n >= M && fhi <= nframes_all - 1) {
                dv = a.den[n % H];
            } else {
                dv = 0.f;
                const int hi = fhi < nframes_all - 1 ? fhi : nframes_all - 1;
                for (int m = flo; m <= hi; ++m)
                    dv += win[n - m * H + M].x;
                dv *= win[M].x;
            }
            xv = dv > 0.f ? y[cg] / dv : 0.f;
            float *out = a.xhat + (int64_t)q * a.n + n;
            if (a.accumulate)
                xv += *out;
            *out = xv;
        }
        if (a.err && writer && n >= M && n < a.n - M) {
            const double rv = a.xref[(int64_t)q * a.n + n];
            d2 += (rv - (double)xv) * (rv - (double)xv);
            r2 += rv * rv;
        }
    }
    if (a.err)
        err_reduce(d2, r2, a.err, q);
}

// Grouped wide inverse: the wide, one-block, decimated-table inverse with NG
// groups of 16 destinations of the tile's zones staged at once (2 or 4; more
// take further passes).  A step of 16 frames then
// reads each lane's window values (the B operand) once for all groups, the
// accumulators of all groups are live together (2 x 16 registers per group),
// and the phase sums of a sample column share its phasors.  Same arithmetic,
// term by term, as inv_kernel<true, true, kInvWideTF>: the same coefficients,
// splits, products and power-of-two scales per group.
template <int NG>
__device__ __forceinline__ bool wave_mfma_groups(f32x16 (&acc)[NG][2], const unsigned short *aph,
                                                 const unsigned short *apl, int gstride,
                                                 const unsigned *gpk, const WaveSteps &ws, int ng)
{
    const unsigned *pc0 = gpk + (ws.lane & 0xffff);
    const unsigned *pc1 = gpk + ((unsigned)ws.lane >> 16);
    auto step = [&](int k0, auto fresh) {
        constexpr bool FRESH = decltype(fresh)::value != 0;
        f16x8v fh[2], fl[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const unsigned *pc = c ? pc1 : pc0;
            unsigned w[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                w[i] = pc[7 - i];
            u4v_t bh, bl;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bh[i] = __builtin_amdgcn_perm(w[2 * i + 1], w[2 * i], 0x05040100u);
                bl[i] = __builtin_amdgcn_perm(w[2 * i + 1], w[2 * i], 0x07060302u);
            }
            fh[c] = __builtin_bit_cast(f16x8v, bh);
            fl[c] = __builtin_bit_cast(f16x8v, bl);
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (g >= ng)
                break;
            const u4v_t a_hi = *reinterpret_cast<const u4v_t *>(aph + g * gstride + k0);
            const u4v_t a_lo = *reinterpret_cast<const u4v_t *>(apl + g * gstride + k0);
            const f16x8v ah = __builtin_bit_cast(f16x8v, a_hi);
            const f16x8v al = __builtin_bit_cast(f16x8v, a_lo);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if constexpr (FRESH)
                    acc[g][c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, fh[c], f32x16{}, 0, 0, 0);
                else
                    acc[g][c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, fh[c], acc[g][c], 0, 0, 0);
                acc[g][c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, fl[c], acc[g][c], 0, 0, 0);
                acc[g][c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, fh[c], acc[g][c], 0, 0, 0);
            }
        }
        pc0 -= 16;
        pc1 -= 16;
    };
    int k0 = ws.kw & 0xffff;
    const int kw1 = (ws.kw >> 16) - 1;
    if (k0 > kw1)   // no frame reaches the wave's samples: the sums are zero
        return false;
    step(k0, IntC<1>{});
    for (k0 += 16; k0 <= kw1; k0 += 16)
        step(k0, IntC<0>{});
    return true;
}

template <int NG>
__global__ __launch_bounds__(256, NG >= 4 ? 2 : 3) void inv_kernel_g(InvLaunch l)
{
    constexpr int TF = kInvWideTF;
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t blk = l.blk_begin + (int64_t)blockIdx.x;
    const CA InvDesc *chs = (const CA InvDesc *)l.ch;
    const CA InvDesc &a = chs[inv_chan_of(chs, l.n_ch, blk)];
    const int nlo = 1 << a.lo_bits;
    const int nhi = (a.G + nlo - 1) >> a.lo_bits;
    const int KBP = inv_group_kbp(l.max_k);
    const int GS = 32 * KBP;   // halves per staged group
    const InvLds lay = inv_lds_layout(l.max_tab, l.max_gtab, l.max_k, KBP, NG);
    v2 *tlo = reinterpret_cast<v2 *>(smem);
    v2 *thi = tlo + nlo;
    unsigned *gpk = reinterpret_cast<unsigned *>(smem + lay.gpk);
    int *rid = reinterpret_cast<int *>(smem + lay.rid);
    unsigned short *ahi = reinterpret_cast<unsigned short *>(smem + lay.ahi);   // [NG][32][KBP]
    unsigned short *alo = reinterpret_cast<unsigned short *>(smem + lay.alo);   // [NG][32][KBP]
    float *fred = reinterpret_cast<float *>(smem + lay.fred);                   // [NG][4]
    int *red = reinterpret_cast<int *>(smem + lay.red);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 31, half = lane >> 5;
    const unsigned local = (unsigned)(blk - a.blk0);
    const unsigned tiles = (unsigned)a.tiles;
    const int q = (int)(local / tiles);
    const int span_lo = (int)a.span_lo, span_end = (int)(a.span_lo + a.span_len - 1);
    const int tile_lo = span_lo + (int)(local - (unsigned)q * tiles) * (kInvTile * TF);
    const int tile_hi = tile_lo + kInvTile * TF - 1 < span_end ? tile_lo + kInvTile * TF - 1 : span_end;
    const int M = a.M, H = a.hop, Gi = a.G;
    const uint32_t hinv = 0xffffffffu / (uint32_t)H;   // floor(2^32 / H) unless H is 1
    const int frame0 = (int)a.frame0, nfr = (int)a.nframes, nframes_all = (int)a.n_frames;
    const v2 *__restrict__ win = reinterpret_cast<const v2 *>(a.win);

#pragma unroll 2
    for (int e = threadIdx.x; e < nlo; e += 256)
        tlo[e] = reinterpret_cast<const v2 *>(a.ph_lo)[e];
#pragma unroll 2
    for (int e = threadIdx.x; e < nhi; e += 256)
        thi[e] = reinterpret_cast<const v2 *>(a.ph_hi)[e];
    // decimated window table, g[j] 2^tg as FP16 hi | lo << 16 (see inv_kernel)
    const float gsc = a.g_scale;
    const int JL = a.dec_reach;
    const int TR = a.dec_row;
    const int n_tab = H * TR;
#pragma unroll 4
    for (int e = threadIdx.x; e < n_tab; e += 256) {
        const int r = e / TR;
        const int j = r + (e - r * TR) * H - JL;
        unsigned w = 0u;
        if (j >= -M && j <= M) {
            unsigned h, lw;
            split_f16(win[j + M].x * gsc, h, lw);
            w = h | (lw << 16);
        }
        gpk[e] = w;
    }

    int mlo = tile_lo - M > 0 ? (tile_lo - M + H - 1) / H : 0;
    int mhi = (tile_hi + M) / H;
    if (mlo < frame0)
        mlo = frame0;
    if (mhi > frame0 + nfr - 1)
        mhi = frame0 + nfr - 1;
    const int K = mhi >= mlo ? mhi - mlo + 1 : 0;
    const int32_t *__restrict__ ridge = a.ridge + (int64_t)q * a.nframes + (mlo - frame0);
    for (int k = threadIdx.x; k < K; k += 256)
        rid[k] = ridge[k];
    if (threadIdx.x < 2)
        red[threadIdx.x] = threadIdx.x == 0 ? 0x7fffffff : -1;
    __syncthreads();
    {
        int dmin = 0x7fffffff, dmax = -1;
        for (int k = threadIdx.x; k < K; k += 256) {
            const int r = rid[k];
            if (r >= 0) {
                dmin = min(dmin, max(r - a.hw, 0));
                dmax = max(dmax, min(r + a.hw, a.n_dst - 1));
            }
        }
        if (dmax >= 0) {
            atomicMin(&red[0], dmin);
            atomicMax(&red[1], dmax);
        }
    }
    __syncthreads();
    const int d_lo = red[0], d_hi = red[1];
    const int zk1 = a.z * a.k1;
    const uint32_t G = (uint32_t)Gi;
    const bool pow2 = a.g_pow2 != 0;
    const uint32_t mh0 = (uint32_t)(mlo * H) % G;
    const uint32_t n0g = (uint32_t)tile_lo % G;
    const uint32_t hg = (uint32_t)H % G;
    const int kn16 = (K + 15) & ~15;
    const int nrd = kn16 / 16;   // rounds of 256 staged coefficients (16 frames)
    constexpr int STAGE = kInvWideKB * 16 / 256;

    const v2 *__restrict__ Trow = reinterpret_cast<const v2 *>(a.T) + (int64_t)(mlo - frame0) * a.n_dst;
    const unsigned short *aph = ahi + col * KBP + 8 * half;
    const unsigned short *apl = alo + col * KBP + 8 * half;
    float y[TF][2];
#pragma unroll
    for (int cg = 0; cg < TF; ++cg)
        y[cg][0] = y[cg][1] = 0.f;
    for (int D0 = d_lo; D0 <= d_hi; D0 += 16 * NG) {
        const int ng = (d_hi - D0) / 16 + 1 < NG ? (d_hi - D0) / 16 + 1 : NG;
        int scg[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            scg[g] = 0;
            if (g >= ng)
                break;
            const int d0 = D0 + 16 * g;
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            float cre[STAGE], cim[STAGE];
            float amax = 0.f;
#pragma unroll
            for (int i = 0; i < STAGE; ++i) {
                cre[i] = cim[i] = 0.f;
                if (i >= nrd)
                    continue;
                const int e = tid + 256 * i;
                const int kk = e >> 4, dd = e & 15;
                const int ld = d0 + dd;
                v2 c = mk(0.f, 0.f);
                const int r = kk < K ? rid[kk] : -1;
                if (r >= 0 && ld <= d_hi && ld >= r - a.hw && ld <= r + a.hw) {
                    const int b = zk1 + ld;
                    const float wgt = (b == 0 || 2 * b == Gi) ? 1.f : 2.f;
                    const v2 t = Trow[(int64_t)kk * a.n_dst + ld];
                    uint32_t mh = mh0 + (uint32_t)kk * hg;
                    mh = pow2 ? (mh & (G - 1)) : mh % G;
                    const int bm = mulmod((uint32_t)b, mh, Gi, a.g_pow2, a.inv_G);
                    const v2 ph = phasor(tlo, thi, bm, a.lo_bits);   // e^{+i 2 pi b m H / G}
                    c = (wgt * a.inv_nfft) * cmul(t, conjv(ph));
                }
                cre[i] = c.x;
                cim[i] = c.y;
                amax = fmaxf(amax, fmaxf(fabsf(c.x), fabsf(c.y)));
            }
            amax = wave_reduce63(amax, 0.f, [](float p, float r) { return fmaxf(p, r); });
            if (lane == 63)
                fred[4 * g + wave] = amax;
            __syncthreads();
            const float bmax = fmaxf(fmaxf(fred[4 * g], fred[4 * g + 1]),
                                     fmaxf(fred[4 * g + 2], fred[4 * g + 3]));
            int ex = 0;
            (void)frexpf(bmax, &ex);
            int sb = 14 - ex;
            sb = sb > 100 ? 100 : (sb < -100 ? -100 : sb);
            scg[g] = sb;
            const float scl = ldexpf(1.f, sb);
            unsigned short *gh = ahi + g * GS, *gl = alo + g * GS;
#pragma unroll
            for (int i = 0; i < STAGE; ++i) {
                const int e = tid + 256 * i;
                const int kk = e >> 4, dd = e & 15;
                if (i < nrd) {
                    unsigned h, lw;
                    split_f16(cre[i] * scl, h, lw);
                    gh[(2 * dd) * KBP + kk] = (unsigned short)h;
                    gl[(2 * dd) * KBP + kk] = (unsigned short)lw;
                    split_f16(cim[i] * scl, h, lw);
                    gh[(2 * dd + 1) * KBP + kk] = (unsigned short)h;
                    gl[(2 * dd + 1) * KBP + kk] = (unsigned short)lw;
                }
            }
        }
        __syncthreads();   // every staged group complete
        // one sample group at a time (not unrolled: the accumulators of all
        // groups are live through it), its sums added into y by selection
#pragma unroll 1
        for (int cg = 0; cg < TF; ++cg) {
            f32x16 acc[NG][2];
            const WaveSteps ws =
                wave_steps<true>(tile_lo, cg, wave, col, half, mlo, 0, K, M, H, JL, TR, hinv);
            if (!wave_mfma_groups<NG>(acc, aph, apl, GS, gpk, ws, ng))
                continue;   // no frame reaches these samples
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                uint32_t nm = n0g + (uint32_t)(256 * cg + 64 * wave + col + 32 * c);
                nm = nm >= G ? nm - G : nm;
                nm = nm >= G ? nm - G : nm;
                const v2 w = phasor(tlo, thi, (int)nm, a.lo_bits);   // e^{i 2 pi n/G}
                const v2 w2 = cmul(w, w), w4 = cmul(w2, w2);
                float tsum = 0.f;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    if (g >= ng)
                        break;
                    const uint32_t bb = (uint32_t)(zk1 + D0 + 16 * g + 2 * half);
                    const v2 e = phasor(tlo, thi, mulmod(bb, nm, Gi, a.g_pow2, a.inv_G), a.lo_bits);
                    // Re(e P), P = sum_g4 w4^g4 (Z_(g4,0) + w Z_(g4,1)), as in inv_kernel
                    const f32x16 &z = acc[g][c];
                    auto vg = [&](int g4) {
                        return mk(fmaf(w.x, z[4 * g4 + 2], fmaf(-w.y, z[4 * g4 + 3], z[4 * g4])),
                                  fmaf(w.x, z[4 * g4 + 3], fmaf(w.y, z[4 * g4 + 2], z[4 * g4 + 1])));
                    };
                    v2 pp = vg(3);
#pragma unroll
                    for (int g4 = 2; g4 >= 0; --g4) {
                        const v2 v = vg(g4);
                        pp = mk(fmaf(pp.x, w4.x, fmaf(-pp.y, w4.y, v.x)),
                                fmaf(pp.x, w4.y, fmaf(pp.y, w4.x, v.y)));
                    }
                    const float t = fmaf(e.x, pp.x, -e.y * pp.y);
                    tsum += t * ldexpf(a.g_unscale, -scg[g]);
                }
                tsum += __shfl_xor(tsum, 32, 64);
#pragma unroll
                for (int k = 0; k < TF; ++k)
                    y[k][c] += k == cg ? tsum : 0.f;
            }
        }
        __syncthreads();   // staged groups consumed before the next pass
    }

    double d2 = 0.0, r2 = 0.0;
#pragma unroll
    for (int cg = 0; cg < TF; ++cg)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int n = tile_lo + 256 * cg + wave * 64 + col + 32 * c;
        const bool writer = half == 0 && n <= tile_hi;
        float xv = 0.f;
        if (writer) {
            const int flo = n - M > 0 ? (n - M + H - 1) / H : 0;
            const int fhi = (n + M) / H;
            float dv;
            if (n >= M && fhi <= nframes_all - 1) {
                dv = a.den[n % H];
            } else {
                dv = 0.f;
                const int hi = fhi < nframes_all - 1 ? fhi : nframes_all - 1;
                for (int m = flo; m <= hi; ++m)
                    dv += win[n - m * H + M].x;
                dv *= win[M].x;
            }
            xv = dv > 0.f ? y[cg][c] / dv : 0.f;
            float *out = a.xhat + (int64_t)q * a.n + n;
            if (a.accumulate)
                xv += *out;
            *out = xv;
        }
        if (a.err && writer && n >= M && n < a.n - M) {
            const double rv = a.xref[(int64_t)q * a.n + n];
            d2 += (rv - (double)xv) * (rv - (double)xv);
            r2 += rv * rv;
        }
    }
    if (a.err)
        err_reduce(d2, r2, a.err, q);
}

// Clear the error sums of every channel of an inverse launch.
__global__ __launch_bounds__(256) void clear_err_kernel(InvLaunch l)
{
    const int c = blockIdx.x;
    if (c >= l.n_ch || !l.ch[c].err)
        return;
    for (int i = threadIdx.x; i < 2 * l.ch[c].n_comp; i += 256)
        l.ch[c].err[i] = 0.0;
}

__global__ __launch_bounds__(64) void put_inv_desc_kernel(InvDesc d, InvDesc *dst)
{
    if (threadIdx.x == 0)
        *dst = d;
}

// Eq. 15 (hop 1): xhat[m] = (1/(N_f g[0])) sum_zone a_l Re T[m,l].
__global__ __launch_bounds__(256) void eq15_kernel(const InvDesc *dp, float scale)
{
    const CA InvDesc &a = *(const CA InvDesc *)dp;
    const int q = blockIdx.y;
    const int64_t mloc = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = mloc < a.nframes;
    const v2 *__restrict__ T = reinterpret_cast<const v2 *>(a.T);
    float xv = 0.f;
    int64_t n = a.frame0 + mloc;
    if (valid) {
        const int r = a.ridge[(int64_t)q * a.nframes + mloc];
        float acc = 0.f;
        if (r >= 0) {
            const int la = r - a.hw < 0 ? 0 : r - a.hw;
            const int lb = r + a.hw > a.n_dst - 1 ? a.n_dst - 1 : r + a.hw;
            for (int l = la; l <= lb; ++l) {
                const int b = a.z * a.k1 + l;
                acc += ((b == 0 || 2 * b == a.G) ? 1.f : 2.f) * T[mloc * a.n_dst + l].x;
            }
        }
        xv = acc * scale;
        float *out = a.xhat + (int64_t)q * a.n + n;
        if (a.accumulate)
            xv += *out;
        *out = xv;
    }
    if (a.err) {
        double d2 = 0.0, r2 = 0.0;
        if (valid && n >= a.M && n < a.n - a.M) {
            const double rv = a.xref[(int64_t)q * a.n + n];
            d2 = (rv - (double)xv) * (rv - (double)xv);
            r2 = rv * rv;
        }
        err_reduce(d2, r2, a.err, q);
    }
}

__global__ void zero_f64(double *p, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Ridge: a 16-lane row per (frame, component).
// ---------------------------------------------------------------------------

// 64-bit key max over the 16 lanes of each DPP row (rotations by 1, 2, 4, 8);
// every lane of the row ends with the row's maximum.
__device__ __forceinline__ unsigned long long row_max_u64(unsigned long long k)
{
#define SST_ROW_STEP(CTRL)                                                                    \
    {                                                                                         \
        const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)k, CTRL,  \
                                                                  0xf, 0xf, false);           \
        const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(k >> 32), \
                                                                  CTRL, 0xf, 0xf, false);     \
        const unsigned long long o = ((unsigned long long)hi << 32) | lo;                     \
        k = o > k ? o : k;                                                                    \
    }
    SST_ROW_STEP(0x121)
    SST_ROW_STEP(0x122)
    SST_ROW_STEP(0x124)
    SST_ROW_STEP(0x128)
#undef SST_ROW_STEP
    return k;
}

// Ridge of component q (Sec. 2.2, zone M_q[m]): per frame, the destination of
// largest |T|^2 in [lo, hi], ties to the smallest l, -1 when all are zero.
// A 16-lane row per frame (lanes across the band), four frames per wave, four
// passes per workgroup (64 frames); the key (|T|^2 bits, ~l) orders by
// magnitude, then by smallest l.
constexpr int kRidgeFrames = 64;   // frames per workgroup

__global__ __launch_bounds__(256) void ridge_kernel(RidgeArgs a)
{
    const int q = blockIdx.y;
    const int sub = threadIdx.x & 15;
    const int64_t m0 = (int64_t)blockIdx.x * kRidgeFrames + (threadIdx.x >> 4);
    unsigned long long key[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int64_t m = m0 + 16 * p;
        key[p] = 0ull;
        // the band, relative to the frame's guide bin when one is given
        int lo = a.band[2 * q], hi = a.band[2 * q + 1];
        int ctr = 0;
        bool none = false;
        if (a.centre && m < a.nframes) {
            ctr = a.centre[(int64_t)q * a.nframes + m];
            none = ctr < 0;   // no guide: no ridge in this frame
        }
        lo = lo + ctr < 0 ? 0 : lo + ctr;
        hi = hi + ctr > a.n_dst - 1 ? a.n_dst - 1 : hi + ctr;
        if (none)
            hi = -1;
        if (m < a.nframes) {
            const v2 *__restrict__ row = reinterpret_cast<const v2 *>(a.T) + m * a.n_dst;
            for (int l = lo + sub; l <= hi; l += 16) {
                const v2 v = row[l];
                const float m2 = v.x * v.x + v.y * v.y;
                const unsigned long long k =
                    ((unsigned long long)__float_as_uint(m2) << 32) | (unsigned)~l;
                key[p] = k > key[p] ? k : key[p];
            }
        }
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const unsigned long long k = row_max_u64(key[p]);
        const int64_t m = m0 + 16 * p;
        if (sub == 0 && m < a.nframes)
            a.ridge[(int64_t)q * a.nframes + m] = (k >> 32) != 0ull ? (int)~(unsigned)k : -1;
    }
}

// Non-zero input rows of pass 1 for window length L: 4, 8 or 16.
template <int NF>
int nz_rows(int L)
{
    const int rows = (L + NF / 16 - 1) / (NF / 16);
    return rows <= 4 ? 4 : (rows <= 8 ? 8 : 16);
}

template <int NF, int NZ, bool MULTI>
hipError_t launch_fwd_nzm(int max_n_src, int max_n_dst, int kind, const GroupLaunch &gl,
                          int grid, hipStream_t s)
{
    const dim3 g(grid), b(Geo<NF>::NT);
    const bool chunked = (int64_t)Geo<NF>::F * max_n_dst > Geo<NF>::LDS;
    const bool debug = kind == kFwdKindDebug;
    if constexpr (!MULTI) {
        if (kind == kFwdKindStats) {
            // the per-frame sums: the general variant (any row length, nine
            // rounds, same rows bit for bit) with the epilogue compiled in
            if (gl.list)
                hipLaunchKernelGGL((fwd_kernel<NF, NZ, 9, false, true, false, kFwdFixup, true>), g,
                                   b, 0, s, gl);
            else
                hipLaunchKernelGGL((fwd_kernel<NF, NZ, 9, false, true, false, kFwdPlain, true>), g,
                                   b, 0, s, gl);
            return hipGetLastError();
        }
    }
    if (gl.list) {
        // fix-up pass: the general variant (any row length, nine rounds) gives
        // every row bit for bit what the variant chosen below gives
        hipLaunchKernelGGL((fwd_kernel<NF, NZ, 9, false, true, MULTI, kFwdFixup>), g, b, 0, s, gl);
    } else if (debug) {
        hipLaunchKernelGGL((fwd_kernel<NF, NZ, 9, true, true, MULTI>), g, b, 0, s, gl);
    } else if (chunked) {
        // rows longer than the buffer; fewer rounds where they suffice keep
        // the register count within the four-waves-per-SIMD budget
        if (NF >= 4096 && fwd_rounds(NF, max_n_src) <= 5)
            hipLaunchKernelGGL((fwd_kernel<NF, NZ, (NF >= 4096 ? 5 : 9), false, true, MULTI>), g, b,
                               0, s, gl);
        else
            hipLaunchKernelGGL((fwd_kernel<NF, NZ, 9, false, true, MULTI>), g, b, 0, s, gl);
    } else {
        switch (fwd_rounds(NF, max_n_src)) {
        case 3: hipLaunchKernelGGL((fwd_kernel<NF, NZ, 3, false, false, MULTI>), g, b, 0, s, gl); break;
        case 5: hipLaunchKernelGGL((fwd_kernel<NF, NZ, 5, false, false, MULTI>), g, b, 0, s, gl); break;
        default: hipLaunchKernelGGL((fwd_kernel<NF, NZ, 9, false, false, MULTI>), g, b, 0, s, gl); break;
        }
    }
    return hipGetLastError();
}

template <int NF, int NZ>
hipError_t launch_fwd_nz(int max_n_src, int max_n_dst, int kind, const GroupLaunch &gl,
                         int grid, hipStream_t s)
{
    return gl.n_ch > 1 ? launch_fwd_nzm<NF, NZ, true>(max_n_src, max_n_dst, kind, gl, grid, s)
                       : launch_fwd_nzm<NF, NZ, false>(max_n_src, max_n_dst, kind, gl, grid, s);
}

template <int NF>
hipError_t launch_fwd_t(int max_L, int max_n_src, int max_n_dst, int kind, const GroupLaunch &gl,
                        int grid, hipStream_t s)
{
    switch (nz_rows<NF>(max_L)) {
    case 4: return launch_fwd_nz<NF, 4>(max_n_src, max_n_dst, kind, gl, grid, s);
    case 8: return launch_fwd_nz<NF, 8>(max_n_src, max_n_dst, kind, gl, grid, s);
    default: return launch_fwd_nz<NF, 16>(max_n_src, max_n_dst, kind, gl, grid, s);
    }
}

template <int NF, int NZ>
hipError_t launch_maxonly_nz(const GroupLaunch &gl, int grid, hipStream_t s)
{
    const dim3 g(grid), b(Geo<NF>::NT);
    if (gl.n_ch > 1)
        hipLaunchKernelGGL((fwd_kernel<NF, NZ, 3, false, false, true, kFwdMaxOnly>), g, b, 0, s, gl);
    else
        hipLaunchKernelGGL((fwd_kernel<NF, NZ, 3, false, false, false, kFwdMaxOnly>), g, b, 0, s, gl);
    return hipGetLastError();
}

template <int NF, int NZ>
hipError_t launch_stft_nz(const GroupLaunch &gl, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((fwd_kernel<NF, NZ, 3, false, false, false, kFwdStft>), dim3(grid),
                       dim3(Geo<NF>::NT), 0, s, gl);
    return hipGetLastError();
}

template <int NF>
hipError_t launch_stft_t(int L, const GroupLaunch &gl, int grid, hipStream_t s)
{
    switch (nz_rows<NF>(L)) {
    case 4: return launch_stft_nz<NF, 4>(gl, grid, s);
    case 8: return launch_stft_nz<NF, 8>(gl, grid, s);
    default: return launch_stft_nz<NF, 16>(gl, grid, s);
    }
}

template <int NF>
hipError_t launch_maxonly_t(int L, const GroupLaunch &gl, int grid, hipStream_t s)
{
    switch (nz_rows<NF>(L)) {
    case 4: return launch_maxonly_nz<NF, 4>(gl, grid, s);
    case 8: return launch_maxonly_nz<NF, 8>(gl, grid, s);
    default: return launch_maxonly_nz<NF, 16>(gl, grid, s);
    }
}

template <typename K>
int occ_of(K kernel, int threads, size_t dyn = 0)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, dyn) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <int NF>
int occ_fwd_t(int L)
{
    // every variant of one N_f and NZ has the same LDS and launch bounds
    switch (nz_rows<NF>(L)) {
    case 4: return occ_of(fwd_kernel<NF, 4, 9, false, true, true>, Geo<NF>::NT);
    case 8: return occ_of(fwd_kernel<NF, 8, 9, false, true, true>, Geo<NF>::NT);
    default: return occ_of(fwd_kernel<NF, 16, 9, false, true, true>, Geo<NF>::NT);
    }
}

}  // namespace

int fwd_rounds(int nfft, int n_src)
{
    const int F = nfft >= 4096 ? 1 : 4096 / nfft;
    const int NT = nfft > 4096 ? nfft / 16 : 256;
    const int need = (F * n_src + NT - 1) / NT;
    return need <= 3 ? 3 : (need <= 5 ? 5 : 9);
}

#define SST_DISPATCH_NF(nfft, EXPR)                 \
    switch (nfft) {                                 \
    case 512: { constexpr int NFv = 512; EXPR; }    \
    case 1024: { constexpr int NFv = 1024; EXPR; }  \
    case 2048: { constexpr int NFv = 2048; EXPR; }  \
    case 4096: { constexpr int NFv = 4096; EXPR; }  \
    case 8192: { constexpr int NFv = 8192; EXPR; }  \
    default: break;                                 \
    }

hipError_t launch_clear_max(const GroupLaunch &g, hipStream_t s)
{
    const unsigned cb = (unsigned)((g.n_ch + 255) / 256);
    hipLaunchKernelGGL(clear_max_kernel, dim3(cb), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_max_prepass(int nfft, int L, const GroupLaunch &g, int grid, hipStream_t s)
{
    if (g.item_stop <= g.item_begin || grid <= 0)
        return hipSuccess;
    SST_DISPATCH_NF(nfft, return launch_maxonly_t<NFv>(L, g, grid, s))
    return hipErrorInvalidValue;
}

hipError_t launch_stft(int nfft, int L, const GroupLaunch &g, int grid, hipStream_t s)
{
    if (g.item_stop <= g.item_begin || grid <= 0)
        return hipSuccess;
    SST_DISPATCH_NF(nfft, return launch_stft_t<NFv>(L, g, grid, s))
    return hipErrorInvalidValue;
}

hipError_t launch_synthesis(int nfft, const SynArgs &a, hipStream_t s)
{
    const int64_t tiles = (a.n + kSynTile - 1) / kSynTile;
    if (tiles <= 0)
        return hipSuccess;
    SST_DISPATCH_NF(nfft, {
        hipLaunchKernelGGL(syn_kernel<NFv>, dim3((unsigned)tiles), dim3(Geo<NFv>::NT), 0, s, a);
        return hipGetLastError();
    })
    return hipErrorInvalidValue;
}

hipError_t launch_gamma(const GroupLaunch &g, hipStream_t s)
{
    const unsigned cb = (unsigned)((g.n_ch + 255) / 256);
    hipLaunchKernelGGL(gamma_kernel, dim3(cb), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_spec_list(const GroupLaunch &g, hipStream_t s)
{
    // at least one workgroup: workgroup 0 sets gamma
    const int64_t items = g.item_stop > g.item_begin ? g.item_stop - g.item_begin : 0;
    const int64_t blocks = items > 0 ? (items + 255) / 256 : 1;
    hipLaunchKernelGGL(spec_list_kernel, dim3((unsigned)(blocks < 1024 ? blocks : 1024)),
                       dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_forward(int nfft, int max_L, int max_n_src, int max_n_dst, int kind,
                          const GroupLaunch &g, int grid, hipStream_t s)
{
    SST_DISPATCH_NF(nfft, return launch_fwd_t<NFv>(max_L, max_n_src, max_n_dst, kind, g, grid, s))
    return hipErrorInvalidValue;
}

hipError_t launch_put_desc(const ChanDesc &d, ChanDesc *dst, bool clear_max, int32_t *list_n,
                           hipStream_t s)
{
    hipLaunchKernelGGL(put_desc_kernel, dim3(1), dim3(64), 0, s, d, dst, clear_max ? 1 : 0, list_n);
    return hipGetLastError();
}

size_t inv_lds_bytes(const InvLaunch &l)
{
    if (l.groups > 1)
        return inv_lds_layout(l.max_tab, l.max_gtab, l.max_k, inv_group_kbp(l.max_k), l.groups)
            .total;
    const int kbp = l.tf > 1 ? InvGeo<kInvWideTF>::KBP : InvGeo<1>::KBP;
    return inv_lds_layout(l.max_tab, l.max_gtab, l.max_k, kbp).total;
}

hipError_t launch_inverse(const InvLaunch &l, int64_t blocks, bool clear_err, hipStream_t s)
{
    if (clear_err) {
        hipLaunchKernelGGL(clear_err_kernel, dim3((unsigned)l.n_ch), dim3(256), 0, s, l);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (blocks <= 0)
        return hipSuccess;
    const size_t lds = inv_lds_bytes(l);
    const dim3 g((unsigned)blocks), b(256);
    if (l.tf > 1) {
        // the host sets tf > 1 only when every tile's frames fit one block
        if (l.max_k > InvGeo<kInvWideTF>::KB)
            return hipErrorInvalidValue;
        if (l.tf == kInvXWideTF) {
            if (!l.dec || l.groups > 1)
                return hipErrorInvalidValue;
            hipLaunchKernelGGL((inv_kernel<true, true, kInvXWideTF>), g, b, lds, s, l);
        } else if (l.groups == 4 && l.dec)
            hipLaunchKernelGGL((inv_kernel_g<4>), g, b, lds, s, l);
        else if (l.groups == 2 && l.dec)
            hipLaunchKernelGGL((inv_kernel_g<2>), g, b, lds, s, l);
        else if (l.dec)
            hipLaunchKernelGGL((inv_kernel<true, true, kInvWideTF>), g, b, lds, s, l);
        else
            hipLaunchKernelGGL((inv_kernel<true, false, kInvWideTF>), g, b, lds, s, l);
    } else if (l.max_k <= InvGeo<1>::KB && l.dec) {
        hipLaunchKernelGGL((inv_kernel<true, true, 1>), g, b, lds, s, l);
    } else if (l.max_k <= InvGeo<1>::KB) {
        hipLaunchKernelGGL((inv_kernel<true, false, 1>), g, b, lds, s, l);
    } else if (l.dec) {
        hipLaunchKernelGGL((inv_kernel<false, true, 1>), g, b, lds, s, l);
    } else {
        hipLaunchKernelGGL((inv_kernel<false, false, 1>), g, b, lds, s, l);
    }
    return hipGetLastError();
}

hipError_t launch_inverse_eq15(const InvDesc &a, const InvDesc *dev, float scale, hipStream_t s)
{
    if (a.err) {
        hipLaunchKernelGGL(zero_f64, dim3((2 * a.n_comp + 63) / 64), dim3(64), 0, s, a.err,
                           2 * a.n_comp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    const int64_t blocks = (a.nframes + 255) / 256;
    hipLaunchKernelGGL(eq15_kernel, dim3((unsigned)blocks, a.n_comp), dim3(256), 0, s, dev, scale);
    return hipGetLastError();
}

hipError_t launch_put_inv_desc(const InvDesc &d, InvDesc *dst, hipStream_t s)
{
    hipLaunchKernelGGL(put_inv_desc_kernel, dim3(1), dim3(64), 0, s, d, dst);
    return hipGetLastError();
}

hipError_t launch_ridge(const RidgeArgs &a, hipStream_t s)
{
    const int64_t blocks = (a.nframes + kRidgeFrames - 1) / kRidgeFrames;
    hipLaunchKernelGGL(ridge_kernel, dim3((unsigned)blocks, a.n_comp), dim3(256), 0, s, a);
    return hipGetLastError();
}

int fwd_frames_per_iter(int nfft)
{
    SST_DISPATCH_NF(nfft, return Geo<NFv>::F)
    return 0;
}
int fwd_threads(int nfft)
{
    SST_DISPATCH_NF(nfft, return Geo<NFv>::NT)
    return 0;
}
int fwd_lds_elems(int nfft)
{
    SST_DISPATCH_NF(nfft, return Geo<NFv>::LDS)
    return 0;
}
template <int NF>
size_t fwd_static_lds_t()
{
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, reinterpret_cast<const void *>(&fwd_kernel<NF, 16, 9, true, true, true>)) !=
        hipSuccess)
        return 0;
    return at.sharedSizeBytes;
}

size_t fwd_lds_bytes(int nfft)
{
    SST_DISPATCH_NF(nfft, return fwd_static_lds_t<NFv>())
    return 0;
}

int fwd_occupancy(int nfft, int L)
{
    SST_DISPATCH_NF(nfft, return occ_fwd_t<NFv>(L))
    return 1;
}
// ---------------------------------------------------------------------------
// Fixed device scratch for callers that cannot allocate (sst_forward_static).
// Each device holds its own copy of the array for the life of the process.
// Host code never passes `scratch` itself to a kernel: its host-side name is a
// stand-in, not a device address.  The device address is looked up once per
// device, with that device current, and cached.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(int dev, unsigned char **out)
{
    static std::mutex mu;
    static unsigned char *ptr[kMaxDevices] = {};
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

}  // namespace sst
