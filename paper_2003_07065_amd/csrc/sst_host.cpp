// Host runtime of the gfx950 downsampled SST library: parameter validation,
// float64 table generation, workspace layout and the C-ABI entry points
// declared in include/sst.h.
//
// Method: He & Cao, arXiv 2003.07065.  Tables built here:
//   - g, g' sampled on [-M, M] (Sec. 2.1; Sec. 2.2), with g' pre-scaled by
//     s = ||g|| / ||g'|| for the packed FFT pair;
//   - the centre phase exp(+i 2 pi ((k M) mod N_f) / N_f) of Eq. 9, the exponent
//     reduced exactly in integers before the float64 sin/cos;
//   - FFT twiddles exp(-i 2 pi r / N_f);
//   - the inverse phase grid exp(+i 2 pi r / (z N_f)) of Eq. 25 on the
//     subdivided grid (Sec. 2.5), split into a low and a high table so that
//     exp(i 2 pi r / G) = hi[r >> b] * lo[r & (2^b - 1)].
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sst.h"
#include "sst_internal.h"

namespace {

thread_local std::string g_err;

sst_status fail(sst_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

sst_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return SST_E_DEVICE;
}

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr size_t kAlign = 256;
constexpr int kMaxPartials = 8192;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int64_t mod_exact(int64_t a, int64_t m)
{
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

}  // namespace

struct sst_plan_s {
    sst_params p{};
    int M = 0, k1 = 0, k2 = 0, n_src = 0, n_dst = 0;
    int64_t n_frames = 0;
    double s_pack = 1.0;
    double g0 = 0.0;
    int G = 0, lo_bits = 0, n_lo = 0, n_hi = 0;
    // workspace layout (bytes)
    size_t off_win = 0, off_cph = 0, off_twid = 0, off_phlo = 0, off_phhi = 0;
    size_t tables_end = 0, off_part = 0, ws_bytes = 0;
    std::vector<unsigned char> blob;   // host image of [off_win, tables_end)
    // bound state
    unsigned char *ws = nullptr;
    int device = -1;
    int cus = 0;
    int fwd_grid_cap = 0;
    int max_grid_cap = 0;
};

namespace {

sst_status validate(const sst_params *p)
{
    if (!p)
        return fail(SST_E_ARG, "params is NULL");
    if (p->struct_size < sizeof(sst_params))
        return fail(SST_E_ARG, "params.struct_size smaller than sizeof(sst_params)");
    if (p->n_samples < 1)
        return fail(SST_E_ARG, "n_samples must be >= 1");
    if (!(p->fs > 0.0) || !std::isfinite(p->fs))
        return fail(SST_E_ARG, "fs must be finite and > 0");
    if (p->win_len < 1 || (p->win_len % 2) == 0)
        return fail(SST_E_ARG, "win_len must be odd and >= 1");
    if ((p->window == nullptr) != (p->dwindow == nullptr))
        return fail(SST_E_ARG, "window and dwindow must be given together");
    if (!p->window && (!(p->sigma > 0.0) || !std::isfinite(p->sigma)))
        return fail(SST_E_ARG, "sigma must be finite and > 0");
    if (p->hop < 1)
        return fail(SST_E_ARG, "hop must be >= 1");
    if (!is_pow2(p->nfft))
        return fail(SST_E_ARG, "nfft must be a power of two");
    if (p->nfft < 512 || p->nfft > 8192)
        return fail(SST_E_UNSUPPORTED, "nfft must lie in [512, 8192]");
    if (p->win_len > p->nfft)
        return fail(SST_E_ARG, "win_len must not exceed nfft");
    if (!(p->f_lo >= 0.0) || !(p->f_hi > p->f_lo) || !(p->f_hi <= 0.5 * p->fs))
        return fail(SST_E_ARG, "band must satisfy 0 <= f_lo < f_hi <= fs/2");
    if (p->subdiv < 1 || (int64_t)p->subdiv * p->nfft > (1 << 20))
        return fail(SST_E_ARG, "subdiv must be >= 1 with subdiv * nfft <= 2^20");
    if (p->thr_mode != SST_THR_ABS && p->thr_mode != SST_THR_REL_MAX)
        return fail(SST_E_ARG, "thr_mode must be SST_THR_ABS or SST_THR_REL_MAX");
    if (!(p->thr >= 0.0) || !std::isfinite(p->thr))
        return fail(SST_E_ARG, "thr must be finite and >= 0");
    if (p->precision != SST_PREC_FP32_FFT)
        return fail(SST_E_UNSUPPORTED, "only SST_PREC_FP32_FFT is built");
    if (p->flags != 0)
        return fail(SST_E_ARG, "params.flags must be 0");
    return SST_OK;
}

}  // namespace

extern "C" {

sst_status sst_plan(const sst_params *params, sst_plan_t *out)
{
    if (!out)
        return fail(SST_E_ARG, "out is NULL");
    *out = nullptr;
    sst_status st = validate(params);
    if (st != SST_OK)
        return st;
    sst_plan_s *pl = new (std::nothrow) sst_plan_s();
    if (!pl)
        return fail(SST_E_NOMEM, "plan allocation failed");
    pl->p = *params;
    pl->p.window = nullptr;
    pl->p.dwindow = nullptr;
    const sst_params &p = *params;
    const int L = p.win_len, NF = p.nfft, z = p.subdiv;
    pl->M = (L - 1) / 2;
    pl->n_frames = (p.n_samples + p.hop - 1) / p.hop;

    // Band of interest snapped outward to source bins (Sec. 2.4, Eqs. 27-29).
    const double df = p.fs / NF;
    int k1 = (int)std::floor(p.f_lo / df + 1e-9);
    int k2 = (int)std::ceil(p.f_hi / df - 1e-9);
    if (k2 > NF / 2)
        k2 = NF / 2;
    if (k1 < 0 || k1 >= k2) {
        delete pl;
        return fail(SST_E_ARG, "band covers no source bin interval");
    }
    pl->k1 = k1;
    pl->k2 = k2;
    pl->n_src = k2 - k1 + 1;
    pl->n_dst = z * (k2 - k1) + 1;

    // Windows (Sec. 2.1: g; Sec. 2.2: g').
    std::vector<double> g(L), gd(L);
    if (p.window) {
        for (int i = 0; i < L; ++i) {
            g[i] = p.window[i];
            gd[i] = p.dwindow[i];
            if (!std::isfinite(g[i]) || !std::isfinite(gd[i])) {
                delete pl;
                return fail(SST_E_ARG, "window values must be finite");
            }
        }
    } else {
        const double amp = std::pow(M_PI * p.sigma * p.sigma, -0.25);
        for (int j = -pl->M; j <= pl->M; ++j) {
            const double t = (double)j;
            g[j + pl->M] = amp * std::exp(-t * t / (2.0 * p.sigma * p.sigma));
            gd[j + pl->M] = -(t / (p.sigma * p.sigma)) * g[j + pl->M];
        }
    }
    double eg = 0.0, egd = 0.0;
    for (int i = 0; i < L; ++i) {
        eg += g[i] * g[i];
        egd += gd[i] * gd[i];
    }
    if (!(eg > 0.0)) {
        delete pl;
        return fail(SST_E_ARG, "window has zero energy");
    }
    pl->s_pack = egd > 0.0 ? std::sqrt(eg / egd) : 1.0;
    pl->g0 = g[pl->M];

    // Inverse phase grid on z N_f points (Sec. 2.5, last paragraph).
    pl->G = z * NF;
    int bits = 0;
    while ((1LL << bits) < pl->G)
        ++bits;
    pl->lo_bits = (bits + 1) / 2;
    pl->n_lo = 1 << pl->lo_bits;
    pl->n_hi = (pl->G + pl->n_lo - 1) >> pl->lo_bits;

    // Workspace layout.
    size_t off = align_up(sizeof(sst::Ctrl));
    pl->off_win = off;
    off = align_up(off + sizeof(float) * 2 * (size_t)L);
    pl->off_cph = off;
    off = align_up(off + sizeof(float) * 2 * (size_t)pl->n_src);
    pl->off_twid = off;
    off = align_up(off + sizeof(float) * 2 * (size_t)NF);
    pl->off_phlo = off;
    off = align_up(off + sizeof(float) * 2 * (size_t)pl->n_lo);
    pl->off_phhi = off;
    off = align_up(off + sizeof(float) * 2 * (size_t)pl->n_hi);
    pl->tables_end = off;
    pl->off_part = off;
    off = align_up(off + sizeof(float) * (size_t)kMaxPartials);
    pl->ws_bytes = off;

    try {
        pl->blob.assign(pl->tables_end - pl->off_win, 0);
    } catch (...) {
        delete pl;
        return fail(SST_E_NOMEM, "table allocation failed");
    }
    auto put = [&](size_t off_abs, size_t i, double re, double im) {
        float *f = reinterpret_cast<float *>(pl->blob.data() + (off_abs - pl->off_win));
        f[2 * i] = (float)re;
        f[2 * i + 1] = (float)im;
    };
    for (int i = 0; i < L; ++i)
        put(pl->off_win, i, g[i], pl->s_pack * gd[i]);
    for (int k = k1; k <= k2; ++k) {
        const double a = kTwoPi * (double)mod_exact((int64_t)k * pl->M, NF) / NF;
        put(pl->off_cph, k - k1, std::cos(a), std::sin(a));
    }
    for (int r = 0; r < NF; ++r) {
        const double a = kTwoPi * (double)r / NF;
        put(pl->off_twid, r, std::cos(a), -std::sin(a));
    }
    for (int r = 0; r < pl->n_lo; ++r) {
        const double a = kTwoPi * (double)r / pl->G;
        put(pl->off_phlo, r, std::cos(a), std::sin(a));
    }
    for (int h = 0; h < pl->n_hi; ++h) {
        const double a = kTwoPi * (double)((int64_t)h << pl->lo_bits) / pl->G;
        put(pl->off_phhi, h, std::cos(a), std::sin(a));
    }
    *out = pl;
    return SST_OK;
}

sst_status sst_plan_query(sst_plan_t pl, sst_shape *out)
{
    if (!pl || !out)
        return fail(SST_E_ARG, "plan or out is NULL");
    out->n_samples = pl->p.n_samples;
    out->n_frames = pl->n_frames;
    out->win_len = pl->p.win_len;
    out->hop = pl->p.hop;
    out->nfft = pl->p.nfft;
    out->subdiv = pl->p.subdiv;
    out->k1 = pl->k1;
    out->k2 = pl->k2;
    out->n_src = pl->n_src;
    out->n_dst = pl->n_dst;
    out->workspace_bytes = pl->ws_bytes;
    out->t_row_bytes = sizeof(float) * 2 * (size_t)pl->n_dst;
    return SST_OK;
}

sst_status sst_plan_bind(sst_plan_t pl, void *workspace, size_t bytes, void *stream)
{
    if (!pl)
        return fail(SST_E_ARG, "plan is NULL");
    if (!workspace || bytes < pl->ws_bytes || (reinterpret_cast<uintptr_t>(workspace) % kAlign))
        return fail(SST_E_WORKSPACE, "workspace NULL, not 256-byte aligned, or smaller than "
                                     "sst_shape.workspace_bytes");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute");
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    e = hipMemcpyAsync(ws + pl->off_win, pl->blob.data(), pl->blob.size(),
                       hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(tables)");
    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute(shared memory)");
    const size_t need = sst::fwd_lds_bytes(pl->p.nfft, pl->n_src);
    if (need == 0 || need > (size_t)max_lds)
        return fail(SST_E_UNSUPPORTED, "forward kernel needs " + std::to_string(need) +
                                           " bytes of LDS, the device offers " +
                                           std::to_string(max_lds));
    pl->ws = ws;
    pl->device = dev;
    pl->cus = cus;
    pl->fwd_grid_cap = cus * sst::fwd_occupancy(pl->p.nfft, pl->p.win_len, pl->n_src);
    int mg = cus * sst::max_occupancy(pl->p.nfft, pl->p.win_len);
    pl->max_grid_cap = mg < kMaxPartials ? mg : kMaxPartials;
    return SST_OK;
}

sst_status sst_forward(sst_plan_t pl, const float *x, int64_t frame0, int64_t nframes, float *T,
                       const sst_fwd_aux *aux, uint32_t flags, void *stream)
{
    if (!pl)
        return fail(SST_E_ARG, "plan is NULL");
    if (!pl->ws)
        return fail(SST_E_STATE, "plan is not bound to a workspace");
    if (!x || !T)
        return fail(SST_E_ARG, "x and T must not be NULL");
    if (frame0 < 0 || nframes < 0 || frame0 + nframes > pl->n_frames)
        return fail(SST_E_ARG, "frame range outside [0, n_frames)");
    if (flags & ~SST_FWD_REUSE_GAMMA)
        return fail(SST_E_ARG, "unknown forward flags");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int NF = pl->p.nfft;
    sst::Ctrl *ctrl = reinterpret_cast<sst::Ctrl *>(pl->ws);
    const float2 *win = reinterpret_cast<const float2 *>(pl->ws + pl->off_win);
    const float2 *twid = reinterpret_cast<const float2 *>(pl->ws + pl->off_twid);

    if (!(flags & SST_FWD_REUSE_GAMMA)) {
        sst::MaxArgs m{};
        m.x = x;
        m.n = pl->p.n_samples;
        m.n_frames = pl->n_frames;
        m.win = win;
        m.twid = twid;
        m.partial = reinterpret_cast<float *>(pl->ws + pl->off_part);
        m.L = pl->p.win_len;
        m.M = pl->M;
        m.hop = pl->p.hop;
        m.k1 = pl->k1;
        m.n_src = pl->n_src;
        const int F = sst::fwd_frames_per_iter(NF);
        const int64_t iters = ((pl->n_frames + 1) / 2 + F - 1) / F;
        const int grid = (int)(iters < pl->max_grid_cap ? iters : pl->max_grid_cap);
        hipError_t e = sst::launch_threshold(NF, m, ctrl, pl->p.thr_mode, (float)pl->p.thr,
                                             grid, s);
        if (e != hipSuccess)
            return hip_fail(e, "threshold launch");
    }
    if (aux && aux->gamma) {
        hipError_t e = hipMemcpyAsync(aux->gamma, &ctrl->gamma, sizeof(float),
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync(gamma)");
    }
    if (nframes == 0)
        return SST_OK;

    sst::FwdArgs a{};
    a.x = x;
    a.n = pl->p.n_samples;
    a.frame0 = frame0;
    a.nframes = nframes;
    a.win = win;
    a.cphase = reinterpret_cast<const float2 *>(pl->ws + pl->off_cph);
    a.twid = twid;
    a.ctrl = ctrl;
    a.T = reinterpret_cast<float2 *>(T);
    if (aux) {
        a.S = reinterpret_cast<float2 *>(aux->S);
        a.Sd = reinterpret_cast<float2 *>(aux->Sd);
        a.idx = aux->idx;
        a.colstats = aux->colstats;
    }
    a.L = pl->p.win_len;
    a.M = pl->M;
    a.hop = pl->p.hop;
    a.k1 = pl->k1;
    a.n_src = pl->n_src;
    a.n_dst = pl->n_dst;
    a.z = pl->p.subdiv;
    {
        const int nt = sst::fwd_threads(NF);
        const double ang = kTwoPi * (double)mod_exact((int64_t)nt * pl->M, NF) / NF;
        a.cph_step = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    a.inv_s = (float)(1.0 / pl->s_pack);
    a.cdelta = (float)(NF / (kTwoPi * pl->s_pack));
    const int F = sst::fwd_frames_per_iter(NF);
    const int64_t iters = (nframes + F - 1) / F;
    const int grid = (int)(iters < pl->fwd_grid_cap ? iters : pl->fwd_grid_cap);
    hipError_t e = sst::launch_forward(NF, a, grid, s);
    if (e != hipSuccess)
        return hip_fail(e, "forward launch");
    return SST_OK;
}

sst_status sst_ridge(sst_plan_t pl, const float *T, int64_t nframes, const int32_t *band,
                     int32_t n_comp, int32_t *ridge, void *stream)
{
    if (!pl)
        return fail(SST_E_ARG, "plan is NULL");
    if (!pl->ws)
        return fail(SST_E_STATE, "plan is not bound to a workspace");
    if (!T || !band || !ridge)
        return fail(SST_E_ARG, "T, band and ridge must not be NULL");
    if (n_comp < 1 || n_comp > 16)
        return fail(SST_E_ARG, "n_comp must lie in [1, 16]");
    if (nframes < 0 || nframes > pl->n_frames)
        return fail(SST_E_ARG, "nframes outside [0, n_frames]");
    if (nframes == 0)
        return SST_OK;
    sst::RidgeArgs a{};
    a.T = reinterpret_cast<const float2 *>(T);
    a.nframes = nframes;
    a.n_dst = pl->n_dst;
    a.n_comp = n_comp;
    for (int q = 0; q < n_comp; ++q) {
        a.band[2 * q] = band[2 * q];
        a.band[2 * q + 1] = band[2 * q + 1];
    }
    a.ridge = ridge;
    hipError_t e = sst::launch_ridge(a, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(e, "ridge launch");
    return SST_OK;
}

sst_status sst_inverse(sst_plan_t pl, const float *T, int64_t frame0, int64_t nframes,
                       const int32_t *ridge, int32_t n_comp, int32_t hw, float *xhat,
                       const float *xref, double *err, uint32_t flags, void *stream)
{
    if (!pl)
        return fail(SST_E_ARG, "plan is NULL");
    if (!pl->ws)
        return fail(SST_E_STATE, "plan is not bound to a workspace");
    if (!T || !ridge || !xhat)
        return fail(SST_E_ARG, "T, ridge and xhat must not be NULL");
    if (flags & ~(SST_INV_ACCUMULATE | SST_INV_EQ15))
        return fail(SST_E_ARG, "unknown inverse flags");
    if (n_comp < 1 || n_comp > 65535)
        return fail(SST_E_ARG, "n_comp must lie in [1, 65535]");
    if (hw < 0 || hw > 512)
        return fail(SST_E_ARG, "hw must lie in [0, 512]");
    if (frame0 < 0 || nframes < 1 || frame0 + nframes > pl->n_frames)
        return fail(SST_E_ARG, "frame range outside [0, n_frames)");
    const bool whole = frame0 == 0 && nframes == pl->n_frames;
    const bool accumulate = (flags & SST_INV_ACCUMULATE) != 0;
    if (err && (!xref || !whole || accumulate))
        return fail(SST_E_ARG, "err needs xref and a whole-signal call without accumulation");
    if (pl->G > 65536)
        return fail(SST_E_UNSUPPORTED, "inverse needs subdiv * nfft <= 65536");

    sst::InvArgs a{};
    a.T = reinterpret_cast<const float2 *>(T);
    a.ridge = ridge;
    a.xhat = xhat;
    a.xref = xref;
    a.err = err;
    a.win = reinterpret_cast<const float2 *>(pl->ws + pl->off_win);
    a.ph_lo = reinterpret_cast<const float2 *>(pl->ws + pl->off_phlo);
    a.ph_hi = reinterpret_cast<const float2 *>(pl->ws + pl->off_phhi);
    a.n = pl->p.n_samples;
    a.n_frames = pl->n_frames;
    a.frame0 = frame0;
    a.nframes = nframes;
    a.L = pl->p.win_len;
    a.M = pl->M;
    a.hop = pl->p.hop;
    a.nfft = pl->p.nfft;
    a.k1 = pl->k1;
    a.z = pl->p.subdiv;
    a.n_dst = pl->n_dst;
    a.hw = hw;
    a.n_comp = n_comp;
    a.G = pl->G;
    a.lo_bits = pl->lo_bits;
    a.g_pow2 = is_pow2(pl->G) ? 1 : 0;
    a.inv_G = (float)(1.0 / pl->G);
    a.inv_nfft = (float)(1.0 / pl->p.nfft);
    a.accumulate = accumulate ? 1 : 0;
    const int W = 2 * hw + 1;
    int fb = 2048 / W;
    a.fb = fb < 1 ? 1 : (fb > 128 ? 128 : fb);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    if (flags & SST_INV_EQ15) {
        if (pl->p.hop != 1)
            return fail(SST_E_ARG, "SST_INV_EQ15 needs hop == 1");
        a.span_lo = frame0;
        a.span_len = nframes;
        hipError_t e = sst::launch_inverse_eq15(a, (float)(1.0 / (pl->p.nfft * pl->g0)), s);
        if (e != hipSuccess)
            return hip_fail(e, "inverse (Eq. 15) launch");
        return SST_OK;
    }
    if (whole) {
        a.span_lo = 0;
        a.span_len = pl->p.n_samples;
    } else {
        int64_t lo = frame0 * pl->p.hop - pl->M;
        int64_t hi = (frame0 + nframes - 1) * pl->p.hop + pl->M;
        if (lo < 0)
            lo = 0;
        if (hi > pl->p.n_samples - 1)
            hi = pl->p.n_samples - 1;
        if (hi < lo)
            return SST_OK;
        a.span_lo = lo;
        a.span_len = hi - lo + 1;
    }
    if (sst::inv_lds_bytes(a) > 64 * 1024)
        return fail(SST_E_UNSUPPORTED, "inverse LDS tables exceed 64 KiB");
    hipError_t e = sst::launch_inverse(a, s);
    if (e != hipSuccess)
        return hip_fail(e, "inverse launch");
    return SST_OK;
}

void sst_destroy(sst_plan_t pl) { delete pl; }

const char *sst_status_string(sst_status s)
{
    switch (s) {
    case SST_OK: return "SST_OK";
    case SST_E_ARG: return "SST_E_ARG: invalid argument";
    case SST_E_UNSUPPORTED: return "SST_E_UNSUPPORTED: not supported by this build";
    case SST_E_WORKSPACE: return "SST_E_WORKSPACE: workspace missing, misaligned or too small";
    case SST_E_DEVICE: return "SST_E_DEVICE: HIP call failed";
    case SST_E_STATE: return "SST_E_STATE: plan not bound";
    case SST_E_NOMEM: return "SST_E_NOMEM: host allocation failed";
    default: return "unknown sst_status";
    }
}

const char *sst_last_error(void) { return g_err.c_str(); }

sst_status sst_critical_hf(double n, double sigma_s, double fs, double *eq38, double *eq46)
{
    if (!(n > 0.0) || !(sigma_s > 0.0) || !(fs > 0.0))
        return fail(SST_E_ARG, "n, sigma_s and fs must be > 0");
    // Sec. 4: Eq. 37 with Eqs. 12, 35 gives Eq. 38; Eq. 46 with the same substitutions.
    if (eq38)
        *eq38 = 3.0 * n / (4.0 * M_PI * sigma_s * fs);
    if (eq46)
        *eq46 = std::sqrt(2.0) * n / (2.0 * M_PI * sigma_s * fs);
    return SST_OK;
}

}  // extern "C"
