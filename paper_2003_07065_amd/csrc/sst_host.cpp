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
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sst.h"
#include "sst_internal.h"

namespace {

thread_local std::string g_err;

std::atomic<uint64_t> g_plan_serial{0};

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
constexpr size_t kGemmTableMax = size_t(64) << 20;   // bytes of one part of the GEMM A table
// The speculative forward starts from the maximum over every k-th item,
// k = max(kSeedStep, items / workgroups): one round of the grid at most.
constexpr int kSeedStep = 32;

int64_t seed_step(int64_t items, int grid_cap, int tuned)
{
    if (tuned > 0)
        return tuned;
    const int64_t k = grid_cap > 0 ? (items + grid_cap - 1) / grid_cap : 1;
    return k > kSeedStep ? k : kSeedStep;
}

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

// A plan's device state: the workspace holding its tables and the launch
// limits of the device it lives on.
struct Bound {
    unsigned char *ws = nullptr;
    int device = -1;
    int cus = 0;
    int fwd_occ = 0;        // forward workgroups that fit one CU
    int fwd_grid_cap = 0;   // persistent forward grid: CUs x min(fwd_occ, tuned count)
    // a thresholding forward has set gamma in this workspace (cleared by every
    // bind, which leaves the control block unset)
    bool gamma_valid = false;
};

struct sst_plan_s {
    sst_params p{};
    int M = 0, k1 = 0, k2 = 0, n_src = 0, n_dst = 0;
    int64_t n_frames = 0;
    double s_pack = 1.0;
    double g0 = 0.0;
    int G = 0, lo_bits = 0, n_lo = 0, n_hi = 0;
    // DFT-as-GEMM tier
    int gemm_ft = 0, row_tiles = 0, ksteps = 0, slab = 0;
    float unscale_g = 1.f, unscale_gd = 1.f, gmax2 = 0.f;
    // inverse: power of two that puts the window's largest |g| in [2^13, 2^14)
    float inv_g_scale = 1.f, inv_g_unscale = 1.f;
    // inverse: groups of 256 output samples per workgroup (1 or kInvWideTF)
    int inv_tf = 1;
    // launch choices set by sst_plan_set_tuning / the autotuner (0 = default)
    sst_tuning tune{};
    size_t off_afrag = 0, off_afrag_lo = 0, afrag_bytes = 0;
    // workspace layout (bytes): control block, descriptor slot, tables
    size_t off_desc = 0, off_idesc = 0, off_win = 0, off_twid = 0, off_phlo = 0, off_phhi = 0;
    size_t off_den = 0, off_den2 = 0;
    size_t tables_end = 0, ws_bytes = 0;
    // speculative threshold (FFT tier): least kept |S|^2 per forward item, the
    // fix-up list and its count
    int64_t n_items = 0;
    size_t off_smin = 0, off_list = 0, off_list_n = 0;
    std::vector<unsigned char> blob;   // host image of [off_win, tables_end)
    uint64_t serial = 0;               // unique per plan (owner of the static scratch)
    Bound bd;                          // the workspace bound by sst_plan_bind
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
    if (p->n_samples >= (int64_t(1) << 30))
        return fail(SST_E_UNSUPPORTED, "n_samples must be below 2^30 (32-bit sample indices)");
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
    if (p->precision != SST_PREC_FP32_FFT && p->precision != SST_PREC_GEMM_BF16 &&
        p->precision != SST_PREC_GEMM_F16X3)
        return fail(SST_E_ARG, "unknown precision");
    if (p->precision != SST_PREC_FP32_FFT && (p->hop % 8) != 0)
        return fail(SST_E_UNSUPPORTED, "the GEMM tiers need hop a multiple of 8");
    if (p->flags != 0)
        return fail(SST_E_ARG, "params.flags must be 0");
    return SST_OK;
}

// Descriptor of one channel for a forward call over frames [frame0, frame0 + nframes).
sst::ChanDesc chan_desc(const sst_plan_s *pl, const unsigned char *ws, const float *x,
                        int64_t frame0, int64_t nframes, float *T, const sst_fwd_aux *aux,
                        sst::Ctrl *ctrl)
{
    sst::ChanDesc d{};
    d.x = x;
    d.n = pl->p.n_samples;
    d.n_frames = pl->n_frames;
    d.frame0 = frame0;
    d.nframes = nframes;
    d.win = reinterpret_cast<const float2 *>(ws + pl->off_win);
    d.ctrl = ctrl;
    d.T = reinterpret_cast<float2 *>(T);
    if (aux) {
        d.S = reinterpret_cast<float2 *>(aux->S);
        d.Sd = reinterpret_cast<float2 *>(aux->Sd);
        d.idx = aux->idx;
        d.colstats = aux->colstats;
    }
    d.L = pl->p.win_len;
    d.M = pl->M;
    d.hop = pl->p.hop;
    d.k1 = pl->k1;
    d.n_src = pl->n_src;
    d.n_dst = pl->n_dst;
    d.z = pl->p.subdiv;
    d.thr_mode = pl->p.thr_mode;
    d.thr = (float)pl->p.thr;
    d.inv_s = (float)(1.0 / pl->s_pack);
    d.cdelta = (float)(pl->p.nfft / (kTwoPi * pl->s_pack));
    return d;
}

// Words per residue row of the decimated inverse window table: at least
// (2 JL) / H + 2 (JL = M + 63 + 16 H), rounded up to a stride whose residue
// mod 64 spreads the lanes' reads over the LDS banks (each lane of a wave
// reads its own residue row; of the strides, these residues leave the fewest
// lanes sharing a bank over a range of hops).
int inv_dec_row(int M, int hop)
{
    const int reach = M + 63 + 16 * hop;
    int tr = (2 * reach) / hop + 2;
    for (;; ++tr) {
        const int m = tr & 63;
        if (m == 6 || m == 10 || m == 26 || m == 38 || m == 42)
            return tr;
    }
}

// Descriptor of one channel's inverse over frames [frame0, frame0 + nframes).
sst::InvDesc inv_desc(const sst_plan_s *pl, const float *T, int64_t frame0, int64_t nframes,
                      const int32_t *ridge, int n_comp, int hw, float *xhat, const float *xref,
                      double *err, bool accumulate)
{
    sst::InvDesc a{};
    a.T = reinterpret_cast<const float2 *>(T);
    a.ridge = ridge;
    a.xhat = xhat;
    a.xref = xref;
    a.err = err;
    a.win = reinterpret_cast<const float2 *>(pl->bd.ws + pl->off_win);
    a.ph_lo = reinterpret_cast<const float2 *>(pl->bd.ws + pl->off_phlo);
    a.ph_hi = reinterpret_cast<const float2 *>(pl->bd.ws + pl->off_phhi);
    a.den = reinterpret_cast<const float *>(pl->bd.ws + pl->off_den);
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
    a.g_scale = pl->inv_g_scale;
    a.g_unscale = pl->inv_g_unscale;
    a.dec_reach = pl->M + 63 + 16 * pl->p.hop;
    a.dec_row = inv_dec_row(pl->M, pl->p.hop);
    a.accumulate = accumulate ? 1 : 0;
    if (frame0 == 0 && nframes == pl->n_frames) {
        a.span_lo = 0;
        a.span_len = pl->p.n_samples;
    } else {
        int64_t lo = frame0 * pl->p.hop - pl->M;
        int64_t hi = (frame0 + nframes - 1) * pl->p.hop + pl->M;
        if (lo < 0)
            lo = 0;
        if (hi > pl->p.n_samples - 1)
            hi = pl->p.n_samples - 1;
        a.span_lo = lo;
        a.span_len = hi >= lo ? hi - lo + 1 : 0;
    }
    const int64_t tile = (int64_t)sst::kInvTileSamples * pl->inv_tf;
    a.tiles = (a.span_len + tile - 1) / tile;
    a.blk0 = 0;
    a.blk_end = (int64_t)n_comp * a.tiles;
    return a;
}

// Records aux->kernel_events[i] (when given) on stream s.
hipError_t record_event(const sst_fwd_aux *aux, int i, hipStream_t s)
{
    if (!aux || !aux->kernel_events[i])
        return hipSuccess;
    return hipEventRecord(reinterpret_cast<hipEvent_t>(aux->kernel_events[i]), s);
}

// Frames of one call that a tile of tf x 256 output samples can meet (even).
int inv_max_k(int M, int hop, int tf)
{
    const int k = (sst::kInvTileSamples * tf - 1 + 2 * M) / hop + 2;
    return (k + 1) & ~1;
}
int inv_max_k(const sst_plan_s *pl) { return inv_max_k(pl->M, pl->p.hop, pl->inv_tf); }
bool inv_wide_fits(const sst_plan_s *pl)
{
    return inv_max_k(pl->M, pl->p.hop, sst::kInvWideTF) <= sst::kInvWideKB;
}
// Words of the plan's decimated inverse window table (InvDesc::dec_row times the hop).
int inv_dec_words(const sst_plan_s *pl)
{
    return pl->p.hop * inv_dec_row(pl->M, pl->p.hop);
}
// Extra-wide tiles (2048 samples) stage every frame they meet in one block
// and need the hop-decimated window table.
bool inv_xwide_fits(const sst_plan_s *pl)
{
    return inv_max_k(pl->M, pl->p.hop, sst::kInvXWideTF) <= sst::kInvWideKB &&
           inv_dec_words(pl) <= sst::kInvDecMax;
}
// The default tile width: the widest that fits.
int inv_default_tf(const sst_plan_s *pl)
{
    return inv_xwide_fits(pl) ? sst::kInvXWideTF : (inv_wide_fits(pl) ? sst::kInvWideTF : 1);
}

// max_dec: the largest decimated window table of the list (inv_dec_words);
// max_L: its longest window; tf: sample groups per workgroup of every channel.
sst::InvLaunch inv_launch(const sst::InvDesc *dev, int n_ch, int64_t blk_begin, int max_k,
                          int max_tab, int max_L, int max_dec, int tf, int groups = 1)
{
    sst::InvLaunch l{};
    l.ch = dev;
    l.n_ch = n_ch;
    l.tf = tf;
    l.groups = groups;
    l.blk_begin = blk_begin;
    l.max_k = max_k;
    l.max_tab = max_tab;
    l.dec = max_dec <= sst::kInvDecMax ? 1 : 0;
    l.max_gtab = ((l.dec ? max_dec : max_L + 2) + 3) & ~3;
    return l;
}

// Wide tiles with a decimated window table may stage 2 or 4 destination
// groups of the tile's zones at once (a tuning choice, when that fits three or
// two workgroups per CU); a plan's choice depends on the plan alone, so
// single-channel and batched calls take the same kernel (and give the same
// bits).
bool inv_groups_fit(const sst_plan_s *pl, int tf, int groups)
{
    if (tf != sst::kInvWideTF || inv_dec_words(pl) > sst::kInvDecMax)
        return false;
    sst::InvLaunch l = inv_launch(nullptr, 1, 0, inv_max_k(pl->M, pl->p.hop, tf),
                                  pl->n_lo + pl->n_hi, pl->p.win_len, inv_dec_words(pl), tf,
                                  groups);
    return sst::inv_lds_bytes(l) <= sst::inv_group_lds_max(groups);
}
// The plan's groups staged together: the tuned value, else 1 (the default).
int inv_groups_of(const sst_plan_s *pl)
{
    const int g = pl->tune.inv_groups;
    return (g > 1 && inv_groups_fit(pl, pl->inv_tf, g)) ? g : 1;
}
// Kind of inverse tile of a plan: 0 narrow, 1 wide, 2 / 3 wide with 2 / 4
// groups staged together, 4 extra-wide.
int inv_kind_of(const sst_plan_s *pl)
{
    if (pl->inv_tf <= 1)
        return 0;
    if (pl->inv_tf == sst::kInvXWideTF)
        return 4;
    const int g = inv_groups_of(pl);
    return g == 4 ? 3 : (g == 2 ? 2 : 1);
}
constexpr int kInvKinds = 5;
int inv_kind_tf(int kind)
{
    return kind == 0 ? 1 : (kind == 4 ? sst::kInvXWideTF : sst::kInvWideTF);
}

// Round to BF16, nearest even.
uint16_t to_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

uint16_t f16_bits(_Float16 h)
{
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}

// A fragments of the DFT-as-GEMM tier: row r = 4 b + p (source bin k1 + b;
// p = Re S, Im S, Re S', Im S'), column j = tap (t = j - M), value
// w[t] e^{-i 2 pi ((k t) mod N_f) / N_f} with w = g (p < 2) or g' (p >= 2),
// computed in float64 and stored in the order the 32x32x16 MFMA reads them:
// fragment (row tile, k step, lane) holds row 32 rt + lane mod 32, taps
// 16 ks + 8 (lane / 32) .. +7.  The FP16 split scales the g rows and the g'
// rows by powers of two that bring their largest magnitude into [2^13, 2^14).
void build_afrag(sst_plan_s *pl, const std::vector<double> &g, const std::vector<double> &gd)
{
    const int L = pl->p.win_len, NF = pl->p.nfft, M = pl->M;
    const bool split = pl->p.precision == SST_PREC_GEMM_F16X3;
    double mg = 0.0, mgd = 0.0;
    for (int j = 0; j < L; ++j) {
        mg = std::max(mg, std::fabs(g[j]));
        mgd = std::max(mgd, std::fabs(gd[j]));
    }
    auto pow2_scale = [](double m) {
        int e = 0;
        std::frexp(m, &e);   // m < 2^e
        return m > 0.0 ? 14 - e : 0;
    };
    const int sg = split ? pow2_scale(mg) : 0, sgd = split ? pow2_scale(mgd) : 0;
    pl->gmax2 = (float)(mg * mg * (1.0 + 1e-6));
    pl->unscale_g = (float)std::ldexp(1.0, -sg);
    pl->unscale_gd = (float)std::ldexp(1.0, -sgd);
    uint16_t *hi = reinterpret_cast<uint16_t *>(pl->blob.data() + (pl->off_afrag - pl->off_win));
    uint16_t *lo = split ? reinterpret_cast<uint16_t *>(pl->blob.data() +
                                                        (pl->off_afrag_lo - pl->off_win))
                         : nullptr;
    for (int rt = 0; rt < pl->row_tiles; ++rt)
        for (int ks = 0; ks < pl->ksteps; ++ks)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 8; ++e) {
                    const int r = rt * 32 + (lane & 31);
                    const int j = ks * 16 + 8 * (lane >> 5) + e;
                    double v = 0.0;
                    if (r < 4 * pl->n_src && j < L) {
                        const int b = r / 4, part = r % 4;
                        const int64_t k = pl->k1 + b, t = j - M;
                        int64_t rr = (k * t) % NF;
                        if (rr < 0)
                            rr += NF;
                        const double ang = kTwoPi * (double)rr / NF;
                        const double w = part < 2 ? g[j] : gd[j];
                        v = (part % 2 == 0) ? w * std::cos(ang) : -w * std::sin(ang);
                        v = std::ldexp(v, part < 2 ? sg : sgd);
                    }
                    const size_t o = (((size_t)rt * pl->ksteps + ks) * 64 + lane) * 8 + e;
                    if (split) {
                        const _Float16 h = (_Float16)v;
                        hi[o] = f16_bits(h);
                        lo[o] = f16_bits((_Float16)(v - (double)h));
                    } else {
                        hi[o] = to_bf16((float)v);
                    }
                }
}


// Forward grid of a binding: CUs x the resident workgroups, capped by the
// tuned count when one is set.
void apply_grid(const sst_plan_s *pl, Bound &bd)
{
    int wg = bd.fwd_occ > 0 ? bd.fwd_occ : 1;
    if (pl->tune.fwd_wg_per_cu > 0 && pl->tune.fwd_wg_per_cu < wg)
        wg = pl->tune.fwd_wg_per_cu;
    bd.fwd_grid_cap = bd.cus * wg;
}

// Device state of a binding to the workspace `ws` on the current device:
// launch limits from the device attributes, then the plan's tables uploaded
// with one asynchronous copy on `s` (no allocation).
sst_status bind_impl(sst_plan_s *pl, Bound &bd, unsigned char *ws, hipStream_t s)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute");
    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute(shared memory)");
    const size_t need = sst::fwd_lds_bytes(pl->p.nfft);
    if (need == 0 || need > (size_t)max_lds)
        return fail(SST_E_UNSUPPORTED, "forward kernel needs " + std::to_string(need) +
                                           " bytes of LDS, the device offers " +
                                           std::to_string(max_lds));
    e = hipMemcpyAsync(ws + pl->off_win, pl->blob.data(), pl->blob.size(),
                       hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(tables)");
    bd.ws = ws;
    bd.device = dev;
    bd.cus = cus;
    bd.gamma_valid = false;
    bd.fwd_occ = sst::fwd_occupancy(pl->p.nfft, pl->p.win_len);
    if (pl->gemm_ft)
        bd.fwd_occ = sst::gemm_occupancy(
            pl->p.precision, pl->gemm_ft,
            sst::gemm_lds_bytes(pl->p.precision, pl->gemm_ft, pl->n_dst, pl->slab, pl->p.win_len));
    apply_grid(pl, bd);
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
    pl->serial = g_plan_serial.fetch_add(1) + 1;
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
    // The widest inverse tiles whose frames fit one staged block.
    pl->inv_tf = inv_default_tf(pl);

    // Workspace layout.
    size_t off = align_up(sizeof(sst::Ctrl));
    pl->off_desc = off;
    off = align_up(off + sizeof(sst::ChanDesc));
    pl->off_idesc = off;
    off = align_up(off + sizeof(sst::InvDesc));
    pl->off_win = off;
    off = align_up(off + sizeof(float) * 2 * (size_t)L);
    pl->off_twid = off;
    off = align_up(off + sizeof(float) * 2 * (size_t)NF);
    pl->off_phlo = off;
    off = align_up(off + sizeof(float) * 2 * (size_t)pl->n_lo);
    pl->off_phhi = off;
    off = align_up(off + sizeof(float) * 2 * (size_t)pl->n_hi);
    pl->off_den = off;
    off = align_up(off + sizeof(float) * (size_t)p.hop);
    pl->off_den2 = off;
    off = align_up(off + sizeof(float) * (size_t)p.hop);
    const bool gemm = p.precision != SST_PREC_FP32_FFT;
    if (gemm) {
        pl->row_tiles = (4 * pl->n_src + 31) / 32;
        pl->ksteps = (L + 15) / 16;
        // the DFT-matrix fragments (4 n_src rows x L taps) stay a small table:
        // the tiers are for narrow bands, where they cost 4 n_src L products
        // per frame against the FFT's N_f log N_f
        if ((size_t)pl->row_tiles * pl->ksteps * 64 * 16 > kGemmTableMax) {
            delete pl;
            return fail(SST_E_UNSUPPORTED, "the GEMM tiers need a DFT-matrix table of at most 64 MiB "
                                           "(4 n_src x L taps): narrow the band or use the FFT tier");
        }
        for (int ft : {64, 32}) {
            const int slab = ((ft - 1) * p.hop + 16 * pl->ksteps + 7) / 8 * 8;
            if (sst::gemm_lds_bytes(p.precision, ft, pl->n_dst, slab, L) <= 80 * 1024) {
                pl->gemm_ft = ft;
                pl->slab = slab;
                break;
            }
        }
        if (!pl->gemm_ft) {
            delete pl;
            return fail(SST_E_UNSUPPORTED, "the GEMM tiers need 32 * n_dst * 8 bytes of LDS "
                                           "histogram plus the sample slab within 80 KiB");
        }
        pl->afrag_bytes = (size_t)pl->row_tiles * pl->ksteps * 64 * 16;
        pl->off_afrag = off;
        off = align_up(off + pl->afrag_bytes);
        if (p.precision == SST_PREC_GEMM_F16X3) {
            pl->off_afrag_lo = off;
            off = align_up(off + pl->afrag_bytes);
        }
    }
    pl->tables_end = off;
    {
        // speculative threshold state: one entry per forward item (FFT tier)
        // or per GEMM tile
        pl->n_items = gemm ? (pl->n_frames + pl->gemm_ft - 1) / pl->gemm_ft
                           : (pl->n_frames + sst::fwd_frames_per_iter(NF) - 1) /
                                 sst::fwd_frames_per_iter(NF);
        pl->off_smin = off;
        off = align_up(off + sizeof(float) * (size_t)pl->n_items);
        pl->off_list = off;
        off = align_up(off + sizeof(int32_t) * (size_t)pl->n_items);
        pl->off_list_n = off;
        off = align_up(off + sizeof(int32_t));
    }
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
    double mgi = 0.0;
    for (int i = 0; i < L; ++i) {
        put(pl->off_win, i, g[i], pl->s_pack * gd[i]);
        mgi = std::max(mgi, std::fabs((double)(float)g[i]));
    }
    {
        int eg = 0;
        std::frexp(mgi, &eg);   // mgi < 2^eg
        const int tg = mgi > 0.0 ? 14 - eg : 0;
        pl->inv_g_scale = (float)std::ldexp(1.0, tg);
        pl->inv_g_unscale = (float)std::ldexp(1.0, -tg);
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
    {   // interior OLA denominators (Eq. 26): g[0] sum of g[j] over j = r mod H, |j| <= M
        float *den = reinterpret_cast<float *>(pl->blob.data() + (pl->off_den - pl->off_win));
        for (int r = 0; r < p.hop; ++r) {
            double acc = 0.0;
            for (int j = -pl->M; j <= pl->M; ++j)
                if ((((j % p.hop) + p.hop) % p.hop) == r)
                    acc += g[j + pl->M];
            den[r] = (float)(pl->g0 * acc);
        }
        // STFT synthesis (Eq. 11): sum of g[j]^2 over j = r mod H
        float *den2 = reinterpret_cast<float *>(pl->blob.data() + (pl->off_den2 - pl->off_win));
        for (int r = 0; r < p.hop; ++r) {
            double acc = 0.0;
            for (int j = -pl->M; j <= pl->M; ++j)
                if ((((j % p.hop) + p.hop) % p.hop) == r)
                    acc += g[j + pl->M] * g[j + pl->M];
            den2[r] = (float)acc;
        }
    }
    if (gemm)
        build_afrag(pl, g, gd);
    if (const char *cache = std::getenv("SST_TUNE_CACHE")) {
        // a matching cache entry, if any (a missing file or entry is no error)
        const std::string keep = g_err;
        if (sst_tuning_load(pl, cache) != SST_OK)
            g_err = keep;
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
    return bind_impl(pl, pl->bd, static_cast<unsigned char *>(workspace),
                     reinterpret_cast<hipStream_t>(stream));
}

static sst_status forward_impl(sst_plan_s *pl, Bound &bd, const float *x, int64_t frame0,
                               int64_t nframes, float *T, const sst_fwd_aux *aux, uint32_t flags,
                               void *stream);

sst_status sst_forward(sst_plan_t pl, const float *x, int64_t frame0, int64_t nframes, float *T,
                       const sst_fwd_aux *aux, uint32_t flags, void *stream)
{
    if (!pl)
        return fail(SST_E_ARG, "plan is NULL");
    if (!pl->bd.ws)
        return fail(SST_E_STATE, "plan is not bound to a workspace");
    return forward_impl(pl, pl->bd, x, frame0, nframes, T, aux, flags, stream);
}

// The plan whose tables the static scratch of each device holds (serial 0:
// none), and that binding's state.  One lock serialises the static calls.
struct StaticOwner {
    uint64_t serial = 0;
    Bound bd;
};
static std::mutex g_static_mu;
static StaticOwner g_static_owner[sst::kMaxDevices];

sst_status sst_forward_static(sst_plan_t pl, const float *x, int64_t frame0, int64_t nframes,
                              float *T, const sst_fwd_aux *aux, uint32_t flags, void *stream)
{
    if (!pl)
        return fail(SST_E_ARG, "plan is NULL");
    if (pl->ws_bytes > sst::kStaticScratchBytes)
        return fail(SST_E_UNSUPPORTED, "the plan needs " + std::to_string(pl->ws_bytes) +
                                           " bytes of workspace; the static scratch holds " +
                                           std::to_string(sst::kStaticScratchBytes));
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    unsigned char *ptr = nullptr;
    e = sst::static_scratch(dev, &ptr);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetSymbolAddress(static scratch)");
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticOwner &o = g_static_owner[dev];
    if (o.serial != pl->serial) {
        o.serial = 0;
        const sst_status st = bind_impl(pl, o.bd, ptr, reinterpret_cast<hipStream_t>(stream));
        if (st != SST_OK)
            return st;
        o.serial = pl->serial;
    }
    apply_grid(pl, o.bd);   // tuning set since the tables were uploaded
    return forward_impl(pl, o.bd, x, frame0, nframes, T, aux, flags, stream);
}

static sst_status forward_impl(sst_plan_s *pl, Bound &bd, const float *x, int64_t frame0,
                               int64_t nframes, float *T, const sst_fwd_aux *aux, uint32_t flags,
                               void *stream)
{
    if (!x || !T)
        return fail(SST_E_ARG, "x and T must not be NULL");
    if (frame0 < 0 || nframes < 0 || frame0 + nframes > pl->n_frames)
        return fail(SST_E_ARG, "frame range outside [0, n_frames)");
    if (flags & ~(SST_FWD_REUSE_GAMMA | SST_FWD_OUT_MAG_F32 | SST_FWD_OUT_MAG_F16))
        return fail(SST_E_ARG, "unknown forward flags");
    if ((flags & SST_FWD_OUT_MAG_F32) && (flags & SST_FWD_OUT_MAG_F16))
        return fail(SST_E_ARG, "choose one compressed output format");
    const int out_fmt = (flags & SST_FWD_OUT_MAG_F32) ? 1 : ((flags & SST_FWD_OUT_MAG_F16) ? 2 : 0);
    if (out_fmt && pl->gemm_ft)
        return fail(SST_E_UNSUPPORTED, "compressed outputs are produced by the FP32 FFT tier");
    if (out_fmt && aux && aux->colstats)
        return fail(SST_E_UNSUPPORTED, "colstats are summed from complex rows, not |T| rows");
    if ((flags & SST_FWD_REUSE_GAMMA) && !bd.gamma_valid)
        return fail(SST_E_STATE, "SST_FWD_REUSE_GAMMA before any thresholding forward call on "
                                 "this binding");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int NF = pl->p.nfft;
    const int F = sst::fwd_frames_per_iter(NF);
    sst::Ctrl *ctrl = reinterpret_cast<sst::Ctrl *>(bd.ws);
    sst::ChanDesc *slot = reinterpret_cast<sst::ChanDesc *>(bd.ws + pl->off_desc);
    const bool threshold = !(flags & SST_FWD_REUSE_GAMMA);
    const bool rel = pl->p.thr_mode == SST_THR_REL_MAX;
    const bool fft = !pl->gemm_ft;
    // per-coefficient outputs take the debug variant; the per-frame sums
    // (colstats) are an epilogue of the production kernel
    const bool debug = aux && (aux->S || aux->Sd || aux->idx);
    const int kind = debug ? sst::kFwdKindDebug
                           : ((aux && aux->colstats) ? sst::kFwdKindStats : sst::kFwdKindPlain);
    // A call over the whole signal that needs gamma takes the speculative
    // forward: threshold at a lower bound of gamma, then redo the items whose
    // decisions the final gamma changes.
    const bool spec = threshold && rel && !debug && frame0 == 0 && nframes == pl->n_frames &&
                      nframes > 0;
    sst::ChanDesc d = chan_desc(pl, bd.ws, x, frame0, nframes, T, aux, ctrl);
    d.out_fmt = out_fmt;
    d.item0 = 0;
    d.item_end = (nframes + F - 1) / F;
    d.mitem0 = 0;
    // threshold items of the FFT tier: forward items of the whole signal
    d.mitem_end = (threshold && rel && fft) ? (pl->n_frames + F - 1) / F : 0;
    int32_t *list = reinterpret_cast<int32_t *>(bd.ws + pl->off_list);
    int32_t *list_n = reinterpret_cast<int32_t *>(bd.ws + pl->off_list_n);
    // the upload also clears the running maximum (and the fix-up count)
    hipError_t e = sst::launch_put_desc(d, slot, threshold, spec ? list_n : nullptr, s);
    if (e != hipSuccess)
        return hip_fail(e, "descriptor upload");
    sst::GroupLaunch g{};
    g.ch = slot;
    g.n_ch = 1;
    g.twid = reinterpret_cast<const float2 *>(bd.ws + pl->off_twid);
    // GEMM tiers: arguments of a launch over frames [f0, f0 + nf)
    auto gemm_args = [&](int64_t f0, int64_t nf, int mode) {
        sst::GemmArgs ga{};
        ga.x = x;
        ga.n = pl->p.n_samples;
        ga.frame0 = f0;
        ga.nframes = nf;
        ga.afrag = bd.ws + pl->off_afrag;
        ga.afrag_lo = pl->off_afrag_lo ? bd.ws + pl->off_afrag_lo : nullptr;
        ga.win = reinterpret_cast<const float2 *>(bd.ws + pl->off_win);
        ga.ctrl = ctrl;
        ga.ctrlw = ctrl;
        ga.T = reinterpret_cast<float2 *>(T);
        if (aux && mode == 0) {
            ga.S = reinterpret_cast<float2 *>(aux->S);
            ga.Sd = reinterpret_cast<float2 *>(aux->Sd);
            ga.idx = aux->idx;
        }
        ga.L = pl->p.win_len;
        ga.M = pl->M;
        ga.hop = pl->p.hop;
        ga.k1 = pl->k1;
        ga.n_src = pl->n_src;
        ga.n_dst = pl->n_dst;
        ga.z = pl->p.subdiv;
        ga.row_tiles = pl->row_tiles;
        ga.ksteps = pl->ksteps;
        ga.slab = pl->slab;
        ga.unscale_g = pl->unscale_g;
        ga.unscale_gd = pl->unscale_gd;
        ga.cdelta = (float)(pl->p.nfft / kTwoPi);
        ga.bound_c = (float)(1.1 * std::sqrt(2.0 * pl->n_src * pl->p.nfft));
        ga.gmax2 = pl->gmax2;
        ga.mode = mode;
        ga.tile_step = 1;
        ga.thr_mode = pl->p.thr_mode;
        ga.thr = (float)pl->p.thr;
        ga.smin = reinterpret_cast<float *>(bd.ws + pl->off_smin);
        ga.list = list;
        ga.list_n = list_n;
        return ga;
    };
    auto gemm_grid = [&](int64_t visits) {
        return (int)(visits < bd.fwd_grid_cap ? visits : bd.fwd_grid_cap);
    };
    if (threshold && !fft) {
        // gamma on the tier's own arithmetic: the maximum over every tile of
        // the signal (a max-only pass), unless the speculative forward below
        // finds it as it goes
        if (rel && !spec) {
            const int64_t tiles_all = (pl->n_frames + pl->gemm_ft - 1) / pl->gemm_ft;
            const sst::GemmArgs gm = gemm_args(0, pl->n_frames, 1);
            if (tiles_all > 0)
                e = sst::launch_gemm_forward(pl->p.precision, pl->gemm_ft, false, gm,
                                             gemm_grid(tiles_all), s);
        }
        if (e == hipSuccess && !spec)
            e = sst::launch_gamma(g, s);
        if (e != hipSuccess)
            return hip_fail(e, "threshold launch");
        bd.gamma_valid = !spec;
    } else if (threshold) {
        g.item_begin = 0;
        g.item_stop = d.mitem_end;
        g.step = spec ? (int)seed_step(d.mitem_end, bd.fwd_grid_cap, pl->tune.seed_step) : 1;
        const int64_t visits = (d.mitem_end + g.step - 1) / g.step;
        const int grid = (int)(visits < bd.fwd_grid_cap ? visits : bd.fwd_grid_cap);
        e = sst::launch_max_prepass(NF, pl->p.win_len, g, grid, s);
        g.step = 0;
        if (e == hipSuccess && !spec)
            e = sst::launch_gamma(g, s);
        if (e != hipSuccess)
            return hip_fail(e, "threshold launch");
        // the speculative path sets gamma in spec_list_kernel, launched below
        // in the same call (an error there returns before anything reuses it)
        bd.gamma_valid = !spec;
    }
    if (aux && aux->gamma && !spec) {
        e = hipMemcpyAsync(aux->gamma, &ctrl->gamma, sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync(gamma)");
    }
    if (nframes == 0)
        return SST_OK;
    if (pl->gemm_ft) {
        if (aux && aux->colstats)
            return fail(SST_E_UNSUPPORTED, "colstats are not produced by the GEMM tiers");
        const int64_t tiles = (nframes + pl->gemm_ft - 1) / pl->gemm_ft;
        const bool dbg = aux && (aux->S || aux->Sd || aux->idx);
        if (spec) {
            // seed the running maximum with every k-th tile (max-only)
            sst::GemmArgs gs = gemm_args(0, nframes, 1);
            gs.tile_step = seed_step(tiles, bd.fwd_grid_cap, pl->tune.seed_step);
            e = sst::launch_gemm_forward(pl->p.precision, pl->gemm_ft, false, gs,
                                         gemm_grid((tiles + gs.tile_step - 1) / gs.tile_step), s);
            if (e != hipSuccess)
                return hip_fail(e, "GEMM threshold seed launch");
        }
        sst::GemmArgs ga = gemm_args(frame0, nframes, 0);
        ga.spec = spec ? 1 : 0;
        e = record_event(aux, 0, s);
        if (e == hipSuccess)
            e = sst::launch_gemm_forward(pl->p.precision, pl->gemm_ft, dbg, ga, gemm_grid(tiles), s);
        if (e == hipSuccess)
            e = record_event(aux, 1, s);
        if (e != hipSuccess)
            return hip_fail(e, "GEMM forward launch");
        if (!spec)
            return SST_OK;
        // gamma, the list of tiles that kept a coefficient at or below it, and
        // those tiles again at the final gamma
        g.item_begin = 0;
        g.item_stop = tiles;
        g.smin = reinterpret_cast<float *>(bd.ws + pl->off_smin);
        g.list = list;
        g.list_n = list_n;
        e = sst::launch_spec_list(g, s);
        if (e == hipSuccess)
            bd.gamma_valid = true;
        if (e == hipSuccess)
            e = sst::launch_gemm_forward(pl->p.precision, pl->gemm_ft, false,
                                         gemm_args(0, nframes, 2), gemm_grid(tiles), s);
        if (e != hipSuccess)
            return hip_fail(e, "GEMM speculative fix-up launch");
        if (aux && aux->gamma) {
            e = hipMemcpyAsync(aux->gamma, &ctrl->gamma, sizeof(float), hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess)
                return hip_fail(e, "hipMemcpyAsync(gamma)");
        }
        return SST_OK;
    }
    g.item_begin = 0;
    g.item_stop = d.item_end;
    const int grid = (int)(d.item_end < bd.fwd_grid_cap ? d.item_end : bd.fwd_grid_cap);
    if (!spec) {
        e = record_event(aux, 0, s);
        if (e == hipSuccess)
            e = sst::launch_forward(NF, pl->p.win_len, pl->n_src, pl->n_dst, kind, g, grid, s);
        if (e == hipSuccess)
            e = record_event(aux, 1, s);
        if (e != hipSuccess)
            return hip_fail(e, "forward launch");
        return SST_OK;
    }
    g.spec = 1;
    g.smin = reinterpret_cast<float *>(bd.ws + pl->off_smin);
    e = record_event(aux, 0, s);
    if (e == hipSuccess)
        e = sst::launch_forward(NF, pl->p.win_len, pl->n_src, pl->n_dst, kind, g, grid, s);
    if (e == hipSuccess)
        e = record_event(aux, 1, s);
    g.spec = 0;
    g.list = list;
    g.list_n = list_n;
    if (e == hipSuccess)
        e = sst::launch_spec_list(g, s);   // gamma, then the fix-up list
    if (e == hipSuccess)
        bd.gamma_valid = true;
    g.smin = nullptr;
    if (e == hipSuccess)
        e = sst::launch_forward(NF, pl->p.win_len, pl->n_src, pl->n_dst, kind, g, grid, s);
    if (e != hipSuccess)
        return hip_fail(e, "speculative forward launch");
    if (aux && aux->gamma) {
        e = hipMemcpyAsync(aux->gamma, &ctrl->gamma, sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync(gamma)");
    }
    return SST_OK;
}

static sst_status ridge_impl(sst_plan_t pl, const float *T, int64_t nframes, const int32_t *band,
                             const int32_t *centre, int32_t n_comp, int32_t *ridge, void *stream)
{
    if (!pl)
        return fail(SST_E_ARG, "plan is NULL");
    if (!pl->bd.ws)
        return fail(SST_E_STATE, "plan is not bound to a workspace");
    if (!T || !band || !ridge)
        return fail(SST_E_ARG, "T, band and ridge must not be NULL");
    if (n_comp < 1 || n_comp > 16)
        return fail(SST_E_ARG, "n_comp must lie in [1, 16]");
    if (nframes < 0 || nframes > pl->n_frames)
        return fail(SST_E_ARG, "nframes outside [0, n_frames]");
    for (int q = 0; q < n_comp; ++q)
        if (centre && (band[2 * q] < -pl->n_dst || band[2 * q + 1] > pl->n_dst))
            return fail(SST_E_ARG, "relative band outside [-n_dst, n_dst]");
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
    a.centre = centre;
    a.ridge = ridge;
    hipError_t e = sst::launch_ridge(a, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(e, "ridge launch");
    return SST_OK;
}

sst_status sst_ridge(sst_plan_t pl, const float *T, int64_t nframes, const int32_t *band,
                     int32_t n_comp, int32_t *ridge, void *stream)
{
    return ridge_impl(pl, T, nframes, band, nullptr, n_comp, ridge, stream);
}

sst_status sst_ridge_guided(sst_plan_t pl, const float *T, int64_t nframes, const int32_t *centre,
                            const int32_t *band, int32_t n_comp, int32_t *ridge, void *stream)
{
    if (!centre)
        return fail(SST_E_ARG, "centre must not be NULL");
    return ridge_impl(pl, T, nframes, band, centre, n_comp, ridge, stream);
}

sst_status sst_inverse(sst_plan_t pl, const float *T, int64_t frame0, int64_t nframes,
                       const int32_t *ridge, int32_t n_comp, int32_t hw, float *xhat,
                       const float *xref, double *err, uint32_t flags, void *stream)
{
    if (!pl)
        return fail(SST_E_ARG, "plan is NULL");
    if (!pl->bd.ws)
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
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    sst::InvDesc a = inv_desc(pl, T, frame0, nframes, ridge, n_comp, hw, xhat, xref, err,
                              accumulate);
    sst::InvDesc *slot = reinterpret_cast<sst::InvDesc *>(pl->bd.ws + pl->off_idesc);

    if (flags & SST_INV_EQ15) {
        if (pl->p.hop != 1)
            return fail(SST_E_ARG, "SST_INV_EQ15 needs hop == 1");
        a.span_lo = frame0;
        a.span_len = nframes;
        hipError_t e = sst::launch_put_inv_desc(a, slot, s);
        if (e == hipSuccess)
            e = sst::launch_inverse_eq15(a, slot, (float)(1.0 / (pl->p.nfft * pl->g0)), s);
        if (e != hipSuccess)
            return hip_fail(e, "inverse (Eq. 15) launch");
        return SST_OK;
    }
    if (a.span_len <= 0)
        return SST_OK;
    if (a.blk_end >= (int64_t(1) << 31))
        return fail(SST_E_UNSUPPORTED, "n_comp * ceil(span / 256) must be below 2^31");
    sst::InvLaunch l = inv_launch(slot, 1, a.blk0, inv_max_k(pl), pl->n_lo + pl->n_hi,
                                  pl->p.win_len, pl->p.hop * a.dec_row, pl->inv_tf,
                                  inv_groups_of(pl));
    if (sst::inv_lds_bytes(l) > (l.groups > 1 ? sst::inv_group_lds_max(l.groups) : 64 * 1024))
        return fail(SST_E_UNSUPPORTED, "inverse tiles need more than 64 KiB of LDS "
                                       "(window too long for the hop)");
    hipError_t e = sst::launch_put_inv_desc(a, slot, s);
    if (e == hipSuccess)
        e = sst::launch_inverse(l, a.blk_end - a.blk0, err != nullptr, s);
    if (e != hipSuccess)
        return hip_fail(e, "inverse launch");
    return SST_OK;
}

void sst_destroy(sst_plan_t pl) { delete pl; }

}  // extern "C"


// ---------------------------------------------------------------------------
// Tuning: launch choices, their measured search and a JSON cache.
// ---------------------------------------------------------------------------

namespace {

std::string tuning_key(const sst_plan_s *pl)
{
    char buf[160];
    std::snprintf(buf, sizeof buf, "gfx950 nfft=%d L=%d H=%d n_src=%d n_dst=%d prec=%d",
                  pl->p.nfft, pl->p.win_len, pl->p.hop, pl->n_src, pl->n_dst, pl->p.precision);
    return buf;
}

sst_status apply_tuning(sst_plan_s *pl, const sst_tuning &t)
{
    if (t.fwd_wg_per_cu < 0 || t.seed_step < 0)
        return fail(SST_E_ARG, "tuning values must be >= 0");
    if (t.inv_tf != 0 && t.inv_tf != 1 && t.inv_tf != sst::kInvWideTF &&
        t.inv_tf != sst::kInvXWideTF)
        return fail(SST_E_ARG, "inv_tf must be 0, 1, 4 or 8");
    if (t.inv_groups < 0 || t.inv_groups == 3 || t.inv_groups > 4)
        return fail(SST_E_ARG, "inv_groups must be 0, 1, 2 or 4");
    if (t.inv_tf == sst::kInvWideTF && !inv_wide_fits(pl))
        return fail(SST_E_UNSUPPORTED, "inv_tf 4: the frames 1024 output samples meet exceed "
                                       "the staged block");
    if (t.inv_tf == sst::kInvXWideTF && !inv_xwide_fits(pl))
        return fail(SST_E_UNSUPPORTED, "inv_tf 8: the frames 2048 output samples meet exceed "
                                       "the staged block, or the window table is too long");
    // grouped staging runs on tiles of four groups: the default width for it is 4
    const int tf = t.inv_tf ? t.inv_tf
                            : (t.inv_groups > 1 ? (inv_wide_fits(pl) ? sst::kInvWideTF : 1)
                                                : inv_default_tf(pl));
    if (t.inv_groups > 1 && !inv_groups_fit(pl, tf, t.inv_groups))
        return fail(SST_E_UNSUPPORTED, "inv_groups 2 / 4 need inv_tf 4, the hop-decimated window "
                                       "table and the staged groups within a third / half of "
                                       "the CU's LDS");
    pl->tune = t;
    pl->inv_tf = tf;
    if (pl->bd.ws)
        apply_grid(pl, pl->bd);
    return SST_OK;
}

// One cache line: "key": {"fwd_wg_per_cu": a, "seed_step": b, "inv_tf": c, "inv_groups": d}
bool parse_entry(const std::string &line, std::string &key, sst_tuning &t)
{
    const size_t q0 = line.find('"');
    if (q0 == std::string::npos)
        return false;
    const size_t q1 = line.find('"', q0 + 1);
    if (q1 == std::string::npos || line.find('{', q1) == std::string::npos)
        return false;
    key = line.substr(q0 + 1, q1 - q0 - 1);
    t = sst_tuning{};
    auto field = [&](const char *name, int32_t &v) {
        const size_t at = line.find(std::string("\"") + name + "\"", q1);
        if (at == std::string::npos)
            return false;
        const size_t colon = line.find(':', at);
        if (colon == std::string::npos)
            return false;
        v = (int32_t)std::strtol(line.c_str() + colon + 1, nullptr, 10);
        return true;
    };
    if (!field("inv_groups", t.inv_groups))   // absent from older caches: default
        t.inv_groups = 0;
    return field("fwd_wg_per_cu", t.fwd_wg_per_cu) && field("seed_step", t.seed_step) &&
           field("inv_tf", t.inv_tf);
}

bool read_cache(const char *path, std::vector<std::pair<std::string, sst_tuning>> &out)
{
    std::FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    char buf[1024];
    while (std::fgets(buf, sizeof buf, f)) {
        std::string key;
        sst_tuning t;
        if (parse_entry(buf, key, t))
            out.emplace_back(key, t);
    }
    std::fclose(f);
    return true;
}

}  // namespace

extern "C" {

sst_status sst_plan_get_tuning(sst_plan_t pl, sst_tuning *out)
{
    if (!pl || !out)
        return fail(SST_E_ARG, "plan or out is NULL");
    *out = pl->tune;
    if (pl->bd.ws && pl->bd.cus > 0)
        out->fwd_wg_per_cu = pl->bd.fwd_grid_cap / pl->bd.cus;
    out->inv_tf = pl->inv_tf;
    out->inv_groups = pl->inv_tf > 1 ? inv_groups_of(pl) : 1;
    return SST_OK;
}

sst_status sst_plan_set_tuning(sst_plan_t pl, const sst_tuning *t)
{
    if (!pl || !t)
        return fail(SST_E_ARG, "plan or tuning is NULL");
    return apply_tuning(pl, *t);
}

sst_status sst_tuning_load(sst_plan_t pl, const char *path)
{
    if (!pl || !path)
        return fail(SST_E_ARG, "plan or path is NULL");
    std::vector<std::pair<std::string, sst_tuning>> entries;
    if (!read_cache(path, entries))
        return fail(SST_E_ARG, std::string("cannot read tuning cache ") + path);
    const std::string key = tuning_key(pl);
    for (const auto &e : entries)
        if (e.first == key)
            return apply_tuning(pl, e.second);
    return fail(SST_E_ARG, "no tuning entry for " + key);
}

sst_status sst_tuning_save(sst_plan_t pl, const char *path)
{
    if (!pl || !path)
        return fail(SST_E_ARG, "plan or path is NULL");
    std::vector<std::pair<std::string, sst_tuning>> entries;
    read_cache(path, entries);   // a missing file starts an empty cache
    sst_tuning cur{};
    sst_plan_get_tuning(pl, &cur);
    const std::string key = tuning_key(pl);
    bool found = false;
    for (auto &e : entries)
        if (e.first == key) {
            e.second = cur;
            found = true;
        }
    if (!found)
        entries.emplace_back(key, cur);
    const std::string tmp = std::string(path) + ".tmp";
    std::FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f)
        return fail(SST_E_ARG, std::string("cannot write ") + tmp);
    std::fprintf(f, "{\n");
    for (size_t i = 0; i < entries.size(); ++i)
        std::fprintf(f,
                     "  \"%s\": {\"fwd_wg_per_cu\": %d, \"seed_step\": %d, \"inv_tf\": %d, "
                     "\"inv_groups\": %d}%s\n",
                     entries[i].first.c_str(), entries[i].second.fwd_wg_per_cu,
                     entries[i].second.seed_step, entries[i].second.inv_tf,
                     entries[i].second.inv_groups, i + 1 < entries.size() ? "," : "");
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0 && std::rename(tmp.c_str(), path) == 0;
    return ok ? SST_OK : fail(SST_E_ARG, std::string("cannot write ") + path);
}

sst_status sst_autotune(sst_plan_t pl, const float *x, float *T, const int32_t *ridge,
                        int32_t n_comp, int32_t hw, float *xhat, int32_t reps, void *stream,
                        sst_tuning *best)
{
    if (!pl)
        return fail(SST_E_ARG, "plan is NULL");
    if (!pl->bd.ws)
        return fail(SST_E_STATE, "plan is not bound to a workspace");
    if (!x || !T || reps < 1)
        return fail(SST_E_ARG, "x and T must not be NULL and reps >= 1");
    if (ridge && !xhat)
        return fail(SST_E_ARG, "the inverse choices need xhat");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess)
        e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) {
        if (ev[0])
            (void)hipEventDestroy(ev[0]);
        return hip_fail(e, "hipEventCreate");
    }
    sst_status st = SST_OK;
    // time reps calls of fn after one untimed call; ms per call, < 0 on error
    // mean time of one call: once untimed, then reps calls; when those take
    // under 20 ms in all, again over as many calls as fill about 20 ms (at
    // most 1000), so that short calls are not timed at the events' noise
    auto timed = [&](auto fn) -> float {
        if ((st = fn()) != SST_OK)
            return -1.f;
        auto run = [&](int n) -> float {
            hipError_t he = hipEventRecord(ev[0], s);
            for (int r = 0; r < n && st == SST_OK && he == hipSuccess; ++r)
                st = fn();
            if (he == hipSuccess)
                he = hipEventRecord(ev[1], s);
            if (he == hipSuccess)
                he = hipEventSynchronize(ev[1]);
            float ms = 0.f;
            if (he == hipSuccess)
                he = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (he != hipSuccess && st == SST_OK)
                st = hip_fail(he, "autotune timing");
            return st == SST_OK ? ms : -1.f;
        };
        const float ms = run(reps);
        if (ms < 0.f || ms >= 20.f)
            return ms < 0.f ? -1.f : ms / reps;
        const float per = ms / reps;
        const int n = per > 0.02f ? std::min(1000, (int)(20.f / per) + 1) : 1000;
        const float ms2 = run(n);
        return ms2 < 0.f ? -1.f : ms2 / n;
    };
    sst_tuning cur = pl->tune;
    sst_tuning chosen = cur;
    // forward: resident workgroups per CU x seed step of the speculative threshold
    const int occ = pl->bd.fwd_occ > 0 ? pl->bd.fwd_occ : 1;
    float best_ms = -1.f;
    // seed steps: frame groups of the FFT tier; GEMM tiles (1 = the exact
    // maximum first, so no tile is redone)
    const int seeds_fft[3] = {0, 16, 128}, seeds_gemm[3] = {0, 1, 4};
    const int *seeds = pl->gemm_ft ? seeds_gemm : seeds_fft;
    for (int wg = occ; wg >= 1 && wg >= occ - 2 && st == SST_OK; --wg)
        for (int si = 0; si < 3; ++si) {
            const int seed = seeds[si];
            sst_tuning t = cur;
            t.fwd_wg_per_cu = wg;
            t.seed_step = seed;
            if ((st = apply_tuning(pl, t)) != SST_OK)
                break;
            const float ms = timed([&] {
                return forward_impl(pl, pl->bd, x, 0, pl->n_frames, T, nullptr, 0, stream);
            });
            if (ms < 0.f)
                break;
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                chosen.fwd_wg_per_cu = wg;
                chosen.seed_step = seed;
            }
        }
    // inverse: tile width, and the grouped staging of the wide tiles
    if (st == SST_OK && ridge) {
        float best_inv = -1.f;
        const int choices[5][2] = {{1, 1}, {sst::kInvWideTF, 1}, {sst::kInvWideTF, 2},
                                   {sst::kInvWideTF, 4}, {sst::kInvXWideTF, 1}};
        for (const auto &ch : choices) {
            const int tf = ch[0], gr = ch[1];
            if (tf == sst::kInvWideTF && !inv_wide_fits(pl))
                continue;
            if (tf == sst::kInvXWideTF && !inv_xwide_fits(pl))
                continue;
            if (gr > 1 && !inv_groups_fit(pl, tf, gr))
                continue;
            sst_tuning t = chosen;
            t.inv_tf = tf;
            t.inv_groups = gr;
            if ((st = apply_tuning(pl, t)) != SST_OK)
                break;
            const float ms = timed([&] {
                return sst_inverse(pl, T, 0, pl->n_frames, ridge, n_comp, hw, xhat, nullptr,
                                   nullptr, 0, stream);
            });
            if (ms < 0.f)
                break;
            if (best_inv < 0.f || ms < best_inv) {
                best_inv = ms;
                chosen.inv_tf = tf;
                chosen.inv_groups = gr;
            }
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    const sst_status st_apply = apply_tuning(pl, st == SST_OK ? chosen : cur);
    if (st != SST_OK)
        return st;
    if (st_apply != SST_OK)
        return st_apply;
    if (best)
        sst_plan_get_tuning(pl, best);
    return SST_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form.  Every channel keeps its own plan (tables, shapes); the batch
// workspace holds each channel's plan workspace, then one descriptor array
// per launch group (channels sharing N_f and the pass-1 tap-row count) for
// the forward and threshold kernels and one InvDesc array for the inverse.
// ---------------------------------------------------------------------------

struct sst_batch_s {
    struct Io {
        const float *x = nullptr;
        float *T = nullptr;
        const int32_t *ridge = nullptr;
        int n_comp = 0, hw = 0;
        float *xhat = nullptr;
        const float *xref = nullptr;
        double *err = nullptr;
    };
    struct Group {
        int nfft = 0, nz = 0;
        std::vector<int> chans;     // ascending channel indices
        int max_L = 0, max_n_src = 0, max_n_dst = 0;
        size_t off_desc = 0;        // ChanDesc[chans.size()]
        std::vector<sst::ChanDesc> desc;
        int fwd_grid_cap = 0;
        // speculative forward: least kept |S|^2 per item of the group, fix-up list
        int64_t n_items = 0;
        size_t off_smin = 0, off_list = 0, off_list_n = 0;
    };
    std::vector<sst_plan_s *> plans;
    std::vector<Io> io;
    std::vector<Group> groups;
    std::vector<size_t> off_chan;
    size_t off_idesc = 0, ws_bytes = 0;
    // one per channel: the channels with one sample group per inverse
    // workgroup first, then those with wide tiles, each in channel order
    // (every inverse launch covers a contiguous run of one kind)
    std::vector<sst::InvDesc> idesc;
    std::vector<int> inv_pos;          // channel -> index in idesc
    unsigned char *ws = nullptr;
    bool committed = false;
    // per channel: a thresholding batched forward has set its gamma since the bind
    std::vector<char> gamma_valid;
    ~sst_batch_s()
    {
        for (sst_plan_s *p : plans)
            delete p;
    }
};

namespace {

int nz_rows_host(int nfft, int L)
{
    const int q = nfft / 16;
    const int rows = (L + q - 1) / q;
    return rows <= 4 ? 4 : (rows <= 8 ? 8 : 16);
}

}  // namespace

extern "C" {

sst_status sst_batch_plan(const sst_params *params, int32_t n_channels, sst_batch_t *out)
{
    if (!out)
        return fail(SST_E_ARG, "out is NULL");
    *out = nullptr;
    if (!params || n_channels < 1)
        return fail(SST_E_ARG, "params NULL or n_channels < 1");
    sst_batch_s *b = new (std::nothrow) sst_batch_s();
    if (!b)
        return fail(SST_E_NOMEM, "batch allocation failed");
    try {
        b->plans.assign((size_t)n_channels, nullptr);
        b->io.assign((size_t)n_channels, sst_batch_s::Io{});
        b->off_chan.assign((size_t)n_channels, 0);
    } catch (...) {
        delete b;
        return fail(SST_E_NOMEM, "batch allocation failed");
    }
    size_t off = 0;
    for (int c = 0; c < n_channels; ++c) {
        if (params[c].precision != SST_PREC_FP32_FFT) {
            delete b;
            return fail(SST_E_UNSUPPORTED, "channel " + std::to_string(c) +
                                               ": the batched calls run the FP32 FFT tier only");
        }
        sst_status st = sst_plan(&params[c], &b->plans[(size_t)c]);
        if (st != SST_OK) {
            g_err = "channel " + std::to_string(c) + ": " + g_err;
            delete b;
            return st;
        }
        b->off_chan[(size_t)c] = off;
        off = align_up(off + b->plans[(size_t)c]->ws_bytes);
    }
    for (int c = 0; c < n_channels; ++c) {
        const sst_plan_s *pl = b->plans[(size_t)c];
        const int nz = nz_rows_host(pl->p.nfft, pl->p.win_len);
        sst_batch_s::Group *grp = nullptr;
        for (auto &gr : b->groups)
            if (gr.nfft == pl->p.nfft && gr.nz == nz)
                grp = &gr;
        if (!grp) {
            b->groups.emplace_back();
            grp = &b->groups.back();
            grp->nfft = pl->p.nfft;
            grp->nz = nz;
        }
        grp->chans.push_back(c);
        grp->max_L = std::max(grp->max_L, pl->p.win_len);
        grp->max_n_src = std::max(grp->max_n_src, pl->n_src);
        grp->max_n_dst = std::max(grp->max_n_dst, pl->n_dst);
    }
    for (auto &gr : b->groups) {
        gr.off_desc = off;
        off = align_up(off + sizeof(sst::ChanDesc) * gr.chans.size());
        for (int c : gr.chans)
            gr.n_items += b->plans[(size_t)c]->n_items;
        gr.off_smin = off;
        off = align_up(off + sizeof(float) * (size_t)gr.n_items);
        gr.off_list = off;
        off = align_up(off + sizeof(int32_t) * (size_t)gr.n_items);
        gr.off_list_n = off;
        off = align_up(off + sizeof(int32_t));
    }
    b->off_idesc = off;
    off = align_up(off + sizeof(sst::InvDesc) * (size_t)n_channels);
    b->ws_bytes = off;
    *out = b;
    return SST_OK;
}

sst_status sst_batch_query(sst_batch_t b, int32_t c, sst_shape *out)
{
    if (!b || !out)
        return fail(SST_E_ARG, "batch or out is NULL");
    if (c < 0 || c >= (int32_t)b->plans.size())
        return fail(SST_E_ARG, "channel out of range");
    sst_status st = sst_plan_query(b->plans[(size_t)c], out);
    out->workspace_bytes = b->ws_bytes;
    return st;
}

sst_status sst_batch_bind(sst_batch_t b, void *workspace, size_t bytes, void *stream)
{
    if (!b)
        return fail(SST_E_ARG, "batch is NULL");
    if (!workspace || bytes < b->ws_bytes || (reinterpret_cast<uintptr_t>(workspace) % kAlign))
        return fail(SST_E_WORKSPACE, "workspace NULL, not 256-byte aligned, or smaller than "
                                     "sst_shape.workspace_bytes");
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    for (size_t c = 0; c < b->plans.size(); ++c) {
        sst_plan_s *pl = b->plans[c];
        sst_status st = sst_plan_bind(pl, ws + b->off_chan[c], pl->ws_bytes, stream);
        if (st != SST_OK)
            return st;
    }
    for (auto &gr : b->groups) {
        const sst_plan_s *p0 = b->plans[(size_t)gr.chans[0]];
        gr.fwd_grid_cap = p0->bd.fwd_grid_cap;
        for (int c : gr.chans) {
            gr.fwd_grid_cap = std::max(gr.fwd_grid_cap, b->plans[(size_t)c]->bd.fwd_grid_cap);
        }
    }
    b->ws = ws;
    b->committed = false;
    b->gamma_valid.assign(b->plans.size(), 0);
    return SST_OK;
}

sst_status sst_batch_set_io(sst_batch_t b, int32_t c, const float *x, float *T,
                            const int32_t *ridge, int32_t n_comp, int32_t hw, float *xhat,
                            const float *xref, double *err)
{
    if (!b)
        return fail(SST_E_ARG, "batch is NULL");
    if (c < 0 || c >= (int32_t)b->plans.size())
        return fail(SST_E_ARG, "channel out of range");
    if (ridge && (n_comp < 1 || n_comp > 65535 || hw < 0 || hw > 512 || !xhat))
        return fail(SST_E_ARG, "inverse buffers need 1 <= n_comp <= 65535, 0 <= hw <= 512 and xhat");
    if (err && !xref)
        return fail(SST_E_ARG, "err needs xref");
    sst_batch_s::Io &o = b->io[(size_t)c];
    o.x = x;
    o.T = T;
    o.ridge = ridge;
    o.n_comp = ridge ? n_comp : 0;
    o.hw = hw;
    o.xhat = xhat;
    o.xref = xref;
    o.err = err;
    b->committed = false;
    return SST_OK;
}

sst_status sst_batch_commit(sst_batch_t b, void *stream)
{
    if (!b)
        return fail(SST_E_ARG, "batch is NULL");
    if (!b->ws)
        return fail(SST_E_STATE, "batch is not bound to a workspace");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (auto &gr : b->groups) {
        gr.desc.assign(gr.chans.size(), sst::ChanDesc{});
        int64_t items = 0, mitems = 0;
        for (size_t i = 0; i < gr.chans.size(); ++i) {
            const int c = gr.chans[i];
            const sst_plan_s *pl = b->plans[(size_t)c];
            const sst_batch_s::Io &o = b->io[(size_t)c];
            const int F = sst::fwd_frames_per_iter(pl->p.nfft);
            sst::ChanDesc d = chan_desc(pl, pl->bd.ws, o.x, 0, pl->n_frames, o.T, nullptr,
                                        reinterpret_cast<sst::Ctrl *>(pl->bd.ws));
            d.item0 = items;
            items += (pl->n_frames + F - 1) / F;
            d.item_end = items;
            d.mitem0 = mitems;
            if (pl->p.thr_mode == SST_THR_REL_MAX)
                mitems += (pl->n_frames + F - 1) / F;   // max-only pre-pass: forward items
            d.mitem_end = mitems;
            gr.desc[i] = d;
        }
        hipError_t e = hipMemcpyAsync(b->ws + gr.off_desc, gr.desc.data(),
                                      sizeof(sst::ChanDesc) * gr.desc.size(),
                                      hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync(descriptors)");
    }
    b->idesc.assign(b->plans.size(), sst::InvDesc{});
    b->inv_pos.assign(b->plans.size(), 0);
    size_t pos = 0;
    for (int kind = 0; kind < kInvKinds; ++kind) {
        int64_t blk = 0;
        for (size_t c = 0; c < b->plans.size(); ++c) {
            const sst_plan_s *pl = b->plans[c];
            if (inv_kind_of(pl) != kind)
                continue;
            const sst_batch_s::Io &o = b->io[c];
            sst::InvDesc a = inv_desc(pl, o.T, 0, pl->n_frames, o.ridge, o.ridge ? o.n_comp : 0,
                                      o.hw, o.xhat, o.xref, o.err, false);
            a.blk0 = blk;
            blk += o.ridge ? (int64_t)o.n_comp * a.tiles : 0;
            a.blk_end = blk;
            b->idesc[pos] = a;
            b->inv_pos[c] = (int)pos++;
        }
    }
    hipError_t e = hipMemcpyAsync(b->ws + b->off_idesc, b->idesc.data(),
                                  sizeof(sst::InvDesc) * b->idesc.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(inverse descriptors)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "hipStreamSynchronize");
    b->committed = true;
    return SST_OK;
}

sst_status sst_batch_forward(sst_batch_t b, int32_t c_begin, int32_t c_end, uint32_t flags,
                             void *stream)
{
    if (!b)
        return fail(SST_E_ARG, "batch is NULL");
    if (!b->ws || !b->committed)
        return fail(SST_E_STATE, "batch not bound or buffers not committed");
    if (c_begin < 0 || c_end > (int32_t)b->plans.size() || c_begin >= c_end)
        return fail(SST_E_ARG, "channel range empty or outside [0, n_channels)");
    if (flags & ~SST_FWD_REUSE_GAMMA)
        return fail(SST_E_ARG, "unknown forward flags");
    for (int c = c_begin; c < c_end; ++c) {
        if (!b->io[(size_t)c].x || !b->io[(size_t)c].T)
            return fail(SST_E_ARG, "channel " + std::to_string(c) + " has no x or T");
        if ((flags & SST_FWD_REUSE_GAMMA) && !b->gamma_valid[(size_t)c])
            return fail(SST_E_STATE, "channel " + std::to_string(c) + ": SST_FWD_REUSE_GAMMA "
                                     "before any thresholding forward call on this binding");
    }
    if (!(flags & SST_FWD_REUSE_GAMMA))
        for (int c = c_begin; c < c_end; ++c)
            b->gamma_valid[(size_t)c] = 0;   // set again once every launch is queued
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (const auto &gr : b->groups) {
        size_t i0 = 0, i1 = 0;
        while (i0 < gr.chans.size() && gr.chans[i0] < c_begin)
            ++i0;
        i1 = i0;
        while (i1 < gr.chans.size() && gr.chans[i1] < c_end)
            ++i1;
        if (i1 == i0)
            continue;
        const sst_plan_s *p0 = b->plans[(size_t)gr.chans[i0]];
        sst::GroupLaunch g{};
        g.ch = reinterpret_cast<const sst::ChanDesc *>(b->ws + gr.off_desc) + i0;
        g.n_ch = (int)(i1 - i0);
        g.twid = reinterpret_cast<const float2 *>(p0->bd.ws + p0->off_twid);
        // Speculative forward (see sst_forward): the maximum over every
        // kSeedStep-th item, the forward at the lower bound of gamma it gives,
        // gamma, then the items whose decisions the final gamma changes.
        const bool spec = !(flags & SST_FWD_REUSE_GAMMA);
        int32_t *list = reinterpret_cast<int32_t *>(b->ws + gr.off_list);
        int32_t *list_n = reinterpret_cast<int32_t *>(b->ws + gr.off_list_n);
        hipError_t e = hipSuccess;
        if (spec) {
            g.list_n = list_n;
            e = sst::launch_clear_max(g, s);
            g.list_n = nullptr;
            g.item_begin = gr.desc[i0].mitem0;
            g.item_stop = gr.desc[i1 - 1].mitem_end;
            // one step over the launch's items, as dense as the densest of the
            // channels' own single-call seeds: every channel's running maximum
            // starts at least as close to its final one as in a single call
            int64_t step = INT64_MAX;
            for (size_t i = i0; i < i1; ++i)
                step = std::min(step, seed_step(gr.desc[i].mitem_end - gr.desc[i].mitem0,
                                                gr.fwd_grid_cap,
                                                b->plans[(size_t)gr.chans[i]]->tune.seed_step));
            g.step = (int)step;
            const int64_t visits = (g.item_stop - g.item_begin + g.step - 1) / g.step;
            const int grid = (int)(visits < gr.fwd_grid_cap ? visits : gr.fwd_grid_cap);
            if (e == hipSuccess)
                e = sst::launch_max_prepass(gr.nfft, gr.max_L, g, grid, s);
            g.step = 0;
            if (e != hipSuccess)
                return hip_fail(e, "batched threshold launch");
        }
        g.item_begin = gr.desc[i0].item0;
        g.item_stop = gr.desc[i1 - 1].item_end;
        const int64_t items = g.item_stop - g.item_begin;
        const int grid = (int)(items < gr.fwd_grid_cap ? items : gr.fwd_grid_cap);
        if (grid <= 0) {
            if (spec && (e = sst::launch_gamma(g, s)) != hipSuccess)
                return hip_fail(e, "batched threshold launch");
            continue;
        }
        g.spec = spec ? 1 : 0;
        g.smin = spec ? reinterpret_cast<float *>(b->ws + gr.off_smin) : nullptr;
        e = sst::launch_forward(gr.nfft, gr.max_L, gr.max_n_src, gr.max_n_dst, sst::kFwdKindPlain,
                                    g, grid, s);
        g.spec = 0;
        if (spec) {
            g.list = list;
            g.list_n = list_n;
            if (e == hipSuccess)
                e = sst::launch_spec_list(g, s);
            g.smin = nullptr;
            if (e == hipSuccess)
                e = sst::launch_forward(gr.nfft, gr.max_L, gr.max_n_src, gr.max_n_dst,
                                        sst::kFwdKindPlain, g,
                                        grid, s);
        }
        if (e != hipSuccess)
            return hip_fail(e, "batched forward launch");
    }
    if (!(flags & SST_FWD_REUSE_GAMMA))
        for (int c = c_begin; c < c_end; ++c)
            b->gamma_valid[(size_t)c] = 1;
    return SST_OK;
}

sst_status sst_batch_inverse(sst_batch_t b, int32_t c_begin, int32_t c_end, void *stream)
{
    if (!b)
        return fail(SST_E_ARG, "batch is NULL");
    if (!b->ws || !b->committed)
        return fail(SST_E_STATE, "batch not bound or buffers not committed");
    if (c_begin < 0 || c_end > (int32_t)b->plans.size() || c_begin >= c_end)
        return fail(SST_E_ARG, "channel range empty or outside [0, n_channels)");
    for (int c = c_begin; c < c_end; ++c) {
        const sst_batch_s::Io &o = b->io[(size_t)c];
        if (!o.T || !o.ridge || !o.xhat)
            return fail(SST_E_ARG, "channel " + std::to_string(c) + " has no T, ridge or xhat");
        if (b->plans[(size_t)c]->G > 65536)
            return fail(SST_E_UNSUPPORTED, "inverse needs subdiv * nfft <= 65536");
        if (b->idesc[(size_t)b->inv_pos[(size_t)c]].blk_end -
                b->idesc[(size_t)b->inv_pos[(size_t)c]].blk0 >= (int64_t(1) << 31))
            return fail(SST_E_UNSUPPORTED, "n_comp * ceil(n_samples / 256) must be below 2^31");
    }
    const sst::InvDesc *dev = reinterpret_cast<const sst::InvDesc *>(b->ws + b->off_idesc);
    // one launch per kind of tile: the range's channels of that kind are a
    // contiguous run of the descriptor array
    for (int kind = 0; kind < kInvKinds; ++kind) {
        int p0 = -1, p1 = -1;
        int max_k = 2, max_tab = 1, max_L = 1, max_dec = 1;
        bool any_err = false;
        for (int c = c_begin; c < c_end; ++c) {
            const sst_plan_s *pl = b->plans[(size_t)c];
            if (inv_kind_of(pl) != kind)
                continue;
            const int pos = b->inv_pos[(size_t)c];
            if (p0 < 0)
                p0 = pos;
            p1 = pos;
            max_k = std::max(max_k, inv_max_k(pl));
            max_tab = std::max(max_tab, pl->n_lo + pl->n_hi);
            max_L = std::max(max_L, pl->p.win_len);
            max_dec = std::max(max_dec, pl->p.hop * b->idesc[(size_t)pos].dec_row);
            any_err = any_err || b->io[(size_t)c].err;
        }
        if (p0 < 0)
            continue;
        sst::InvLaunch l = inv_launch(dev + p0, p1 - p0 + 1, b->idesc[(size_t)p0].blk0, max_k,
                                      max_tab, max_L, max_dec, inv_kind_tf(kind),
                                      kind == 3 ? 4 : (kind == 2 ? 2 : 1));
        // grouped tiles of several channels may need more than one channel's
        // LDS (the maxima of different channels); up to the CU's 160 KiB
        if (sst::inv_lds_bytes(l) > ((kind == 2 || kind == 3) ? 160 * 1024 : 64 * 1024))
            return fail(SST_E_UNSUPPORTED, "inverse tiles need more than 64 KiB of LDS "
                                           "(window too long for the hop)");
        const int64_t blocks = b->idesc[(size_t)p1].blk_end - l.blk_begin;
        if (blocks >= (int64_t(1) << 31))
            return fail(SST_E_UNSUPPORTED, "the channel range needs 2^31 or more inverse tiles; "
                                           "split it over several calls");
        hipError_t e = sst::launch_inverse(l, blocks, any_err,
                                           reinterpret_cast<hipStream_t>(stream));
        if (e != hipSuccess)
            return hip_fail(e, "batched inverse launch");
    }
    return SST_OK;
}

void sst_batch_destroy(sst_batch_t b) { delete b; }


sst_status sst_stft(sst_plan_t pl, const float *x, int64_t frame0, int64_t nframes, float *S,
                    float *Sd, void *stream)
{
    if (!pl)
        return fail(SST_E_ARG, "plan is NULL");
    if (!pl->bd.ws)
        return fail(SST_E_STATE, "plan is not bound to a workspace");
    if (!x || !S)
        return fail(SST_E_ARG, "x and S must not be NULL");
    if (frame0 < 0 || nframes < 0 || frame0 + nframes > pl->n_frames)
        return fail(SST_E_ARG, "frame range outside [0, n_frames)");
    if (nframes == 0)
        return SST_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int F = sst::fwd_frames_per_iter(pl->p.nfft);
    sst_fwd_aux aux{};
    aux.S = S;
    aux.Sd = Sd;
    sst::ChanDesc d = chan_desc(pl, pl->bd.ws, x, frame0, nframes, nullptr, &aux,
                                reinterpret_cast<sst::Ctrl *>(pl->bd.ws));
    d.item0 = 0;
    d.item_end = (nframes + F - 1) / F;
    sst::ChanDesc *slot = reinterpret_cast<sst::ChanDesc *>(pl->bd.ws + pl->off_desc);
    hipError_t e = sst::launch_put_desc(d, slot, false, nullptr, s);
    sst::GroupLaunch g{};
    g.ch = slot;
    g.n_ch = 1;
    g.twid = reinterpret_cast<const float2 *>(pl->bd.ws + pl->off_twid);
    g.item_begin = 0;
    g.item_stop = d.item_end;
    const int grid = (int)(d.item_end < pl->bd.fwd_grid_cap ? d.item_end : pl->bd.fwd_grid_cap);
    if (e == hipSuccess)
        e = sst::launch_stft(pl->p.nfft, pl->p.win_len, g, grid, s);
    if (e != hipSuccess)
        return hip_fail(e, "STFT launch");
    return SST_OK;
}

sst_status sst_stft_inverse(sst_plan_t pl, const float *S, float *xhat, void *stream)
{
    if (!pl)
        return fail(SST_E_ARG, "plan is NULL");
    if (!pl->bd.ws)
        return fail(SST_E_STATE, "plan is not bound to a workspace");
    if (!S || !xhat)
        return fail(SST_E_ARG, "S and xhat must not be NULL");
    sst::SynArgs a{};
    a.S = reinterpret_cast<const float2 *>(S);
    a.win = reinterpret_cast<const float2 *>(pl->bd.ws + pl->off_win);
    a.den2 = reinterpret_cast<const float *>(pl->bd.ws + pl->off_den2);
    a.twid = reinterpret_cast<const float2 *>(pl->bd.ws + pl->off_twid);
    a.xhat = xhat;
    a.n = pl->p.n_samples;
    a.n_frames = pl->n_frames;
    a.M = pl->M;
    a.hop = pl->p.hop;
    a.k1 = pl->k1;
    a.k2 = pl->k2;
    a.n_src = pl->n_src;
    a.inv_nfft = (float)(1.0 / pl->p.nfft);
    hipError_t e = sst::launch_synthesis(pl->p.nfft, a, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(e, "STFT synthesis launch");
    return SST_OK;
}

sst_status sst_renyi(const void *C, int32_t kind, int64_t rows, int32_t cols, int64_t ld,
                     int32_t alpha, double *work, double *out, void *stream)
{
    if (!C || !work || !out)
        return fail(SST_E_ARG, "C, work and out must not be NULL");
    if (kind < SST_RENYI_COMPLEX64 || kind > SST_RENYI_MAG_F16)
        return fail(SST_E_ARG, "unknown kind");
    if (rows < 1 || cols < 1 || ld < cols)
        return fail(SST_E_ARG, "need rows >= 1, cols >= 1 and ld >= cols");
    if (alpha < 2 || alpha > 4)
        return fail(SST_E_ARG, "alpha must be an integer in [2, 4]");
    static_assert(2 * sst::kRenyiParts <= SST_RENYI_WORK_DOUBLES, "work holds the partials");
    sst::RenyiArgs a{};
    a.C = C;
    a.rows = rows;
    a.ld = ld;
    a.cols = cols;
    a.alpha = alpha;
    a.work = work;
    a.out = out;
    hipError_t e = sst::launch_renyi(a, kind, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(e, "Renyi launch");
    return SST_OK;
}

const char *sst_status_string(sst_status s)
{
    switch (s) {
    case SST_OK: return "SST_OK";
    case SST_E_ARG: return "SST_E_ARG: invalid argument";
    case SST_E_UNSUPPORTED: return "SST_E_UNSUPPORTED: valid for the method, not supported by the library";
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
