// Exercises the host paths of the C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (no GPU): plans of every DFT size and tier,
// custom windows, invalid parameters, queries, batches, the tuning cache,
// the refusals of calls that need a device.  Exit status 0 when every
// expectation holds.  Test infrastructure only.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sst.h"

static int failures = 0;
#define EXPECT(c)                                                          \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "expectation failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static sst_params params(int nfft, int L, double sigma, int hop, double f_lo, double f_hi, int z,
                         int prec)
{
    sst_params p;
    std::memset(&p, 0, sizeof p);
    p.struct_size = sizeof(sst_params);
    p.n_samples = 1 << 16;
    p.fs = 25600.0;
    p.win_len = L;
    p.sigma = sigma;
    p.hop = hop;
    p.nfft = nfft;
    p.f_lo = f_lo;
    p.f_hi = f_hi;
    p.subdiv = z;
    p.thr_mode = SST_THR_REL_MAX;
    p.thr = 1e-3;
    p.precision = prec;
    return p;
}

int main(int argc, char **argv)
{
    const char *cache = argc > 1 ? argv[1] : "sanitize_tune.json";
    // every DFT size, both GEMM tiers, bands with k1 > 0
    for (int nfft : {512, 1024, 2048, 4096, 8192})
        for (int prec : {SST_PREC_FP32_FFT, SST_PREC_GEMM_BF16, SST_PREC_GEMM_F16X3}) {
            if (prec != SST_PREC_FP32_FFT && nfft > 2048)
                continue;
            sst_params p = params(nfft, nfft / 2 - 1, nfft / 16.0, 8, 300.0, 6000.0, 3, prec);
            sst_plan_t pl = nullptr;
            EXPECT(sst_plan(&p, &pl) == SST_OK);
            sst_shape sh;
            EXPECT(sst_plan_query(pl, &sh) == SST_OK);
            EXPECT(sh.n_dst == 3 * (sh.k2 - sh.k1) + 1 && sh.workspace_bytes % 256 == 0);
            sst_tuning t;
            EXPECT(sst_plan_get_tuning(pl, &t) == SST_OK);
            t.seed_step = 16;
            EXPECT(sst_plan_set_tuning(pl, &t) == SST_OK);
            EXPECT(sst_tuning_save(pl, cache) == SST_OK);
            EXPECT(sst_tuning_load(pl, cache) == SST_OK);
            // calls that need a bound plan refuse cleanly
            float dummy = 0.f;
            EXPECT(sst_forward(pl, &dummy, 0, 1, &dummy, nullptr, 0, nullptr) == SST_E_STATE);
            EXPECT(sst_stft(pl, &dummy, 0, 1, &dummy, nullptr, nullptr) == SST_E_STATE);
            EXPECT(sst_plan_bind(pl, nullptr, 0, nullptr) == SST_E_WORKSPACE);
            sst_destroy(pl);
        }
    // custom window
    {
        sst_params p = params(1024, 255, 32.0, 4, 0.0, 12800.0, 1, SST_PREC_FP32_FFT);
        std::vector<double> g(255), gd(255);
        for (int j = 0; j < 255; ++j) {
            g[j] = 1.0 - std::abs(j - 127) / 128.0;
            gd[j] = j < 127 ? 1.0 / 128.0 : -1.0 / 128.0;
        }
        p.window = g.data();
        p.dwindow = gd.data();
        sst_plan_t pl = nullptr;
        EXPECT(sst_plan(&p, &pl) == SST_OK);
        sst_destroy(pl);
    }
    // invalid parameters: every check returns an error and a message
    {
        sst_params bad = params(4096, 1024, 128.0, 16, 0.0, 6400.0, 4, SST_PREC_FP32_FFT);
        sst_plan_t pl = nullptr;
        EXPECT(sst_plan(&bad, &pl) == SST_E_ARG && pl == nullptr);
        EXPECT(std::strlen(sst_last_error()) > 0);
        bad = params(16384, 1023, 128.0, 16, 0.0, 6400.0, 4, SST_PREC_FP32_FFT);
        EXPECT(sst_plan(&bad, &pl) == SST_E_UNSUPPORTED);
        bad = params(8192, 8191, 900.0, 16, 0.0, 12800.0, 1, SST_PREC_GEMM_BF16);   // table > 64 MiB
        EXPECT(sst_plan(&bad, &pl) == SST_E_UNSUPPORTED && pl == nullptr);
        EXPECT(sst_plan(nullptr, &pl) == SST_E_ARG);
        EXPECT(std::strlen(sst_status_string(-99)) > 0);
    }
    // batch of mixed channels
    {
        std::vector<sst_params> ps;
        for (int c = 0; c < 12; ++c)
            ps.push_back(params(1024 << (c % 3), (256 << (c % 3)) - 1, 8.0 * (1 << (c % 3)),
                                4 << (c % 4), 0.0, 6400.0, 2 + (c % 2) * 2, SST_PREC_FP32_FFT));
        sst_batch_t b = nullptr;
        EXPECT(sst_batch_plan(ps.data(), (int)ps.size(), &b) == SST_OK);
        sst_shape sh;
        for (int c = 0; c < 12; ++c)
            EXPECT(sst_batch_query(b, c, &sh) == SST_OK);
        EXPECT(sst_batch_query(b, 12, &sh) == SST_E_ARG);
        float dummy = 0.f;
        EXPECT(sst_batch_set_io(b, 3, &dummy, &dummy, nullptr, 0, 0, nullptr, nullptr, nullptr) ==
               SST_OK);
        EXPECT(sst_batch_forward(b, 0, 12, 0, nullptr) == SST_E_STATE);
        sst_batch_destroy(b);
    }
    double e38 = 0, e46 = 0;
    EXPECT(sst_critical_hf(9035089.0, 0.02, 44100.0, &e38, &e46) == SST_OK && e38 > 2445.0);
    EXPECT(sst_renyi(nullptr, 0, 1, 1, 1, 3, nullptr, nullptr, nullptr) == SST_E_ARG);
    std::printf("host driver: %d failure(s)\n", failures);
    return failures == 0 ? 0 : 1;
}
