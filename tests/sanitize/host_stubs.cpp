// Host-only stand-ins for the device launchers of the HIP library, so that the
// host runtime (sst_host.cpp: validation, float64 tables, workspace layout,
// tuning cache, batch planning) can be built with AddressSanitizer and
// UndefinedBehaviorSanitizer by a plain host compiler and run without a GPU.
// Every launcher reports "no device"; the geometry helpers return the values
// the host layout needs.  Test infrastructure only.
#include "sst_internal.h"

namespace sst {

hipError_t launch_clear_max(const GroupLaunch &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_max_prepass(int, int, const GroupLaunch &, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_gamma(const GroupLaunch &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_spec_list(const GroupLaunch &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_forward(int, int, int, int, int, const GroupLaunch &, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_gemm_forward(int, int, bool, const GemmArgs &, int, hipStream_t) { return hipErrorNoDevice; }
size_t gemm_lds_bytes(int, int, int, int, int) { return 16384; }   // fits: the plan proceeds
int gemm_occupancy(int, int, size_t) { return 1; }
hipError_t launch_put_desc(const ChanDesc &, ChanDesc *, bool, int32_t *, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_inverse(const InvLaunch &, int64_t, bool, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_inverse_eq15(const InvDesc &, const InvDesc *, float, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_put_inv_desc(const InvDesc &, InvDesc *, hipStream_t) { return hipErrorNoDevice; }
size_t inv_lds_bytes(const InvLaunch &) { return 0; }
hipError_t launch_ridge(const RidgeArgs &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_synthesis(int, const SynArgs &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_stft(int, int, const GroupLaunch &, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_renyi(const RenyiArgs &, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t static_scratch(int, unsigned char **out) { *out = nullptr; return hipErrorNoDevice; }
int fwd_frames_per_iter(int nfft) { return nfft >= 4096 ? 1 : 4096 / nfft; }
int fwd_threads(int nfft) { return nfft > 4096 ? nfft / 16 : 256; }
int fwd_lds_elems(int nfft) { const int v = nfft > 4096 ? nfft : 4096; return v + v / 16; }
int fwd_occupancy(int, int) { return 1; }
int fwd_rounds(int, int) { return 9; }
size_t fwd_lds_bytes(int nfft) { return 8 * (size_t)fwd_lds_elems(nfft); }

}  // namespace sst
