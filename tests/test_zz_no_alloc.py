"""sst_forward_static (the entry point that allocates nothing: its workspace is
the library's fixed per-device scratch) against sst_forward on a plan bound to
a caller-allocated workspace, through the C ABI: T, gamma and the debug
outputs are equal bit for bit, on two calls in a row, the second with a
smaller input, and a chunked call reusing the static call's gamma."""
import numpy as np
import pytest

from workloads import SSTConfig

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    ("c2-shape", 1 << 15, SSTConfig(25600.0, 1023, 128.0, 16, 4096, 0.0, 6400.0, 4, "rel", 1e-3, 6)),
    ("nf1024-smaller", 10007, SSTConfig(25600.0, 255, 32.0, 8, 1024, 0.0, 6400.0, 2, "rel", 1e-3, 2)),
]


def _signal(n, fs, seed):
    rng = np.random.default_rng(seed)
    t = np.arange(n) / fs
    x = np.cos(2 * np.pi * (0.11 * fs * t + 0.02 * fs * t * t)) + 0.3 * rng.standard_normal(n)
    return x.astype(np.float32)


def _same(a, b):
    return torch.equal(torch.view_as_real(a) if a.is_complex() else a,
                       torch.view_as_real(b) if b.is_complex() else b)


def test_static_forward_equals_bound_forward():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2003_07065_amd as sst
    for k, (name, n, cfg) in enumerate(CASES):
        print(f"[no-alloc] {name} N={n} nfft={cfg.nfft}", flush=True)
        x = torch.from_numpy(_signal(n, cfg.fs, k)).cuda()
        bound = sst.Plan.from_config(n, cfg, device="cuda")
        static = sst.Plan.from_config(n, cfg)          # never bound
        assert static.shape.workspace_bytes <= 32 << 20
        g_ref = torch.empty(1, dtype=torch.float32, device="cuda")
        g_s = torch.empty_like(g_ref)
        T_ref = bound.forward(x, gamma=g_ref)
        T_s = torch.full_like(T_ref, complex(float("nan"), 0.0))
        static.forward_static(x, T_s, gamma=g_s)
        torch.cuda.synchronize()
        assert _same(T_s, T_ref), name
        assert _same(g_s, g_ref), name
        # a chunk with the debug outputs, reusing the static call's gamma
        f0, nf = bound.n_frames // 3, 37
        outs = []
        for p, fn in ((bound, bound.forward), (static, static.forward_static)):
            S = torch.empty((nf, p.n_src), dtype=torch.complex64, device="cuda")
            idx = torch.empty((nf, p.n_src), dtype=torch.int32, device="cuda")
            T = torch.empty((nf, p.n_dst), dtype=torch.complex64, device="cuda")
            fn(x, T, f0, nf, S=S, idx=idx, reuse_gamma=True)
            outs.append((T, S, idx))
        torch.cuda.synchronize()
        for a, b in zip(outs[0], outs[1]):
            assert _same(a, b), name
        assert _same(outs[1][0], T_ref[f0:f0 + nf]), name
