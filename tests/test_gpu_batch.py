"""GPU: the batched form (sst_batch_*) against single-channel calls and the oracle.

Every work item of a batched launch computes what sst_forward / sst_inverse
compute for its channel, with the same arithmetic, so T and x̂ must be
bit-identical to single-channel calls; one channel is also checked against the
float64 oracle with the parity rules of tests/parity.py.  The channel list mixes
every launch group kind: several DFT sizes, pass-1 tap-row counts 4 and 16, hops,
subdivisions, absolute and relative thresholds, bands with k1 > 0, a one-sample
signal and a row longer than the histogram (chunked)."""
import sys
import zlib

import numpy as np
import pytest

import oracle
from tests.parity import reconciled_T, relf
from workloads import SSTConfig

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CHANNELS = [
    (20011, SSTConfig(25600.0, 255, 32.0, 8, 1024, 0.0, 6400.0, 2, "rel", 1e-3, 1)),
    (7001, SSTConfig(25600.0, 511, 64.0, 4, 2048, 0.0, 6400.0, 4, "rel", 1e-3, 3)),
    (30000, SSTConfig(25600.0, 1023, 128.0, 16, 4096, 0.0, 6400.0, 4, "rel", 1e-3, 6)),
    (5000, SSTConfig(25600.0, 1023, 128.0, 32, 4096, 0.0, 6400.0, 2, "abs", 1e-2, 3)),
    (1, SSTConfig(25600.0, 255, 32.0, 4, 1024, 0.0, 6400.0, 4, "rel", 1e-3, 2)),
    (12345, SSTConfig(25600.0, 2047, 256.0, 32, 8192, 0.0, 5000.0, 8, "rel", 1e-3, 26)),
    (9000, SSTConfig(25600.0, 1023, 100.0, 8, 1024, 300.0, 5000.0, 3, "rel", 1e-3, 2)),
    (12288, SSTConfig(25600.0, 255, 32.0, 16, 1024, 0.0, 6400.0, 2, "rel", 1e-3, 1)),
]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _signal(i, n, fs):
    rng = np.random.default_rng(zlib.crc32(f"batch{i}".encode()))
    t = np.arange(n) / fs
    f0 = rng.uniform(200.0, 3000.0)
    x = (np.cos(2 * np.pi * (f0 * t + 300.0 * t * t)) + 0.4 * np.cos(2 * np.pi * 0.7 * f0 * t)
         + 0.3 * rng.standard_normal(n))
    return x.astype(np.float32)


@pytest.fixture(scope="module")
def sst():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2003_07065_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def data(sst):
    dev = torch.device("cuda", 0)
    xs, plans, Ts, ridges, xhats = [], [], [], [], []
    for i, (n, cfg) in enumerate(CHANNELS):
        x = torch.from_numpy(_signal(i, n, cfg.fs)).to(dev)
        p = sst.Plan.from_config(n, cfg, device=dev)
        rng = np.random.default_rng(100 + i)
        n_comp = 1 + i % 3
        r = rng.integers(-1, p.n_dst, size=(n_comp, p.n_frames)).astype(np.int32)
        xs.append(x)
        plans.append(p)
        Ts.append(torch.empty((p.n_frames, p.n_dst), dtype=torch.complex64, device=dev))
        ridges.append(torch.from_numpy(r).to(dev))
        xhats.append(torch.empty((n_comp, n), dtype=torch.float32, device=dev))
    return dict(dev=dev, xs=xs, plans=plans, Ts=Ts, ridges=ridges, xhats=xhats)


def _single(data, i):
    p = data["plans"][i]
    cfg = CHANNELS[i][1]
    T = p.forward(data["xs"][i])
    xh = p.inverse(T, data["ridges"][i], cfg.hw)
    torch.cuda.synchronize()
    return T, xh


def _make_batch(sst, data, Ts=None):
    b = sst.Batch(CHANNELS, device=data["dev"])
    Ts = Ts or data["Ts"]
    for i, (n, cfg) in enumerate(CHANNELS):
        b.set_io(i, data["xs"][i], Ts[i], data["ridges"][i], cfg.hw, data["xhats"][i])
    b.commit()
    return b


def test_batch_forward_and_inverse_equal_single_calls(sst, data):
    b = _make_batch(sst, data)
    _say(f"[batch] {len(CHANNELS)} channels, groups by (N_f, tap rows)")
    b.forward()
    b.inverse()
    torch.cuda.synchronize()
    for i in range(len(CHANNELS)):
        T1, xh1 = _single(data, i)
        same_t = torch.equal(torch.view_as_real(data["Ts"][i]), torch.view_as_real(T1))
        same_x = torch.equal(data["xhats"][i], xh1)
        _say(f"  channel {i}: nfft={CHANNELS[i][1].nfft} T equal={same_t} xhat equal={same_x}")
        assert same_t and same_x, i


def test_batch_subranges_share_T_memory(sst, data):
    """Two forward calls over disjoint channel ranges whose T buffers alias."""
    dev = data["dev"]
    sizes = [p.n_frames * p.n_dst for p in data["plans"]]
    half = 4
    cap = max(sum(sizes[:half]), sum(sizes[half:]))
    pool = torch.empty(cap, dtype=torch.complex64, device=dev)
    Ts, off = [], 0
    for i, p in enumerate(data["plans"]):
        if i == half:
            off = 0
        Ts.append(pool[off:off + sizes[i]].view(p.n_frames, p.n_dst))
        off += sizes[i]
    b = _make_batch(sst, data, Ts)
    b.forward(0, half)
    torch.cuda.synchronize()
    first = [t.clone() for t in Ts[:half]]
    b.forward(half, len(CHANNELS))
    torch.cuda.synchronize()
    for i in range(len(CHANNELS)):
        T1, _ = _single(data, i)
        got = first[i] if i < half else Ts[i]
        assert torch.equal(torch.view_as_real(got), torch.view_as_real(T1)), i


def test_batch_matches_oracle_on_one_channel(sst, data):
    i = 1
    n, cfg = CHANNELS[i]
    b = _make_batch(sst, data)
    b.forward()
    torch.cuda.synchronize()
    p = data["plans"][i]
    idx = torch.empty((p.n_frames, p.n_src), dtype=torch.int32, device=data["dev"])
    S = torch.empty((p.n_frames, p.n_src), dtype=torch.complex64, device=data["dev"])
    p.forward(data["xs"][i], S=S, idx=idx)
    torch.cuda.synchronize()
    o = oracle.forward(data["xs"][i].cpu().numpy().astype(np.float64), cfg)
    e_s = relf(S.cpu().numpy(), o.S)
    e_t = relf(data["Ts"][i].cpu().numpy(), reconciled_T(o.S, idx.cpu().numpy(), p.n_dst))
    _say(f"  channel {i}: relF S={e_s:.2e} T(reconciled)={e_t:.2e}")
    assert e_s <= 1e-5 and e_t <= 1e-5


def test_batch_graph_replays_match_eager(sst, data):
    """forward + inverse of the whole batch captured in one HIP graph."""
    b = _make_batch(sst, data)
    b.forward()
    b.inverse()
    torch.cuda.synchronize()
    ref_T = [t.clone() for t in data["Ts"]]
    ref_x = [x.clone() for x in data["xhats"]]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            b.forward()
            b.inverse()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in data["Ts"]:
            t.zero_()
        for x in data["xhats"]:
            x.fill_(7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(CHANNELS)):
            assert torch.equal(torch.view_as_real(data["Ts"][i]), torch.view_as_real(ref_T[i])), (rep, i)
            assert torch.equal(data["xhats"][i], ref_x[i]), (rep, i)
        _say(f"  replay {rep}: every channel equal to the eager result")


def test_batch_speculative_fixup_equals_single(sst):
    """Batched speculative forward with a channel whose maximum the pre-pass
    misses (an impulse far above unit noise; see the single-channel test of
    the fix-up pass) next to an ordinary one: T equals single-channel calls."""
    dev = torch.device("cuda", 0)
    cfg = CHANNELS[2][1]
    chans = [(1 << 16, cfg), (30011, cfg)]
    xs = []
    for i, (n, _) in enumerate(chans):
        rng = np.random.default_rng(50 + i)
        x = rng.standard_normal(n).astype(np.float32)
        if i == 0:
            x[(16 * 32 * 3 + 16) * cfg.hop] += 15000.0
        xs.append(torch.from_numpy(x).to(dev))
    b = sst.Batch(chans, device=dev)
    Ts = []
    for i, (n, c) in enumerate(chans):
        p = sst.Plan.from_config(n, c, device=dev)
        Ts.append(torch.empty((p.n_frames, p.n_dst), dtype=torch.complex64, device=dev))
        b.set_io(i, xs[i], Ts[i], None, 0, None)
    b.commit()
    b.forward()
    torch.cuda.synchronize()
    for i, (n, c) in enumerate(chans):
        p = sst.Plan.from_config(n, c, device=dev)
        T1 = p.forward(xs[i])
        torch.cuda.synchronize()
        same = torch.equal(torch.view_as_real(Ts[i]), torch.view_as_real(T1))
        _say(f"  spec channel {i}: T equal to the single call: {same}")
        assert same, i
