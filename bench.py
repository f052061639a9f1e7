#!/usr/bin/env python3
"""Benchmark of the downsampled SST + direct inverse on one MI355X.

One step = the whole hot path over one synthetic signal already resident in
HBM: the threshold gamma = rho max|S| over every frame and the fused forward
transform (framing, FFT pair, IF, selective subdivided reassignment, T rows) in
one sst_forward call, the ridge argmax of every component, and the direct
inverse of every component.

Workload (default, c3): the long run-up channel, N = 2^26 samples at 25.6 kHz,
a fundamental sweeping 50 -> 600 Hz with 8 harmonics plus pink noise at 15 dB,
Gaussian window of 2047 taps (sigma 256), hop 32, N_f = 8192, band [0, 5 kHz],
subdivision 8, threshold 1e-3 max|S|; T (214.8 GB) stays resident in HBM; the
ridges are searched within +-26 bins of each harmonic order of the sweep and
the 8 harmonics are reconstructed with zones of half-width 26 bins.
``--workload c2`` runs the N = 2^20 three-component channel; ``c4`` the
batched uneven channels; ``c5`` the precision tiers.

Prints ONE JSON line.  Per-kernel times come from HIP events recorded on the
stream the library launches on.  The roofline object refers to the fused
forward kernel (the dominant HBM writer); its algorithmic bytes are the signal
read plus the dense complex64 T write.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
FP32_VALU_TFLOPS = 157.3   # MI355X vector FP32 (dual-issue / packed) peak
METRIC = "SST Msamples/s and % of HBM/MFMA roofline, batched vs plain, at stated error"


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2003_07065_amd", "csrc", "sst_kernels.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(workload: str):
    """HBM traffic of the fused forward kernel from committed rocprofv3 counter runs,
    or None when absent or taken on another version of the kernels."""
    p = os.path.join(ROOT, "profiles", f"fwd_kernel_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d


def log(msg: str):
    """Progress of a long run, on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_sample: int, hw: int, ridge_fn):
    """The float64 oracle, as it stands, on the first n_sample samples of the
    workload's own signal (a bounded sample; the threshold maximum is taken over
    that sample): STFT pair, threshold, reassignment, and the inverse of every
    component along the closed-form ridges."""
    import numpy as np
    import oracle
    c = w.cfg
    x = w.x[:n_sample].astype(np.float64)
    t0 = time.perf_counter()
    o = oracle.forward(x, c)
    ridge = ridge_fn(o.band.k1, o.band.n_dst, -(-n_sample // c.hop))
    for q in range(ridge.shape[0]):
        oracle.inverse(o.T, np.ascontiguousarray(ridge[q]), hw, o.g, c.hop, c.nfft, o.band.k1,
                       c.subdiv, n_sample)
    dt = time.perf_counter() - t0
    return {"value": n_sample / dt / 1e6, "unit": "Msamples/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"first {n_sample} samples of the workload's signal ({n_sample / w.n:.4g} "
                      f"of it) as a signal of their own, whole pipeline (threshold, STFT pair, "
                      f"reassignment, {ridge.shape[0]}-component inverse) in float64, "
                      f"{dt:.2f} s"}


def run_c4(args):
    """Batched uneven channels (c4): one persistent launch per DFT-size group and
    channel range, captured in one HIP graph, against a per-channel loop of the
    single-channel calls on the same buffers."""
    import numpy as np
    import torch
    import paper_2003_07065_amd as sst
    from workloads import make_c4, ridge_bins

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    ws = make_c4(n_channels=args.c4_channels, log2_min=args.c4_log2_min,
                 log2_max=args.c4_log2_max)
    gen_s = time.perf_counter() - t0
    plans = [sst.Plan.from_config(w.n, w.cfg, device=dev) for w in ws]
    sizes = [p.n_frames * p.n_dst for p in plans]
    pool_elems = min(sum(sizes), int(args.t_pool_gb * 1e9) // 8)
    if max(sizes) > pool_elems:
        raise SystemExit("T pool smaller than the largest channel's T")
    passes, a, acc = [], 0, 0
    for i, sz in enumerate(sizes):
        if acc + sz > pool_elems:
            passes.append((a, i))
            a, acc = i, 0
        acc += sz
    passes.append((a, len(sizes)))
    pool = torch.empty(pool_elems, dtype=torch.complex64, device=dev)
    Ts = []
    for a, b in passes:
        off = 0
        for i in range(a, b):
            Ts.append(pool[off:off + sizes[i]].view(plans[i].n_frames, plans[i].n_dst))
            off += sizes[i]
    xs = [torch.from_numpy(w.x).to(dev) for w in ws]
    ridges, xh_b, xh_l = [], [], []
    for w, p in zip(ws, plans):
        c = w.cfg
        r = ridge_bins(w.inst_freq(w.frame_times()), c.fs, c.nfft, p.k1, c.subdiv, p.n_dst)
        ridges.append(torch.from_numpy(np.ascontiguousarray(r, dtype=np.int32)).to(dev))
        xh_b.append(torch.empty((r.shape[0], w.n), dtype=torch.float32, device=dev))
        xh_l.append(torch.empty((r.shape[0], w.n), dtype=torch.float32, device=dev))
    batch = sst.Batch([(w.n, w.cfg) for w in ws], device=dev)
    for i, w in enumerate(ws):
        batch.set_io(i, xs[i], Ts[i], ridges[i], w.cfg.hw, xh_b[i])
    batch.commit()
    stream = torch.cuda.current_stream(dev)

    def batched(evs=None):
        for k, (a, b) in enumerate(passes):
            if evs:
                evs[2 * k].record(stream)
            batch.forward(a, b)
            if evs:
                evs[2 * k + 1].record(stream)
            batch.inverse(a, b)
        if evs:
            evs[-1].record(stream)

    def loop():
        for i, w in enumerate(ws):
            plans[i].forward(xs[i], Ts[i])
            plans[i].inverse(Ts[i], ridges[i], w.cfg.hw, xhat=xh_l[i])

    def timed(fn, steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    for _ in range(args.warmup):
        batched()
        loop()
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(xh_b, xh_l))
    loop_ms = timed(loop, args.steps)
    eager_ms = timed(batched, args.steps)
    # per-segment split of one eager batched step
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(passes) + 1)]
    torch.cuda.synchronize()
    batched(evs)
    torch.cuda.synchronize()
    fwd_ms = sum(evs[2 * k].elapsed_time(evs[2 * k + 1]) for k in range(len(passes)))
    inv_ms = sum(evs[2 * k + 1].elapsed_time(evs[2 * k + 2]) for k in range(len(passes)))
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            batched()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph_ms = timed(g.replay, args.steps)
    same_graph = all(torch.equal(a, b) for a, b in zip(xh_b, xh_l))

    n_total = sum(w.n for w in ws)
    t_bytes = sum(8 * p.n_frames * p.n_dst for p in plans)
    fwd_bytes = t_bytes + 4 * n_total
    achieved = fwd_bytes / (fwd_ms / 1e3) / 1e9
    out = {
        "metric": METRIC, "value": round(n_total / (graph_ms / 1e3) / 1e6, 2), "unit": "Msamples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(graph_ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched uneven channels: {len(ws)} channels (seed 0), lengths "
                               f"log-uniform in [2^{args.c4_log2_min:g}, 2^{args.c4_log2_max:g}], "
                               "H in {4,8,16,32}, N_f in "
                               "{1024,2048,4096}, z in {2,4}, L=N_f/4-1, sigma=N_f/32, band "
                               "[0, 6.4 kHz], 1-4 chirp/AM-FM components + noise 5-25 dB, "
                               "closed-form ridges",
                   "n_channels": len(ws), "n_samples_total": n_total, "T_bytes_total": t_bytes,
                   "T_pool_bytes": pool_elems * 8, "passes": len(passes),
                   "generation_s": round(gen_s, 1)},
        "roofline": {"kernel": "fwd_kernel (batched groups)", "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes_per_step": fwd_bytes, "forward_ms": round(fwd_ms, 3)},
        "segments_ms": {"forward_incl_threshold": round(fwd_ms, 3), "inverse": round(inv_ms, 3)},
        "batched_eager_ms": round(eager_ms, 3), "batched_graph_ms": round(graph_ms, 3),
        "plain_loop_ms": round(loop_ms, 3),
        "speedup_vs_plain_loop": round(loop_ms / graph_ms, 3),
        "batched_equals_plain_loop": bool(same and same_graph),
    }
    print(json.dumps(out), flush=True)


def run_c5(args):
    """Precision tier (c5): many equal-length channels, STFT + SST forward in the
    FP32 FFT path and as DFT-as-GEMM on the matrix cores (BF16, FP16 hi/lo x3);
    speedup of each tier over the FP32 FFT path and its error on channel 0."""
    import numpy as np
    import torch
    import paper_2003_07065_amd as sst
    from workloads import make_c5, ridge_bins

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n = 1 << 20
    nch = args.c5_channels
    t0 = time.perf_counter()
    xs, w0 = [], None
    for c0 in range(0, nch, 32):
        chunk = make_c5(n_channels=min(32, nch - c0), n=n, nfft=args.c5_nfft, seed=c0,
                        f_hi=args.c5_band_hi)
        if w0 is None:
            w0 = chunk[0]
        for w in chunk:
            xs.append(torch.from_numpy(w.x).to(dev))
            if w is not w0:
                w.comps = None
    gen_s = time.perf_counter() - t0
    cfg = w0.cfg
    stream = torch.cuda.current_stream(dev)
    res = {}
    T0 = {}
    for prec in ("fp32", "bf16", "f16x3"):
        plan = sst.Plan.from_config(n, cfg, device=dev, precision=prec)
        T = torch.empty((plan.n_frames, plan.n_dst), dtype=torch.complex64, device=dev)
        tuning = plan.autotune(xs[0], T, reps=2) if not args.no_tune else plan.get_tuning()
        log(f"c5 {prec}: tuning {tuning}")

        def step(reuse=False):
            for x in xs:
                plan.forward(x, T, reuse_gamma=reuse)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        for _ in range(args.steps):
            step()
        e[1].record(stream)
        for _ in range(args.steps):
            step(reuse=True)
        e[2].record(stream)
        torch.cuda.synchronize()
        full_ms = e[0].elapsed_time(e[1]) / args.steps
        fwd_ms = e[1].elapsed_time(e[2]) / args.steps
        # error of the tier on channel 0: T against the FP32 FFT path, inverse SNR
        plan.forward(xs[0], T)
        ridge = ridge_bins(w0.inst_freq(w0.frame_times()), cfg.fs, cfg.nfft, plan.k1,
                           cfg.subdiv, plan.n_dst)
        xh = plan.inverse(T, torch.from_numpy(ridge).to(dev), cfg.hw).cpu().numpy()
        torch.cuda.synchronize()
        T0[prec] = T.cpu().numpy()
        M = (cfg.win_len - 1) // 2
        snr = []
        for q in range(ridge.shape[0]):
            ref = w0.comps[q][M:n - M].astype(np.float64)
            snr.append(round(10 * math.log10(np.sum(ref ** 2)
                                             / np.sum((ref - xh[q][M:n - M]) ** 2)), 3))
        flops = None
        if prec != "fp32":
            products = 3 if prec == "f16x3" else 1
            flops = 2.0 * 4 * plan.n_src * cfg.win_len * plan.n_frames * nch * products
        res[prec] = {"tuning": tuning,
                     "ms_with_threshold": round(full_ms, 3), "forward_ms": round(fwd_ms, 3),
                     "Msamples_per_s": round(n * nch / (full_ms / 1e3) / 1e6, 1),
                     "snr_db_channel0": snr,
                     "mfma_tflops": (round(flops / (fwd_ms / 1e3) / 1e12, 1) if flops else None)}
        del plan, T
    base = res["fp32"]["ms_with_threshold"]
    for prec in ("bf16", "f16x3"):
        res[prec]["speedup_vs_fp32_fft"] = round(base / res[prec]["ms_with_threshold"], 3)
        res[prec]["forward_speedup_vs_fp32_fft"] = round(res["fp32"]["forward_ms"]
                                                         / res[prec]["forward_ms"], 3)
        d = T0[prec] - T0["fp32"]
        res[prec]["T_relF_vs_fp32_fft"] = float(np.linalg.norm(d) / np.linalg.norm(T0["fp32"]))
    peak = 2500.0
    best = res["f16x3"]
    out = {
        "metric": METRIC, "value": best["Msamples_per_s"], "unit": "Msamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms_with_threshold"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16x3",
        "data": "synthetic",
        "config": {"workload": f"precision tier: {nch} channels x 2^20 samples at 25.6 kHz, "
                               f"three AM-FM components + noise 10 dB, N_f={args.c5_nfft}, "
                               f"L=N_f-1, sigma=N_f/8, H=8, band [0, {args.c5_band_hi:g} Hz], z=1, "
                               "rho=1e-3; STFT+SST forward (threshold included)",
                   "generation_s": round(gen_s, 1)},
        "roofline": {"kernel": "gemm_kernel (FP16 hi/lo x3, 32x32x16 MFMA)", "bound": "mfma",
                     "achieved": best["mfma_tflops"], "peak": peak, "unit": "TFLOP/s",
                     "frac": round(best["mfma_tflops"] / peak, 4), "traffic": None},
        "tiers": res,
    }
    print(json.dumps(out), flush=True)


def run_c5x(args):
    """Narrow-band crossover of the filter-bank STFT (DFT-as-GEMM) against the
    FP32 FFT path: c5 channels (2^20 samples, H = 8, L = N_f - 1), bands
    [0, f_hi] swept at N_f 1024 and 4096.  The GEMM tiers' work grows with
    n_src L (4 n_src L products per frame), the FFT's with N_f log2 N_f, so the
    matrix cores win below some band width; each point is the forward call
    with gamma reused (the threshold pre-pass excluded), HIP events over
    `steps` passes over the channels."""
    import torch
    import paper_2003_07065_amd as sst
    from workloads import SSTConfig, make_c5

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n = 1 << 20
    nch = min(args.c5_channels, 32)
    xs = [torch.from_numpy(w.x).to(dev) for w in make_c5(n_channels=nch, n=n, nfft=1024)]
    stream = torch.cuda.current_stream(dev)
    rows = []
    for nfft in (1024, 4096):
        for f_hi in (100.0, 200.0, 400.0, 800.0, 1600.0, 3200.0, 6400.0, 12800.0):
            cfg = SSTConfig(fs=25600.0, win_len=nfft - 1, sigma=nfft / 8.0, hop=8, nfft=nfft,
                            f_lo=0.0, f_hi=f_hi, subdiv=1, thr_mode="rel", thr=1e-3, hw=1)
            row = {"nfft": nfft, "f_hi": f_hi}
            for prec in ("fp32", "bf16", "f16x3"):
                try:
                    plan = sst.Plan.from_config(n, cfg, device=dev, precision=prec)
                except sst.SSTError as e:
                    row[prec] = None
                    row[prec + "_why"] = str(e).split(":")[-1].strip()[:80]
                    continue
                row["n_src"] = plan.n_src
                T = torch.empty((plan.n_frames, plan.n_dst), dtype=torch.complex64, device=dev)
                for x in xs[:2]:
                    plan.forward(x, T)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(args.steps):
                    for x in xs:
                        plan.forward(x, T, reuse_gamma=True)
                e1.record(stream)
                torch.cuda.synchronize()
                row[prec] = round(e0.elapsed_time(e1) / args.steps / nch, 4)   # ms per channel
                del plan, T
            row["nsrc_L_over_nf_log2nf"] = round(row.get("n_src", 0) * (nfft - 1)
                                                 / (nfft * math.log2(nfft)), 2)
            log(f"c5x nfft={nfft} f_hi={f_hi:g}: {row}")
            rows.append(row)
    cross = {}
    for nfft in (1024, 4096):
        for prec in ("bf16", "f16x3"):
            wins = [r for r in rows if r["nfft"] == nfft and r.get(prec) and r.get("fp32")
                    and r[prec] < r["fp32"]]
            best = max(wins, key=lambda r: r["f_hi"]) if wins else None
            cross[f"{prec}_nfft{nfft}"] = (
                {"widest_winning_band_hz": best["f_hi"], "n_src": best["n_src"],
                 "speedup": round(best["fp32"] / best[prec], 3),
                 "nsrc_L_over_nf_log2nf": best["nsrc_L_over_nf_log2nf"]} if best else None)
    out = {"metric": "forward ms per channel vs band width (filter-bank STFT crossover)",
           "unit": "ms", "n_gpus": 1, "steps": args.steps, "higher_is_better": False,
           "data": "synthetic",
           "config": {"workload": f"{nch} c5 channels x 2^20 samples at 25.6 kHz, H=8, "
                                  "L=N_f-1, sigma=N_f/8, z=1, bands [0, f_hi]; forward with "
                                  "gamma reused"},
           "sweep": rows, "crossover": cross}
    print(json.dumps(out), flush=True)


def measure_extras(plan, xg, T, n, stream, steps):
    """The transform's other outputs on the same resident signal, each timed with
    HIP events over `steps` calls (outside the step): the STFT product, its
    synthesis (Eqs. 10-11), the compressed |T| rows, and the Renyi entropy of T.
    GB/s counts the algorithmic bytes (inputs read once, outputs written once)."""
    import torch
    import paper_2003_07065_amd as sst

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    res = {}
    nfr, nsrc, ndst = plan.n_frames, plan.n_src, plan.n_dst
    S = torch.empty((nfr, nsrc), dtype=torch.complex64, device=xg.device)
    ms = timed(lambda: plan.stft(xg, S))
    b = 4 * n + 8 * nfr * nsrc
    res["stft_product"] = {"ms": round(ms, 4), "GB_per_s": round(b / ms / 1e6, 1),
                           "hbm_frac": round(b / ms / 1e6 / HBM_PEAK_GBS, 4)}
    xh = torch.empty(n, dtype=torch.float32, device=xg.device)
    ms = timed(lambda: plan.stft_inverse(S, xh))
    b = 8 * nfr * nsrc + 4 * n
    res["stft_synthesis"] = {"ms": round(ms, 4), "GB_per_s": round(b / ms / 1e6, 1),
                             "Msamples_per_s": round(n / ms / 1e3, 1)}
    del S, xh
    for fmt, bpb in (("mag_f32", 4), ("mag_f16", 2)):
        dt = torch.float32 if fmt == "mag_f32" else torch.float16
        Tm = torch.as_strided(T.view(dt), (nfr, ndst), (ndst, 1))   # aliases T's memory
        ms = timed(lambda: plan.forward(xg, Tm, out=fmt))
        b = 4 * n + bpb * nfr * ndst
        res["forward_" + fmt] = {"ms_whole_call": round(ms, 4), "GB_per_s": round(b / ms / 1e6, 1),
                                 "Msamples_per_s": round(n / ms / 1e3, 1)}
    plan.forward(xg, T)   # T holds the complex rows again
    ms = timed(lambda: sst.renyi(T, 3))
    b = 8 * nfr * ndst
    r = float(sst.renyi(T, 3)[2].cpu())
    res["renyi_T"] = {"ms": round(ms, 4), "GB_per_s": round(b / ms / 1e6, 1),
                      "hbm_frac": round(b / ms / 1e6 / HBM_PEAK_GBS, 4), "bits": round(r, 4)}
    return res


def run_single(args):
    """One long channel (c3 default, c2): a step is the whole hot path over the
    resident signal -- threshold and fused forward (one sst_forward call),
    ridges, and the direct inverse of every component."""
    import numpy as np
    import torch
    import paper_2003_07065_amd as sst
    from workloads import make_c2, make_c3, ridge_bins

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    if args.workload == "c3":
        w = make_c3(n=args.n or (1 << 26))
    else:
        w = make_c2(n=args.n or (1 << 20))
    gen_s = time.perf_counter() - t0
    log(f"{args.workload}: generated {w.n} samples in {gen_s:.1f} s")
    c = w.cfg
    comps = w.comps
    w.comps = None
    plan = sst.Plan.from_config(w.n, c, device=dev)
    xg = torch.from_numpy(w.x).to(dev)
    T = torch.empty((plan.n_frames, plan.n_dst), dtype=torch.complex64, device=dev)
    f_true = w.inst_freq(w.frame_times())
    ridge_true = ridge_bins(f_true, c.fs, c.nfft, plan.k1, c.subdiv, plan.n_dst)
    n_comp = ridge_true.shape[0]
    ridge = torch.empty((n_comp, plan.n_frames), dtype=torch.int32, device=dev)
    centre = None
    if args.workload == "c3":
        # run-up: the harmonics sweep over most of the band, so each ridge is
        # searched within +-hw bins of its order of the (tacho-like) shaft speed
        centre = torch.from_numpy(ridge_true).to(dev)
        bands = [(-c.hw, c.hw)] * n_comp
        ridge_desc = f"guided ridges (+-{c.hw} bins around each harmonic order)"
    else:
        # ridge search bands: +-8% around each component's nominal frequency
        bands = []
        for q in range(n_comp):
            f0 = float(np.median(f_true[q]))
            lo = int(math.floor(c.subdiv * (0.92 * f0 / c.delta_f - plan.k1)))
            hi = int(math.ceil(c.subdiv * (1.08 * f0 / c.delta_f - plan.k1)))
            bands.append((max(lo, 0), min(hi, plan.n_dst - 1)))
        ridge_desc = "ridges in +-8% bands"
    xhat = torch.empty((n_comp, w.n), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)

    # launch choices: the library's autotuner on these buffers (before the timed
    # region), or the defaults
    t0 = time.perf_counter()
    if args.no_tune:
        tuning = dict(plan.get_tuning(), source="default")
    else:
        rt = torch.from_numpy(ridge_true).to(dev)
        tuning = dict(plan.autotune(xg, T, rt, c.hw, xhat, reps=3), source="autotuned")
        del rt
        if os.environ.get("SST_TUNE_CACHE"):
            plan.tuning_save(os.environ["SST_TUNE_CACHE"])
    tuning["search_s"] = round(time.perf_counter() - t0, 2)
    log(f"tuning {tuning}")

    def step(evs=None):
        if evs:
            evs[0].record(stream)
        # gamma from every frame and the fused forward kernel (the library
        # records evs[1] and evs[2] right around that kernel's launch)
        plan.forward(xg, T, kernel_events=(evs[1], evs[2]) if evs else None)
        if evs:
            evs[3].record(stream)
        plan.ridge(T, bands, out=ridge, centre=centre)
        if evs:
            evs[4].record(stream)
        plan.inverse(T, ridge, c.hw, xhat=xhat)
        if evs:
            evs[5].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"{args.warmup} warm-up steps done")

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    for row in evs:
        for ev in row:
            ev.record(stream)   # creates the events; the timed steps record them again
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"{args.steps} timed steps done in {wall:.2f} s")

    seg = np.array([[evs[k][i].elapsed_time(evs[k][i + 1]) for i in range(5)]
                    for k in range(args.steps)])          # ms
    step_ms = np.array([evs[k][0].elapsed_time(evs[k][5]) for k in range(args.steps)])
    total_ms = float(step_ms.sum())
    ms_per_step = total_ms / args.steps
    value = w.n * args.steps / (total_ms / 1e3) / 1e6

    # Accuracy of the timed result: SNR of every component (Eq. 33, FP64 on the GPU).
    xref = torch.from_numpy(comps.astype(np.float32)).to(dev)
    err = torch.zeros((n_comp, 2), dtype=torch.float64, device=dev)
    plan.inverse(T, ridge, c.hw, xhat=xhat, xref=xref, err=err)
    torch.cuda.synchronize()
    e = err.cpu().numpy()
    snr = [float(10.0 * np.log10(e[q, 1] / e[q, 0])) for q in range(n_comp)]
    ridge_hit = float((ridge.cpu().numpy() == ridge_true).mean())
    del xref

    calib = None
    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib << 20
        a = torch.empty(nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.neg(a, out=b)   # one elementwise kernel: reads nb bytes, writes nb bytes
        torch.cuda.synchronize()
        calib = {"copy_bytes_each_way": nb}
        del a, b

    fwd_ms = float(np.mean(seg[:, 1]))                     # the fused forward kernel alone
    thr_ms = float(np.mean(seg[:, 0] + seg[:, 2]))         # gamma seed, gamma, fix-up pass
    ridge_ms = float(np.mean(seg[:, 3]))
    inv_ms = float(np.mean(seg[:, 4]))
    t_bytes = 8 * plan.n_dst * plan.n_frames
    x_bytes = 4 * w.n
    fwd_alg_bytes = t_bytes + x_bytes
    achieved = fwd_alg_bytes / (fwd_ms / 1e3) / 1e9
    traffic = load_traffic(args.workload)
    roof = {"kernel": f"fwd_kernel (fused framing + FFT pair + IF + reassignment, "
                      f"N_f={c.nfft})",
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (traffic or {}).get("bytes_per_launch"),
            "algorithmic_bytes_per_launch": fwd_alg_bytes,
            "avg_launch_ms": round(fwd_ms, 4)}
    # whole-step HBM roofline: every algorithmic byte of the step at peak bandwidth
    inv_bytes = n_comp * (8 * (2 * c.hw + 1) * plan.n_frames + 4 * w.n)
    step_bytes = fwd_alg_bytes + inv_bytes + x_bytes
    if args.workload == "c3":
        desc = (f"downsampled SST + direct inverse, one channel, N=2^26 at 25.6 kHz: run-up "
                f"50->600 Hz with 8 harmonics (1/h, random phases) + pink noise 15 dB (seed 0), "
                f"Gaussian L=2047 sigma=256, H=32, N_f=8192, band [0, 5 kHz], z=8, "
                f"gamma=1e-3 max|S|, {ridge_desc}, 8-harmonic inverse hw={c.hw}")
    else:
        desc = (f"downsampled SST + direct inverse, one channel, N=2^20 at 25.6 kHz, 3 AM-FM "
                f"components + white noise 10 dB (seed 0), Gaussian L=1023 sigma=128, H=16, "
                f"N_f=4096, band [0, 6.4 kHz], z=4, gamma=1e-3 max|S|, {ridge_desc}, "
                f"3-component inverse hw={c.hw}")
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Msamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "n_samples": w.n, "n_frames": plan.n_frames,
                   "n_dst": plan.n_dst, "T_bytes": t_bytes, "generation_s": round(gen_s, 1)},
        "roofline": roof,
        "tuning": tuning,
        "segments_ms": {"forward_kernel": round(fwd_ms, 4),
                        "threshold_and_fixup": round(thr_ms, 4),
                        "ridge": round(ridge_ms, 4), "inverse": round(inv_ms, 4)},
        "step_hbm_roofline_frac": round(step_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "accuracy": {"snr_db": [round(s, 3) for s in snr], "ridge_equals_true_if_bin": ridge_hit},
        "wall_s": round(wall, 3),
        "kernel_source_sha256_16": kernel_source_hash(),
    }
    if calib:
        out["calibration"] = calib
    if not args.no_extras:
        out["extras"] = measure_extras(plan, xg, T, w.n, stream, args.steps)
    if not args.no_cpu_baseline:
        del T
        torch.cuda.empty_cache()
        w.comps = comps
        sample = args.cpu_sample or (1 << 20 if args.workload == "c3" else 1 << 18)

        def ridge_fn(k1, n_dst, nfr):
            t = np.arange(nfr, dtype=np.float64) * c.hop / c.fs
            return ridge_bins(w.inst_freq(t), c.fs, c.nfft, k1, c.subdiv, n_dst)

        log(f"oracle on the first {sample} samples")
        out["cpu_baseline"] = cpu_baseline(w, sample, c.hw, ridge_fn)
    print(json.dumps(out), flush=True)


def run_e1(args):
    """The paper's own simulated signal (Sec. 3, Eqs. 30-31: three AM-FM components,
    N = 8192 at 1024 Hz, 5 dB noise, Gaussian window sigma = 0.03 s): the TF
    concentration study of Fig. 3 -- the third-order Renyi entropy (Eq. 32) of SST
    and STFT over a grid of time hops H_t and frequency downsampling H_f = N / N_f
    -- and the reconstruction SNR (Eq. 33) of the three components against the
    zone half-width f_w (Figs. 6-7), all on the GPU."""
    import numpy as np
    import torch
    import paper_2003_07065_amd as sst
    from workloads import SSTConfig, make_paper_eq30, ridge_bins

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    w = make_paper_eq30()
    c0 = w.cfg
    n = w.n
    xg = torch.from_numpy(w.x).to(dev)
    xref = torch.from_numpy(w.comps.astype(np.float32)).to(dev)
    hts = [1, 5, 10, 20, 40, 60]
    nfs = [8192, 4096, 2048, 1024, 512]
    stream = torch.cuda.current_stream(dev)
    rows = []
    for nf in nfs:
        for ht in hts:
            cfg = SSTConfig(c0.fs, c0.win_len, c0.sigma, ht, nf, 0.0, c0.fs / 2, 1, "rel", c0.thr,
                            0)
            plan = sst.Plan.from_config(n, cfg, device=dev)
            T = plan.forward(xg)
            S = plan.stft(xg)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                plan.forward(xg, T)
            e1.record(stream)
            r_t = sst.renyi(T, 3)
            r_s = sst.renyi(S, 3)
            torch.cuda.synchronize()
            rows.append({"H_t": ht, "N_f": nf, "H_f": n // nf,
                         "renyi_sst_bits": round(float(r_t[2].cpu()), 4),
                         "renyi_stft_bits": round(float(r_s[2].cpu()), 4),
                         "sst_ms": round(e0.elapsed_time(e1) / args.steps, 4)})
            del plan, T, S
    # reconstruction SNR against the zone half-width, H_t = 1, N_f = N
    snr = []
    for fw in (2.0, 5.0, 10.0, 20.0, 30.0):
        cfg = SSTConfig(c0.fs, c0.win_len, c0.sigma, 1, n, 0.0, c0.fs / 2, 1, "rel", c0.thr, 0)
        plan = sst.Plan.from_config(n, cfg, device=dev)
        T = plan.forward(xg)
        hw = int(round(fw * cfg.subdiv / cfg.delta_f))
        ridge = ridge_bins(w.inst_freq(w.frame_times()), cfg.fs, cfg.nfft, plan.k1, cfg.subdiv,
                           plan.n_dst)
        err = torch.zeros((3, 2), dtype=torch.float64, device=dev)
        plan.inverse(T, torch.from_numpy(ridge).to(dev), hw, xref=xref, err=err)
        e = err.cpu().numpy()
        snr.append({"f_w_hz": fw, "hw_bins": hw,
                    "snr_db": [round(float(10 * np.log10(e[q, 1] / e[q, 0])), 3) for q in range(3)]})
        del plan, T
    out = {"metric": "SST Renyi entropy (bits) vs downsampling and reconstruction SNR vs f_w, "
                     "paper Sec. 3 workload", "unit": "bits / dB", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "Eqs. 30-31: three AM-FM components, N=8192, fs=1024 Hz, 5 dB "
                                  "white noise (seed 0), Gaussian sigma=0.03 s (L=247), full band, "
                                  "z=1, gamma=1e-6 max|S|"},
           "renyi_grid": rows, "snr_vs_fw": snr}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=["c3", "c2", "c4", "c5", "c5x", "e1"], default="c3",
                    help="c3: the long run-up channel, N=2^26 (default); c2: N=2^20; "
                         "c4: batched uneven channels; c5: precision tiers; c5x: narrow-band "
                         "crossover of the GEMM tiers; e1: the paper's Sec. 3 concentration "
                         "and reconstruction study")
    ap.add_argument("--c5-channels", type=int, default=512)
    ap.add_argument("--c5-nfft", type=int, default=512, choices=[512, 1024])
    ap.add_argument("--c5-band-hi", type=float, default=6400.0,
                    help="c5: upper edge of the band in Hz (1000 for the narrow-band variant)")
    ap.add_argument("--c4-channels", type=int, default=256)
    ap.add_argument("--c4-log2-min", type=float, default=16.0,
                    help="c4: channel lengths are log-uniform in [2^min, 2^max] samples")
    ap.add_argument("--c4-log2-max", type=float, default=22.0)
    ap.add_argument("--t-pool-gb", type=float, default=120.0,
                    help="c4: device memory for T; channels are processed in passes that fit")
    ap.add_argument("--n", type=int, default=0,
                    help="signal length (default: the workload's, 2^26 for c3, 2^20 for c2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip timing the STFT product / synthesis, |T| rows and Renyi entropy")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the library's default launch choices instead of autotuning")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle sample in samples (default 2^20 for c3, 2^18 for c2)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2003_07065_amd  # noqa: F401  (fails loudly without the built library)

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c4":
        run_c4(args)
    elif args.workload == "c5":
        run_c5(args)
    elif args.workload == "c5x":
        run_c5x(args)
    elif args.workload == "e1":
        run_e1(args)
    else:
        run_single(args)


if __name__ == "__main__":
    main()
