"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/sst.h declares, validates parameters, and derives the same
band / destination shapes as the oracle.  Nothing here launches a kernel."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2003_07065_amd as sst

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "sst.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sst_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert {"sst_plan", "sst_forward", "sst_inverse"} <= set(names)
    L = sst.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(sst.EXPORTED)


def _params(**kw):
    d = dict(n_samples=1 << 15, fs=25600.0, win_len=1023, sigma=128.0, hop=16, nfft=4096,
             f_lo=0.0, f_hi=6400.0, subdiv=4, thr_mode="rel", thr=1e-3)
    d.update(kw)
    return d


@pytest.mark.parametrize("fs,nfft,f_lo,f_hi,z", [
    (25600.0, 4096, 0.0, 6400.0, 4), (25600.0, 8192, 0.0, 5000.0, 8),
    (1024.0, 4096, 0.0, 512.0, 1), (44100.0, 8192, 6900.0, 9500.0, 8),
    (1000.0, 512, 33.3, 250.0, 3), (25600.0, 1024, 0.0, 6400.0, 2)])
def test_shapes_match_oracle_band(fs, nfft, f_lo, f_hi, z):
    p = sst.Plan(**_params(fs=fs, nfft=nfft, f_lo=f_lo, f_hi=f_hi, subdiv=z, win_len=255,
                           sigma=32.0))
    b = oracle.band(fs, nfft, f_lo, f_hi, z)
    assert (p.k1, p.k2, p.n_src, p.n_dst) == (b.k1, b.k2, b.n_src, b.n_dst)
    assert p.n_frames == -(-(1 << 15) // 16)
    assert p.shape.t_row_bytes == 8 * b.n_dst
    assert p.shape.workspace_bytes > 0 and p.shape.workspace_bytes % 256 == 0


@pytest.mark.parametrize("bad,status", [
    (dict(win_len=1024), sst.SST_E_ARG),          # even window
    (dict(win_len=8191), sst.SST_E_ARG),          # L > N_f
    (dict(nfft=3000), sst.SST_E_ARG),             # not a power of two
    (dict(nfft=16384, win_len=1023), sst.SST_E_UNSUPPORTED),
    (dict(nfft=256, win_len=255), sst.SST_E_UNSUPPORTED),
    (dict(f_hi=20000.0), sst.SST_E_ARG),          # above fs/2
    (dict(f_lo=100.0, f_hi=100.0), sst.SST_E_ARG),
    (dict(subdiv=0), sst.SST_E_ARG),
    (dict(subdiv=512), sst.SST_E_ARG),            # z N_f > 2^20
    (dict(hop=0), sst.SST_E_ARG),
    (dict(n_samples=0), sst.SST_E_ARG),
    (dict(sigma=0.0), sst.SST_E_ARG),
    (dict(thr=-1.0), sst.SST_E_ARG),
    (dict(fs=float("nan")), sst.SST_E_ARG),
])
def test_plan_rejects_invalid(bad, status):
    with pytest.raises(sst.SSTError) as ei:
        sst.Plan(**_params(**bad))
    assert ei.value.status == status
    assert sst.lib().sst_last_error()


def test_plan_rejects_bad_struct_size_and_null():
    L = sst.lib()
    p = sst.Params()
    p.struct_size = 8
    h = ctypes.c_void_p()
    assert L.sst_plan(ctypes.byref(p), ctypes.byref(h)) == sst.SST_E_ARG
    assert L.sst_plan(None, ctypes.byref(h)) == sst.SST_E_ARG
    assert L.sst_plan_query(None, None) == sst.SST_E_ARG


def test_unbound_plan_refuses_work():
    p = sst.Plan(**_params())
    L = sst.lib()
    aux = sst.FwdAux()
    rc = L.sst_forward(p._h, ctypes.c_void_p(16), 0, 1, ctypes.c_void_p(16), ctypes.byref(aux),
                       0, None)
    assert rc == sst.SST_E_STATE
    rc = L.sst_inverse(p._h, ctypes.c_void_p(16), 0, 1, ctypes.c_void_p(16), 1, 2,
                       ctypes.c_void_p(16), None, None, 0, None)
    assert rc == sst.SST_E_STATE
    band = (ctypes.c_int32 * 2)(0, 10)
    assert L.sst_ridge(p._h, ctypes.c_void_p(16), 1, band, 1, ctypes.c_void_p(16),
                       None) == sst.SST_E_STATE


def test_bind_rejects_small_or_misaligned_workspace():
    p = sst.Plan(**_params())
    L = sst.lib()
    assert L.sst_plan_bind(p._h, None, 1 << 20, None) == sst.SST_E_WORKSPACE
    assert L.sst_plan_bind(p._h, ctypes.c_void_p(4096), 16, None) == sst.SST_E_WORKSPACE
    assert L.sst_plan_bind(p._h, ctypes.c_void_p(4096 + 8), 1 << 30, None) == sst.SST_E_WORKSPACE


def test_status_strings():
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert sst.status_string(s)
    assert "unknown" in sst.status_string(-99)


def test_custom_window_must_come_in_pairs():
    g, gd = oracle.gaussian_windows(255, 32.0)
    p = sst.Plan(**_params(win_len=255, sigma=32.0), window=g, dwindow=gd)
    assert p.n_dst == 4097
    with pytest.raises(sst.SSTError):
        sst.Plan(**_params(win_len=255), window=g, dwindow=None)


def test_critical_hf_matches_paper(golden):
    """Sec. 4: Eq. 38 gives H_f < 64 and Eq. 46 H_f < 60 for the simulation; Sec. 5.1 quotes
    2446 for the aero-engine record."""
    sim = golden["eq38_sim_hf_bound"]
    e38, e46 = sst.critical_hf(sim["n"], sim["sigma_s"], sim["fs"])
    assert round(e38) == golden["eq38_sim_hf_bound"]["value"]
    assert round(e46) == golden["eq46_sim_hf_bound"]["value"]
    aero = golden["eq38_aero_hf_bound"]
    e38a, _ = sst.critical_hf(aero["n"], aero["sigma_s"], aero["fs"])
    assert round(e38a) == aero["value"]
    # the aero record's actual H_f sits below it (Sec. 5.1)
    assert round(golden["aero_hf"]["n"] / golden["aero_hf"]["nfft"]) == golden["aero_hf"]["value"]
    with pytest.raises(sst.SSTError):
        sst.critical_hf(0.0, 0.03, 1024.0)


def test_sigma_f_example(golden):
    """Sec. 4, Eq. 35: sigma_f = 1/(2 pi sigma) = 5.31 Hz for sigma = 0.03 s."""
    sf = 1.0 / (2 * np.pi * 0.03)
    assert abs(sf - golden["sigma_f_sim_hz"]["value"]) < golden["sigma_f_sim_hz"]["tol"]
    assert abs(6 * sf - golden["six_sigma_f_sim_hz"]["value"]) < golden["six_sigma_f_sim_hz"]["tol"]


def _batch_params(cfgs):
    arr = (sst.Params * len(cfgs))()
    keep = []
    for i, kw in enumerate(cfgs):
        d = _params(**kw)
        arr[i] = sst._params(d["n_samples"], d["fs"], d["win_len"], d["sigma"], d["hop"],
                             d["nfft"], d["f_lo"], d["f_hi"], d["subdiv"], d["thr_mode"],
                             d["thr"], None, None, keep)
    return arr


def test_batch_plan_shapes_and_workspace():
    cfgs = [dict(), dict(nfft=1024, win_len=255, sigma=32.0, hop=8, subdiv=2),
            dict(nfft=8192, win_len=2047, sigma=256.0, hop=32, f_hi=5000.0, subdiv=8,
                 n_samples=3000)]
    L = sst.lib()
    h = ctypes.c_void_p()
    assert L.sst_batch_plan(_batch_params(cfgs), len(cfgs), ctypes.byref(h)) == sst.SST_OK
    try:
        total = None
        for c, kw in enumerate(cfgs):
            sh = sst.Shape()
            assert L.sst_batch_query(h, c, ctypes.byref(sh)) == sst.SST_OK
            single = sst.Plan(**_params(**kw))
            assert (sh.n_frames, sh.n_src, sh.n_dst, sh.k1) == (
                single.n_frames, single.n_src, single.n_dst, single.k1)
            # the batch workspace holds every channel's own workspace
            assert sh.workspace_bytes >= single.shape.workspace_bytes
            total = sh.workspace_bytes if total is None else total
            assert sh.workspace_bytes == total
        sh = sst.Shape()
        assert L.sst_batch_query(h, len(cfgs), ctypes.byref(sh)) == sst.SST_E_ARG
        assert L.sst_batch_query(h, -1, ctypes.byref(sh)) == sst.SST_E_ARG
    finally:
        L.sst_batch_destroy(h)


def test_batch_plan_names_the_bad_channel():
    L = sst.lib()
    h = ctypes.c_void_p()
    rc = L.sst_batch_plan(_batch_params([dict(), dict(hop=0)]), 2, ctypes.byref(h))
    assert rc == sst.SST_E_ARG
    assert b"channel 1" in L.sst_last_error()
    assert L.sst_batch_plan(None, 1, ctypes.byref(h)) == sst.SST_E_ARG
    assert L.sst_batch_plan(_batch_params([dict()]), 0, ctypes.byref(h)) == sst.SST_E_ARG


def test_batch_refuses_work_before_bind_and_commit():
    L = sst.lib()
    h = ctypes.c_void_p()
    assert L.sst_batch_plan(_batch_params([dict(), dict()]), 2, ctypes.byref(h)) == sst.SST_OK
    try:
        assert L.sst_batch_forward(h, 0, 2, 0, None) == sst.SST_E_STATE
        assert L.sst_batch_inverse(h, 0, 2, None) == sst.SST_E_STATE
        assert L.sst_batch_commit(h, None) == sst.SST_E_STATE
        assert L.sst_batch_bind(h, None, 1 << 20, None) == sst.SST_E_WORKSPACE
        assert L.sst_batch_set_io(h, 2, None, None, None, 0, 0, None, None,
                                  None) == sst.SST_E_ARG
        # inverse buffers are checked when recorded
        assert L.sst_batch_set_io(h, 0, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                  ctypes.c_void_p(16), 0, 2, ctypes.c_void_p(16), None,
                                  None) == sst.SST_E_ARG
        assert L.sst_batch_set_io(h, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), None, 0, 0,
                                  None, None, ctypes.c_void_p(16)) == sst.SST_E_ARG
    finally:
        L.sst_batch_destroy(h)


def test_gemm_precision_validation():
    L = sst.lib()
    h = ctypes.c_void_p()
    keep = []
    ok = sst._params(1 << 15, 25600.0, 511, 64.0, 8, 512, 0.0, 6400.0, 1, "rel", 1e-3, None, None,
                     keep, "bf16")
    assert L.sst_plan(ctypes.byref(ok), ctypes.byref(h)) == sst.SST_OK
    L.sst_destroy(h)
    bad_hop = sst._params(1 << 15, 25600.0, 511, 64.0, 6, 512, 0.0, 6400.0, 1, "rel", 1e-3, None,
                          None, keep, "f16x3")
    assert L.sst_plan(ctypes.byref(bad_hop), ctypes.byref(h)) == sst.SST_E_UNSUPPORTED
    # narrow bands at any DFT size (the filter-bank use of the tiers)
    narrow = sst._params(1 << 15, 25600.0, 1023, 128.0, 8, 4096, 1000.0, 1500.0, 2, "rel", 1e-3,
                         None, None, keep, "f16x3")
    assert L.sst_plan(ctypes.byref(narrow), ctypes.byref(h)) == sst.SST_OK
    L.sst_destroy(h)
    # a DFT-matrix table beyond 64 MiB (4097 bins x 8191 taps) is refused
    big = sst._params(1 << 15, 25600.0, 8191, 900.0, 8, 8192, 0.0, 12800.0, 1, "rel", 1e-3, None,
                      None, keep, "bf16")
    assert L.sst_plan(ctypes.byref(big), ctypes.byref(h)) == sst.SST_E_UNSUPPORTED
    assert b"64 MiB" in L.sst_last_error()
    unknown = sst._params(1 << 15, 25600.0, 511, 64.0, 8, 512, 0.0, 6400.0, 1, "rel", 1e-3, None,
                          None, keep)
    unknown.precision = 7
    assert L.sst_plan(ctypes.byref(unknown), ctypes.byref(h)) == sst.SST_E_ARG
    # the batched calls run the FP32 FFT tier only
    arr = (sst.Params * 1)()
    arr[0] = ok
    assert L.sst_batch_plan(arr, 1, ctypes.byref(h)) == sst.SST_E_UNSUPPORTED
    # a histogram row that cannot fit 32 frames of LDS is refused at plan time
    wide = sst._params(1 << 15, 25600.0, 1023, 128.0, 8, 2048, 0.0, 12800.0, 4, "rel", 1e-3, None,
                       None, keep, "bf16")
    assert L.sst_plan(ctypes.byref(wide), ctypes.byref(h)) == sst.SST_E_UNSUPPORTED


def test_forward_static_rejects_oversized_workspace():
    """sst_forward_static refuses, before any device call, a plan whose workspace
    exceeds the fixed scratch (2^26 samples at hop 8: 8 bytes per frame of
    threshold state alone is 67 MB)."""
    p = sst.Plan(**_params(n_samples=1 << 26, hop=8))
    assert p.shape.workspace_bytes > 32 << 20
    st = sst.lib().sst_forward_static(p._h, None, 0, 0, None, None, 0, None)
    assert st == sst.SST_E_UNSUPPORTED
    assert b"static scratch" in sst.lib().sst_last_error()


def test_tuning_set_get_and_validation():
    p = sst.Plan(**_params())
    t = p.get_tuning()
    # c2 shape: a 1024-sample tile meets 130 frames, a 2048-sample one 194
    assert t["inv_tf"] == 4 and t["seed_step"] == 0
    p.set_tuning(fwd_wg_per_cu=2, seed_step=64, inv_tf=1)
    t = p.get_tuning()
    assert (t["fwd_wg_per_cu"], t["seed_step"], t["inv_tf"]) == (2, 64, 1)
    with pytest.raises(sst.SSTError) as e:
        p.set_tuning(inv_tf=3)
    assert e.value.status == sst.SST_E_ARG
    with pytest.raises(sst.SSTError) as e:
        p.set_tuning(seed_step=-1)
    assert e.value.status == sst.SST_E_ARG
    # hop 4 with a 1023-tap window: 1024 samples meet 512 frames, beyond the staged block
    q = sst.Plan(**_params(hop=4))
    assert q.get_tuning()["inv_tf"] == 1
    for tf in (4, 8):
        with pytest.raises(sst.SSTError) as e:
            q.set_tuning(inv_tf=tf)
        assert e.value.status == sst.SST_E_UNSUPPORTED


def test_tuning_inverse_groups():
    """Grouped staging of the wide inverse (2 or 4 destination groups staged
    together): a tuning choice, accepted where its LDS fits three or two
    workgroups per CU."""
    c3 = dict(nfft=8192, win_len=2047, sigma=256.0, hop=32, f_hi=5000.0, subdiv=8)
    p = sst.Plan(**_params(**c3))     # 1024 samples meet 98 frames: 4 groups in about 79 KiB
    t = p.get_tuning()
    assert (t["inv_tf"], t["inv_groups"]) == (8, 1)   # 2048 samples meet 130 frames
    for g in (2, 4):
        p.set_tuning(inv_groups=g)   # grouped staging takes tiles of 1024 samples
        assert (p.get_tuning()["inv_tf"], p.get_tuning()["inv_groups"]) == (4, g)
    p.set_tuning(inv_groups=1)
    assert (p.get_tuning()["inv_tf"], p.get_tuning()["inv_groups"]) == (8, 1)
    p.set_tuning(inv_tf=4, inv_groups=1)
    assert (p.get_tuning()["inv_tf"], p.get_tuning()["inv_groups"]) == (4, 1)
    with pytest.raises(sst.SSTError) as e:
        p.set_tuning(inv_tf=8, inv_groups=2)
    assert e.value.status == sst.SST_E_UNSUPPORTED
    p.set_tuning(inv_tf=1)
    assert p.get_tuning()["inv_groups"] == 1   # narrow tiles stage one group at a time
    with pytest.raises(sst.SSTError) as e:
        p.set_tuning(inv_tf=1, inv_groups=4)
    assert e.value.status == sst.SST_E_UNSUPPORTED
    for bad in (3, 5, -1):
        with pytest.raises(sst.SSTError) as e:
            p.set_tuning(inv_groups=bad)
        assert e.value.status == sst.SST_E_ARG
    q = sst.Plan(**_params())         # c2 shape: 130 frames per tile: 2 groups fit, 4 do not
    q.set_tuning(inv_groups=2)
    assert (q.get_tuning()["inv_tf"], q.get_tuning()["inv_groups"]) == (4, 2)
    with pytest.raises(sst.SSTError) as e:
        q.set_tuning(inv_groups=4)
    assert e.value.status == sst.SST_E_UNSUPPORTED


def test_tuning_cache_round_trip(tmp_path, monkeypatch):
    """The JSON cache is keyed by shape: an entry saved for one plan applies to a
    plan of the same shape (explicitly, and through SST_TUNE_CACHE at plan time)
    and not to another shape; entries of other shapes are kept on save."""
    import json
    path = str(tmp_path / "tune.json")
    a = sst.Plan(**_params())
    a.set_tuning(fwd_wg_per_cu=3, seed_step=16, inv_tf=1)
    a.tuning_save(path)
    other = sst.Plan(**_params(hop=8))
    other.set_tuning(seed_step=128)
    other.tuning_save(path)
    a.set_tuning(fwd_wg_per_cu=2, seed_step=16, inv_tf=1)
    a.tuning_save(path)                      # replaces a's entry, keeps the other one
    d = json.load(open(path))
    assert len(d) == 2
    key = [k for k in d if "H=16" in k][0]
    assert key.startswith("gfx950 nfft=4096 L=1023 H=16 n_src=1025 n_dst=4097")
    assert d[key] == {"fwd_wg_per_cu": 2, "seed_step": 16, "inv_tf": 1, "inv_groups": 1}
    b = sst.Plan(**_params())
    b.tuning_load(path)
    assert b.get_tuning() == {"fwd_wg_per_cu": 2, "seed_step": 16, "inv_tf": 1, "inv_groups": 1}
    monkeypatch.setenv("SST_TUNE_CACHE", path)
    c = sst.Plan(**_params())
    assert c.get_tuning()["seed_step"] == 16 and c.get_tuning()["inv_tf"] == 1
    e = sst.Plan(**_params(nfft=8192, win_len=2047, sigma=256.0))   # no entry: defaults
    assert e.get_tuning()["seed_step"] == 0
    with pytest.raises(sst.SSTError):
        e.tuning_load(path)
    monkeypatch.setenv("SST_TUNE_CACHE", str(tmp_path / "missing.json"))
    assert sst.Plan(**_params()).get_tuning()["seed_step"] == 0
