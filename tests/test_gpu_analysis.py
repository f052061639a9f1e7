"""GPU: the analysis measures (sst_renyi: Renyi entropy of Sec. 3, Eq. 32)
against the float64 oracle on identical inputs."""
import sys

import numpy as np
import pytest

import oracle
from workloads import make_c2, make_paper_eq30

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sst():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2003_07065_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("wl", ["eq30", "c2-shape"])
def test_renyi_matches_oracle(sst, wl):
    """R of the SST matrix T (complex64) and of |T| as float32 and float16, each
    against the oracle on the same values; the float64 sums are reduced in a
    fixed order, so repeated calls agree bit for bit."""
    w = make_paper_eq30() if wl == "eq30" else make_c2(n=1 << 15)
    c = w.cfg
    plan = sst.Plan.from_config(w.n, c, device="cuda")
    T = plan.forward(torch.from_numpy(w.x).cuda())
    out = sst.renyi(T, 3)
    out2 = sst.renyi(T, 3)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    Tc = T.cpu().numpy()
    r_o = oracle.renyi(Tc.astype(np.complex128), 3.0)
    r_g = float(out[2].cpu())
    s1 = float(np.sum(np.abs(Tc.astype(np.complex128)) ** 2))
    _say(f"[renyi] {wl}: gpu {r_g:.9f} oracle {r_o:.9f} bits; sum P {float(out[0].cpu()):.6e} "
         f"vs {s1:.6e}")
    assert abs(r_g - r_o) <= 1e-6
    assert abs(float(out[0].cpu()) - s1) <= 1e-6 * s1
    for dt in (torch.float32, torch.float16):
        mag = T.abs().to(dt)
        r_m = float(sst.renyi(mag, 3)[2].cpu())
        ref = oracle.renyi(mag.cpu().numpy().astype(np.float64), 3.0)
        assert abs(r_m - ref) <= 1e-6, (dt, r_m, ref)
    # a sub-block of columns through the row stride
    sub = float(sst.renyi(T[:, 100:700], 3)[2].cpu())
    assert abs(sub - oracle.renyi(Tc[:, 100:700].astype(np.complex128), 3.0)) <= 1e-6
    for alpha in (2, 4):
        r_a = float(sst.renyi(T, alpha)[2].cpu())
        assert abs(r_a - oracle.renyi(Tc.astype(np.complex128), float(alpha))) <= 1e-6
