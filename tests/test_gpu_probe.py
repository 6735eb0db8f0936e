"""The issue-rate probe behind the sweep roofline (ct_probe_alu_rates): it runs,
reports rates in the range the hardware allows, and its peak bounds what the
sweep kernel achieves on a large launch."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_probe_rates_are_physical(ct):
    r = ct.probe_alu_rates()
    # lanes per clock per CU: 4 SIMDs; nothing can issue above 4 x 64 lanes
    for k in ("add", "fma", "exp"):
        assert 1.0 < r[k] <= 256.0, r
    # the exp is slower than the add (transcendental unit), and the add not slower than the FMA
    assert r["exp"] < r["add"] and r["fma"] <= r["add"] * 1.05, r
    assert 1.0 < r["mfma_f32"] <= 512.0, r
    # overlap ratio: between full overlap (0.5) and none (1), with timing noise
    assert 0.45 < r["mfma_exp_overlap"] < 1.3, r
    assert r["clock_hz"] > 1e8


def test_large_sweep_stays_below_issue_roof(ct):
    """One lagged sweep launch at a large shape, timed by events stamped with the
    kernel's start and end, does not exceed the issue-rate roof of its instruction
    mix (a check on the roofline model and on the timing itself)."""
    import sys, os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    import workloads as W
    r = ct.probe_alu_rates()
    roof = bench.pair_roof(2, r, clock=r["clock_hz"])
    x, y, w, _g = W.config_inputs(W.CONFIGS["roofline_2d"], T=16384, M=65536)
    dev = torch.device("cuda")
    xt, yt = torch.as_tensor(x, device=dev), torch.as_tensor(y, device=dev)
    from paper_2511_11514_amd import _lib
    L = _lib.lib()
    ct.sinkhorn_grad(xt, yt, None, eps=0.002, iters=2, debias=False)   # warm
    torch.cuda.synchronize()
    L.ct_profile_clear()
    L.ct_profile_enable(1)
    ct.sinkhorn_grad(xt, yt, None, eps=0.002, iters=6, debias=False)
    torch.cuda.synchronize()
    L.ct_profile_enable(0)
    import ctypes
    kind = (ctypes.c_int32 * 4)()
    pr, t = ctypes.c_double(), ctypes.c_float()
    best = 0.0
    for i in range(L.ct_profile_count()):
        _lib.check("ct_profile_read", L.ct_profile_read(i, kind, ctypes.byref(pr), ctypes.byref(t)))
        if kind[0] == 1 and kind[1] == 0 and t.value > 0:
            best = max(best, pr.value / (t.value * 1e-3))
    L.ct_profile_clear()
    nominal = bench.pair_roof(2, bench.NOMINAL_RATES)
    print(f"best launch {best:.3e} pairs/s, probed roof {roof:.3e}, nominal roof {nominal:.3e}")
    assert best > 0.0
    # the issue-rate bound holds; the probe's chains can run a little below the
    # instruction mix's own rates, so the probed roof is only a loose check
    assert best < 1.02 * nominal, (best, nominal)
    assert best < 1.10 * roof, (best, roof)
