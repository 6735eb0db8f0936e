"""CPU checks of the C ABI: the library loads, exports every function declared
in include/ct.h, and rejects invalid arguments on the host before any GPU work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ct.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ct_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    from paper_2511_11514_amd import lib
    L = lib()
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert L.ct_version().startswith(b"ct ")


def test_binding_declares_every_symbol():
    from paper_2511_11514_amd import _lib
    assert set(_declared()) <= set(_lib._SIGS)


def _call_sinkhorn(**kw):
    from paper_2511_11514_amd import _lib
    L = _lib.lib()
    args = dict(x=1, T=10, y=1, w=None, M=20, o=_lib.SinkhornOpts(2, 10, 0.01, _lib.CT_DEBIAS),
                gx=1, gw=None, val=None, pot=None, pp=None, aux=None, ws=256, nb=1 << 30)
    args.update(kw)
    P = ctypes.c_void_p
    return L.ct_sinkhorn_grad(P(args["x"]), args["T"], P(args["y"]), P(args["w"]), args["M"],
                              ctypes.byref(args["o"]), P(args["gx"]), P(args["gw"]),
                              P(args["val"]), P(args["pot"]), P(args["pp"]), P(args["aux"]),
                              P(args["ws"]), args["nb"], None)


def test_sinkhorn_rejects_bad_arguments_before_launch():
    from paper_2511_11514_amd import _lib
    O = _lib.SinkhornOpts
    assert _call_sinkhorn(x=None) == _lib.CT_E_ARG
    assert _call_sinkhorn(T=0) == _lib.CT_E_SHAPE
    assert _call_sinkhorn(M=-3) == _lib.CT_E_SHAPE
    assert _call_sinkhorn(o=O(4, 10, 0.01, 1)) == _lib.CT_E_SHAPE
    assert _call_sinkhorn(o=O(2, 10, 0.0, 1)) == _lib.CT_E_ARG
    assert _call_sinkhorn(o=O(2, 10, float("nan"), 1)) == _lib.CT_E_ARG
    assert _call_sinkhorn(o=O(2, -1, 0.01, 1)) == _lib.CT_E_ARG
    assert _call_sinkhorn(o=O(2, 10, 0.01, 1 << 20)) == _lib.CT_E_ARG
    assert _call_sinkhorn(o=O(2, 10, 0.01, _lib.CT_FUSED | _lib.CT_UNFUSED)) == _lib.CT_E_ARG
    assert _call_sinkhorn(o=O(2, 10, 0.01, _lib.CT_TINY | _lib.CT_FUSED)) == _lib.CT_E_ARG
    assert _call_sinkhorn(o=O(2, 10, 0.01, _lib.CT_TINY | _lib.CT_UNFUSED)) == _lib.CT_E_ARG
    assert _call_sinkhorn(o=O(2, 10, 0.01, _lib.CT_MESH | _lib.CT_TINY)) == _lib.CT_E_ARG
    assert _call_sinkhorn(o=O(2, 10, 0.01, _lib.CT_MESH | _lib.CT_FUSED)) == _lib.CT_E_ARG
    assert _call_sinkhorn(o=O(2, 10, 0.01, _lib.CT_MESH | _lib.CT_UNFUSED)) == _lib.CT_E_ARG
    assert _call_sinkhorn(o=O(2, 10, 0.01, _lib.CT_GRAD_W)) == _lib.CT_E_ARG   # grad_w missing
    assert _call_sinkhorn(o=O(2, 10, 0.01, _lib.CT_WARM_START)) == _lib.CT_E_ARG  # pot missing
    assert _call_sinkhorn(gx=None) == _lib.CT_E_ARG
    assert _call_sinkhorn(ws=None) == _lib.CT_E_ARG
    assert _call_sinkhorn(ws=257) == _lib.CT_E_WORKSPACE
    assert _call_sinkhorn(nb=16) == _lib.CT_E_WORKSPACE
    msg = _lib.lib().ct_last_error().decode()
    assert "workspace" in msg


def test_workspace_size_is_monotone_and_rejects_bad_shapes():
    from paper_2511_11514_amd import _lib
    L = _lib.lib()
    o = _lib.SinkhornOpts(2, 10, 0.01, 1)
    a = L.ct_sinkhorn_workspace_size(1000, 2000, ctypes.byref(o))
    b = L.ct_sinkhorn_workspace_size(2000, 4000, ctypes.byref(o))
    assert 0 < a < b
    assert L.ct_sinkhorn_workspace_size(0, 10, ctypes.byref(o)) == 0
    bad = _lib.SinkhornOpts(5, 10, 0.01, 1)
    assert L.ct_sinkhorn_workspace_size(10, 10, ctypes.byref(bad)) == 0


def test_tuning_table_round_trip_and_validation(tmp_path):
    """The tuning table text format: eight fields per entry, read back through
    ct_tuning_entry and ct_tuning_save; malformed lines are rejected."""
    import paper_2511_11514_amd as ct
    from paper_2511_11514_amd import _lib
    ct.tuning_clear()
    try:
        f = tmp_path / "t.txt"
        f.write_text("# comment\n2 12 14 2 4 8 1 17\n\n3 14 16 4 2 16 0 123\n")
        ct.tuning_load(str(f))
        assert sorted(ct.tuning_table()) == [(2, 12, 14, 2, 4, 8, 1, 17),
                                             (3, 14, 16, 4, 2, 16, 0, 123)]
        g = tmp_path / "g.txt"
        ct.tuning_save(str(g))
        ct.tuning_clear()
        assert ct.tuning_table() == []
        ct.tuning_load(str(g))
        assert len(ct.tuning_table()) == 2
        for bad in ("2 12 14 2 4 8 17\n",          # seven fields
                    "2 12 14 3 4 8 1 17\n",        # R = 3
                    "2 12 14 2 3 8 1 17\n",        # WS = 3
                    "2 12 14 2 4 32 1 17\n",       # 32 blocks per CU
                    "4 12 14 2 4 8 1 17\n"):       # d = 4
            h = tmp_path / "bad.txt"
            h.write_text(bad)
            with pytest.raises(_lib.CtError):
                ct.tuning_load(str(h))
        buf = (ctypes.c_int32 * 8)()
        assert _lib.lib().ct_tuning_entry(99, buf) == _lib.CT_E_ARG
    finally:
        ct.tuning_clear()


def test_probe_rejects_bad_arguments_before_launch():
    from paper_2511_11514_amd import _lib
    import ctypes
    L = _lib.lib()
    out = (ctypes.c_double * 6)()
    n = L.ct_probe_workspace_size()
    assert n >= 4 * 256
    assert L.ct_probe_alu_rates(None, ctypes.c_void_p(256), n, None) == _lib.CT_E_ARG
    assert L.ct_probe_alu_rates(out, None, n, None) == _lib.CT_E_ARG
    assert L.ct_probe_alu_rates(out, ctypes.c_void_p(256), n - 1, None) == _lib.CT_E_WORKSPACE


def test_plan_ensemble_rejects_bad_arguments_before_launch():
    import numpy as np
    from paper_2511_11514_amd import _lib
    L = _lib.lib()
    s0 = np.zeros(6)
    Q, R = np.eye(3), 0.01 * np.eye(3)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    prob = _lib.PlanProblem(_lib.CT_DYN_DOUBLE_INTEGRATOR, 3, 10, 0.05, dp(s0))
    sk = _lib.SinkhornOpts(3, 10, 0.01, _lib.CT_DEBIAS)
    u = np.zeros((2, 10, 3))
    val = np.zeros(2)
    best = ctypes.c_int32()
    P = ctypes.c_void_p
    def call(flow=_lib.CT_FLOW_SINKHORN, S=2, uu=u, ws=256):
        o = _lib.PlanOpts(flow, 1, 0.5, dp(Q), dp(R), sk, 0.0)
        return L.ct_plan_ensemble(ctypes.byref(prob), ctypes.byref(o), S, P(256), None, 20,
                                  None if uu is None else dp(uu), None, dp(val), ctypes.byref(best),
                                  P(ws), 1 << 30, None)
    assert call(flow=_lib.CT_FLOW_SVGD) in (_lib.CT_E_ARG, _lib.CT_E_UNSUPPORTED)
    assert call(S=0) == _lib.CT_E_ARG
    assert call(uu=None) == _lib.CT_E_ARG
    assert call(ws=0) == _lib.CT_E_ARG
    o = _lib.PlanOpts(_lib.CT_FLOW_SINKHORN, 1, 0.5, dp(Q), dp(R), sk, 0.0)
    assert L.ct_plan_ensemble_workspace_size(ctypes.byref(prob), ctypes.byref(o), 2, 20, 0) > 0
    assert L.ct_plan_ensemble_workspace_size(ctypes.byref(prob), ctypes.byref(o), 0, 20, 0) == 0


def test_grid_entry_points_reject_bad_arguments_before_launch():
    from paper_2511_11514_amd import _lib
    L = _lib.lib()
    P = ctypes.c_void_p

    def desc(n=(4, 5, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 2.0, 0.0), u=256, floor=0.0):
        return _lib.GridDesc((ctypes.c_int32 * 3)(*n), (ctypes.c_float * 3)(*lo),
                             (ctypes.c_float * 3)(*hi), u, floor)

    def score(g=None, d=2, T=10, x=256, out=256):
        g = g if g is not None else desc()
        return L.ct_grid_score(P(x), T, d, ctypes.byref(g), P(out), None)

    assert score(d=4) == _lib.CT_E_SHAPE
    assert score(T=0) == _lib.CT_E_SHAPE
    assert score(x=None) == _lib.CT_E_ARG
    assert score(out=None) == _lib.CT_E_ARG
    assert score(g=desc(u=None)) == _lib.CT_E_ARG
    assert score(g=desc(n=(1, 5, 1))) == _lib.CT_E_SHAPE
    assert score(g=desc(n=(4, 5, 1)), d=3) == _lib.CT_E_SHAPE            # axis 2 has 1 node
    assert score(g=desc(hi=(1.0, 0.0, 0.0))) == _lib.CT_E_ARG             # hi <= lo on axis 1
    assert score(g=desc(lo=(float("nan"), 0.0, 0.0))) == _lib.CT_E_ARG
    assert score(g=desc(floor=-1.0)) == _lib.CT_E_ARG
    assert L.ct_grid_score(P(256), 10, 2, None, P(256), None) == _lib.CT_E_ARG

    g = desc()
    n = L.ct_grid_samples_workspace_size(ctypes.byref(g), 2)
    assert n > 0
    assert L.ct_grid_samples_workspace_size(ctypes.byref(desc(n=(400, 500, 1))), 2) > n
    assert L.ct_grid_samples_workspace_size(ctypes.byref(g), 4) == 0
    assert L.ct_grid_samples_workspace_size(ctypes.byref(desc(n=(1 << 15, 1 << 14, 1))), 2) == 0
    M = ctypes.c_int64()

    def samples(g=g, y=256, w=256, m=ctypes.byref(M), ws=256, nb=n):
        return L.ct_grid_samples(ctypes.byref(g), 2, P(y), P(w), m, P(ws), nb, None)

    assert samples(y=None) == _lib.CT_E_ARG
    assert samples(w=None) == _lib.CT_E_ARG
    assert samples(m=None) == _lib.CT_E_ARG
    assert samples(ws=None) == _lib.CT_E_ARG
    assert samples(ws=257) == _lib.CT_E_WORKSPACE
    assert samples(nb=n - 1) == _lib.CT_E_WORKSPACE
    assert samples(g=desc(floor=float("inf"))) == _lib.CT_E_ARG


def test_svgd_score_and_grid_plan_reject_bad_arguments_before_launch():
    import numpy as np
    from paper_2511_11514_amd import _lib
    L = _lib.lib()
    P = ctypes.c_void_p
    n = L.ct_svgd_workspace_size(100, 2)
    assert L.ct_svgd_grad_score(P(256), 100, 2, None, 0.0, P(256), None, P(256), n, None) == _lib.CT_E_ARG
    assert L.ct_svgd_grad_score(P(256), 100, 4, P(256), 0.0, P(256), None, P(256), n, None) == _lib.CT_E_SHAPE
    assert L.ct_svgd_grad_score(P(256), 100, 2, P(256), float("nan"), P(256), None, P(256), n,
                                None) == _lib.CT_E_ARG
    assert L.ct_svgd_grad_score(P(256), 100, 2, P(256), 0.0, P(256), None, P(256), n - 1,
                                None) == _lib.CT_E_WORKSPACE
    s0 = np.zeros(3)
    Q, R = np.eye(2), 0.01 * np.eye(2)
    u = np.zeros((10, 2))
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    prob = _lib.PlanProblem(_lib.CT_DYN_UNICYCLE, 2, 10, 0.05, dp(s0))
    o = _lib.PlanOpts(_lib.CT_FLOW_SVGD_GRID, 1, 0.05, dp(Q), dp(R), _lib.SinkhornOpts(2, 10, 0.01, 1),
                      0.0, None)
    assert L.ct_plan(ctypes.byref(prob), ctypes.byref(o), None, None, 0, None, dp(u), None, None,
                     P(256), 1 << 30, None) == _lib.CT_E_ARG
    assert "grid" in L.ct_last_error().decode()
    assert L.ct_plan_workspace_size(ctypes.byref(prob), ctypes.byref(o), 0) > \
        L.ct_svgd_workspace_size(10, 2)


def test_status_sync_rejects_bad_workspaces():
    from paper_2511_11514_amd import _lib
    L = _lib.lib()
    assert L.ct_status_sync(None, 0.0, None, None, None, None) == _lib.CT_E_ARG
    assert L.ct_status_sync(ctypes.c_void_p(257), 0.0, None, None, None, None) == \
        _lib.CT_E_WORKSPACE
    assert L.ct_status_sync(ctypes.c_void_p(256), -1.0, None, None, None, None) == _lib.CT_E_ARG


def test_status_codes_match_the_header():
    """The binding's status constants are the header's."""
    import re
    from paper_2511_11514_amd import _lib
    src = open(os.path.join(ROOT, "include", "ct.h")).read()
    codes = dict(re.findall(r"#define (CT_(?:OK|WARN_[A-Z_]+|E_[A-Z_]+)) \(?(-?\d+)\)?", src))
    assert set(codes) >= {"CT_OK", "CT_WARN_NOT_CONVERGED", "CT_E_ARG", "CT_E_SHAPE",
                          "CT_E_NONFINITE", "CT_E_WORKSPACE", "CT_E_HIP", "CT_E_UNSUPPORTED",
                          "CT_E_CAPTURE"}
    for name, v in codes.items():
        assert getattr(_lib, name) == int(v), name


def test_static_scratch_entry_rejects_before_launch():
    """ct_sinkhorn_grad_static validates like ct_sinkhorn_grad and refuses a problem
    whose scratch exceeds its static array, all on the host (nothing enqueued)."""
    from paper_2511_11514_amd import _lib
    L = _lib.lib()
    P = ctypes.c_void_p
    assert L.ct_sinkhorn_static_scratch_bytes() == 64 << 20

    def call(T, M, o, x=1, gx=1):
        return L.ct_sinkhorn_grad_static(P(x), T, P(1), None, M, ctypes.byref(o), P(gx), None,
                                         None, None, None, None, None)
    O = _lib.SinkhornOpts
    ok = O(2, 10, 0.01, _lib.CT_DEBIAS)
    assert call(10, 20, ok, x=None) == _lib.CT_E_ARG
    assert call(10, 20, ok, gx=None) == _lib.CT_E_ARG
    assert call(0, 20, ok) == _lib.CT_E_SHAPE
    assert call(10, 20, O(2, 10, -1.0, 1)) == _lib.CT_E_ARG
    assert L.ct_sinkhorn_workspace_size(4096, 16384, ctypes.byref(ok)) > 64 << 20
    assert call(4096, 16384, ok) == _lib.CT_E_WORKSPACE
    assert b"static scratch" in L.ct_last_error()


def test_svgd_workspace_grows_as_the_header_states():
    """ct_svgd_workspace_size as include/ct.h describes it: the bracket's sample and
    candidate buffers appear at T = 11000 (4 MiB + 4 bytes per 125 pairs), the
    group boxes' buffers at T = 24576 (another 8 bytes per 125 pairs and 4 bytes per
    pair of 64-point groups); d = 2 and 3 agree up to O(T)."""
    from paper_2511_11514_amd import _lib
    L = _lib.lib()
    pairs = lambda T: T * (T - 1) // 2
    for d in (2, 3):
        ws = lambda T: L.ct_svgd_workspace_size(T, d)
        assert ws(10999) < ws(11000)
        assert ws(11000) - ws(10999) >= (1 << 22) + 4 * (pairs(11000) // 125) * 0.99
        assert ws(24576) - ws(24575) >= 8 * (pairs(24576) // 125) * 0.99
        ng = (24576 + 63) // 64
        assert ws(24576) - ws(24575) >= 4 * ng * (ng + 1) // 2
        assert 200e6 < ws(65536) < 300e6 and 400e6 < ws(92681) < 500e6
        # above the median's limit (only a given bandwidth is accepted) the bracket's buffers go
        assert ws(92682) < ws(92681) / 10
