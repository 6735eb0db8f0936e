"""GPU check of the allocation-free entry point ct_sinkhorn_grad_static against
ct_sinkhorn_grad (same kernels and schedules, so identical bits), on two calls in
a row that share the static scratch, the second smaller than the first (its
scratch still holds the first call's contents), plus the first call against the
FP64 oracle at 1e-5 (Sec. II-B, eqs. 5-7)."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _call(ct, x, y, w, eps, iters, static):
    out = ct.sinkhorn_grad(x, y, w, eps=eps, iters=iters, value=True, grad_w=True,
                           potentials=True, aux=True, static_scratch=static)
    torch.cuda.synchronize()
    return out


def test_static_scratch_matches_workspace_call_twice(ct):
    from paper_2511_11514_amd import _lib
    _lib.lib().ct_profile_enable(0)
    dev = torch.device("cuda")
    cfg = W.CONFIGS["grad_2d"]
    eps, iters = 0.01, 40
    for T, M in ((1500, 2601), (301, 777)):
        print(f"static scratch case T={T} M={M}", flush=True)
        x, y, _w, _g = W.config_inputs(cfg, T=T, M=M)
        w = np.random.default_rng(T).uniform(0.5, 1.5, M).astype(np.float32)
        t = lambda a: torch.as_tensor(a, device=dev)
        ref = _call(ct, t(x), t(y), t(w), eps, iters, static=False)
        got = _call(ct, t(x), t(y), t(w), eps, iters, static=True)
        for name in ("grad_x", "grad_w", "value", "pot", "pot_plus", "aux"):
            a, b = getattr(got, name), getattr(ref, name)
            assert torch.equal(a, b), (T, M, name, (a - b).abs().max().item())
        if T == 1500:
            r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters)
            assert rel(got.grad_x.cpu().numpy(), r.grad_x) < 1e-5
            assert rel(got.grad_w.cpu().numpy(), r.grad_w) < 1e-5
            assert abs(got.value.item() - r.value) / abs(r.value) < 1e-5


def test_static_scratch_rejects_oversized_problem(ct):
    from paper_2511_11514_amd import _lib
    dev = torch.device("cuda")
    x = torch.rand(4096, 2, device=dev)
    y = torch.rand(16384, 2, device=dev)
    with pytest.raises(_lib.CtError) as e:
        ct.sinkhorn_grad(x, y, None, eps=0.01, iters=5, static_scratch=True)
    assert e.value.code == _lib.CT_E_WORKSPACE
