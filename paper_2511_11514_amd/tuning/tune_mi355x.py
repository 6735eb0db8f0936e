"""Run the schedule autotuner on an MI355X for the workload shapes and store the
table next to this file (mi355x.txt), which bench.py loads.

    python -m paper_2511_11514_amd.tuning.tune_mi355x
"""
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import paper_2511_11514_amd as ct  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mi355x.txt")


def size_class(n: int) -> int:
    """ceil(log2 n): the table's size class of a query or key count."""
    c = 0
    while (1 << c) < n:
        c += 1
    return c


def refine_pass(name: str, tmp: str, iters: int = 60, reps: int = 5) -> None:
    """Per-launch tuning times each schedule alone, but a gradient pass runs the
    cross sweeps and the self sweeps on two streams at once.  Refine the entries
    of the classes one pass of this workload uses (cross T x M and M x T, self
    M x M and T x T) by coordinate descent on the time of the whole pass."""
    c = W.CONFIGS[name]
    x, y, w, _g = W.config_inputs(c)
    dev = torch.device("cuda")
    x, y, w = (torch.as_tensor(a, device=dev) for a in (x, y, w))

    def run():
        ct.sinkhorn_grad(x, y, w, eps=c.eps, iters=iters, value=True, grad_w=True)

    def timed():
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ct.tuning_save(tmp)
    table = {}
    for line in open(tmp):
        f = line.split()
        if f and not f[0].startswith("#"):
            table[tuple(int(v) for v in f[:3])] = [int(v) for v in f[3:]]

    def load():
        with open(tmp, "w") as fh:
            for k, v in sorted(table.items()):
                fh.write(" ".join(str(t) for t in k + tuple(v)) + "\n")
        ct.tuning_clear()
        ct.tuning_load(tmp)

    keys = []
    for nq, nk in ((c.T, c.M), (c.M, c.T), (c.M, c.M), (c.T, c.T)):
        k = (c.d, size_class(nq), size_class(nk))
        if k not in keys:
            keys.append(k)
    load()
    best = timed()
    print(f"refine {name}: start {best:.2f} ms per {iters}-iteration pass", flush=True)
    for k in keys:
        cur = table.get(k)
        for R in (1, 2, 4):
            for WS in (2, 4):
                for bpc in (2, 4, 8, 16):
                    cand = [R, WS, bpc, 1, cur[4] if cur else 0]
                    if cur and cand[:4] == cur[:4]:
                        continue
                    table[k] = cand
                    load()
                    ms = timed()
                    if ms < best:
                        best, cur = ms, cand
                    if cur is None:
                        table.pop(k)
                    else:
                        table[k] = cur
        print(f"refine {name}: class {k} -> {cur}, {best:.2f} ms", flush=True)
    load()


def main(out=OUT):
    ct.tuning_clear()
    t0 = time.time()
    for name in ("planner_2d", "grad_2d", "autograd_3d", "roofline_2d"):
        c = W.CONFIGS[name]
        ct.autotune_sinkhorn(c.T, c.M, c.d, c.eps)
        print(f"tuned {name} ({time.time() - t0:.0f} s)", flush=True)
    c = W.CONFIGS["batched_2d"]
    for tc in range(9, 14):            # T in [500, 8000]
        for mc in range(10, 16):       # M in [1024, 32768]
            ct.autotune_sinkhorn(1 << tc, 1 << mc, 2, c.eps)
    print(f"tuned per-problem classes of the batch ({time.time() - t0:.0f} s)", flush=True)
    # last among the class entries, so that nothing overwrites the refined ones
    for name in ("grad_2d", "autograd_3d"):
        refine_pass(name, out + ".refine")
        print(f"refined {name} ({time.time() - t0:.0f} s)", flush=True)
    os.remove(out + ".refine")
    # batched path: lockstep schedule, then the persistent kernel's (queries per lane,
    # key-splitting waves), by timing the 256-problem batch
    probs = W.batch_inputs(c)
    dev = torch.device("cuda")
    xs = [torch.as_tensor(p[0], device=dev) for p in probs]
    ys = [torch.as_tensor(p[1], device=dev) for p in probs]
    tmp = out + ".part"
    ct.tuning_save(tmp)
    base = open(tmp).read()

    def time_batch(persistent):
        bs = ct.BatchedSinkhorn(xs, ys, None, eps=c.eps, iters=6, persistent=persistent)
        bs.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        bs.run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    # lockstep launches (the default batched execution): key (2, 1, 0)
    lbest = None
    for R in (2, 4):
        for WS in (2, 4):
            for bpc in (4, 8, 16):
                with open(tmp, "w") as fh:
                    fh.write(base + f"2 1 0 {R} {WS} {bpc} 1 0\n")
                ct.tuning_clear()
                ct.tuning_load(tmp)
                ms = time_batch(False)
                print(f"lockstep R={R} WS={WS} blocks/CU={bpc}: {ms:.2f} ms", flush=True)
                if lbest is None or ms < lbest[0]:
                    lbest = (ms, R, WS, bpc)
    base += f"2 1 0 {lbest[1]} {lbest[2]} {lbest[3]} 1 {int(lbest[0] * 1000)}\n"
    best = None
    for R, WS in [(1, 4), (2, 4), (2, 2), (4, 4), (4, 2), (4, 1)]:
        with open(tmp, "w") as fh:
            fh.write(base + f"2 0 0 {R} {WS} 1 0 0\n")
        ct.tuning_clear()
        ct.tuning_load(tmp)
        bs = ct.BatchedSinkhorn(xs, ys, None, eps=c.eps, iters=6, persistent=True)
        bs.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        bs.run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        print(f"batched R={R} WS={WS}: {ms:.2f} ms", flush=True)
        if best is None or ms < best[0]:
            best = (ms, R, WS)
    with open(tmp, "w") as fh:
        fh.write(base + f"2 0 0 {best[1]} {best[2]} 1 0 {int(best[0] * 1000)}\n")
    ct.tuning_clear()
    ct.tuning_load(tmp)
    ct.tuning_save(out)
    os.remove(tmp)
    print("wrote", out, len(ct.tuning_table()), "entries", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else OUT)
