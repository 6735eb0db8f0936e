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
