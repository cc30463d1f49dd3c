"""Trains the learned cost model on this device's own timings and writes it.

The library generates sections on the program workload's 32-field struct
(N = 2^16 .. 2^24, 1-16 reads, 1-2 writes, half of them gathers of 1-32
neighbours) under many layouts, times each one on the device, and trains
the 16 -> 64 -> 64 -> 64 -> 1 network with its own forward, backward and
Adam kernels (adha_costmodel_train), several times from different initial
weights (an ensemble whose mean prediction the planner uses).  The model file (checksummed) and a
JSON report of the run are written side by side; the benchmark and the
learned-plan test load the file kept in this package.

    python -m paper_1407_4859_amd.train_costmodel OUT.adha [--samples N] [--epochs E]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("out", help="model file to write")
    ap.add_argument("--samples", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--min-log2n", type=int, default=16)
    ap.add_argument("--max-log2n", type=int, default=24)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--ensemble", type=int, default=5, help="networks trained on the same timings")
    a = ap.parse_args(argv)
    import torch
    from paper_1407_4859_amd import adha as A
    if not torch.cuda.is_available():
        print("a GPU is needed to time the training sections", file=sys.stderr)
        return 1
    ctx = A.Ctx(0)
    t0 = time.time()
    rep = A.costmodel_train(ctx, A.train_opts(n_samples=a.samples, epochs=a.epochs, min_log2_n=a.min_log2n,
                                              max_log2_n=a.max_log2n, reps=3, seed=a.seed, progress_every=1000,
                                              ensemble=a.ensemble))
    A.costmodel_save(ctx, a.out)
    info = {"samples": a.samples, "epochs": a.epochs, "ensemble": a.ensemble, "log2n": [a.min_log2n, a.max_log2n], "seed": a.seed,
            "device": torch.cuda.get_device_name(0), "seconds": round(time.time() - t0, 1),
            "report": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in rep.items()}}
    with open(os.path.splitext(a.out)[0] + ".json", "w") as fh:
        json.dump(info, fh, indent=1)
    print(json.dumps(info), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
