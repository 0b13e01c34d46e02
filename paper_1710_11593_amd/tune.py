"""Plan tuner: measures the leaf size L and the dense/FFT crossover s* of the
recursive solve on the current GPU and writes the plan cache that
fracsolve_create reads for options leaf = 0 / crossover = 0.

For every (product precision, width bucket) it times whole solves through the
C ABI (the float32 form with its float64 refinement step) over the candidate
leaf sizes and crossovers, and keeps the fastest.  Run as

    python -m paper_1710_11593_amd.tune [--out PATH] [--N 16384] [--reps 3]

The default output path is the one the library reads: $FRACSOLVE_TUNE_CACHE,
else $XDG_CACHE_HOME/fracsolve/plan.json, else ~/.cache/fracsolve/plan.json.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

BUCKETS = (64, 128, 256, 512, 1024, 2048, 4096)
LEAVES = (4, 8, 16)
CROSSOVERS = (-1, 16, 32, 64, 128, 256, 512, 1024)
PRECISIONS = ("fp64", "fp32")


def default_path() -> str:
    p = os.environ.get("FRACSOLVE_TUNE_CACHE")
    if p:
        return p
    x = os.environ.get("XDG_CACHE_HOME")
    if x:
        return os.path.join(x, "fracsolve", "plan.json")
    return os.path.join(os.path.expanduser("~"), ".cache", "fracsolve", "plan.json")


def _source(M, N, gamma, dev):
    """A smooth source of 4 sine modes (inputs only; no solver arithmetic)."""
    import numpy as np
    import torch

    x = np.arange(1, M + 1) / (M + 1)
    t = np.arange(1, N + 1) / N
    G = np.stack([(1.0 + j) * t ** (1.0 + 0.3 * j) for j in range(4)], axis=1)
    S = np.stack([np.sin((j + 1) * math.pi * x) for j in range(4)])
    return (torch.from_numpy(G).to(dev) @ torch.from_numpy(S).to(dev)).contiguous()


def time_plan(M, N, precision, leaf, crossover, reps=3, gamma=0.5, equation="diffusion", f=None):
    """Median wall time (ms) of one solve with this plan, or None if the
    library refuses the combination."""
    import torch

    from paper_1710_11593_amd import binding

    dev = torch.device("cuda")
    if f is None:
        f = _source(M, N, gamma, dev)
    try:
        s = binding.Solver([dict(gamma=gamma, M=M, N=N)], precision=precision,
                           refine_steps=1 if precision != "fp64" else 0, leaf=leaf, crossover=crossover,
                           equation=equation)
    except binding.FracsolveError:
        return None
    out = torch.empty_like(f)
    try:
        s.solve([f], out=[out])
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            s.solve([f], out=[out])
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
    finally:
        s.close()
    ts.sort()
    return ts[len(ts) // 2]


def tune(N=16384, reps=3, precisions=PRECISIONS, buckets=BUCKETS, leaves=LEAVES, crossovers=CROSSOVERS,
         log=print):
    import torch

    entries, timings = [], {}
    dev = torch.device("cuda")
    for prec in precisions:
        pcode = {"fp64": 0, "fp32": 1}[prec]
        for M in buckets:
            f = _source(M, N, 0.5, dev)
            best = None
            for leaf in leaves:
                for cross in crossovers:
                    if cross > 0 and cross >= N:
                        continue
                    ms = time_plan(M, N, prec, leaf, cross, reps=reps, f=f)
                    timings["%s M=%d L=%d s*=%d" % (prec, M, leaf, cross)] = ms
                    if ms is not None and (best is None or ms < best[0]):
                        best = (ms, leaf, cross)
            del f
            if best is None:
                continue
            log("tune: %s M<=%d: L=%d s*=%d (%.3f ms at N=%d)" % (prec, M, best[1], best[2], best[0], N))
            entries.append({"precision": pcode, "equation": 0, "m_max": M, "leaf": best[1],
                            "crossover": best[2], "ms": round(best[0], 4)})
    # widths above the largest bucket take its plan
    for prec in precisions:
        pcode = {"fp64": 0, "fp32": 1}[prec]
        last = [e for e in entries if e["precision"] == pcode]
        if last:
            e = dict(last[-1])
            e["m_max"] = 1 << 20
            entries.append(e)
    props = torch.cuda.get_device_properties(0)
    return {"fracsolve_plan": 1, "device": getattr(props, "gcnArchName", props.name), "N": N, "reps": reps,
            "entries": entries, "timings_ms": timings}


def write(plan: dict, path: str):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(plan, fh, indent=1)
    os.replace(tmp, path)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default="")
    ap.add_argument("--N", type=int, default=16384)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--precision", default="fp64,fp32")
    ap.add_argument("--buckets", default=",".join(str(b) for b in BUCKETS))
    args = ap.parse_args(argv)
    plan = tune(N=args.N, reps=args.reps, precisions=tuple(args.precision.split(",")),
                buckets=tuple(int(b) for b in args.buckets.split(",")))
    path = args.out or default_path()
    write(plan, path)
    print("tune: plan written to %s" % path, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
