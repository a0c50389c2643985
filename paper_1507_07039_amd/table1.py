"""The paper's run-time experiment (Sec. III, Table I) on one MI355X.

For each size N (Ne = Na = N) the experiment takes random square networks W
with P = C = identity (the method's default when no interaction or
co-expression data exist, Sec. II-A; the library z-scores the identity like
any prior) and times the whole message-passing procedure per network, as the
paper does (reading and normalising W stay outside the timed region).  Two
ways of running a size on the GPU:

  single   one network after another through panda_run;
  batched  all networks of the size in one batch (grouped launches, graph
           replay); the time per network is the batch's time over their count
           (loading the priors included, as panda_run includes it).

The random W are U(0,1) entries (inputs.table1_priors; the paper does not
say how its random networks were drawn), seeds 1000 N + k.  Prints one JSON
line: seconds per network, iterations, and the paper's printed times on its
own CPUs (context only: other hardware, other programs).

    python -m paper_1507_07039_amd.table1 [--networks 100] [--sizes 125 250 ...]
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys
import time

import numpy as np

# Table I of the paper: average seconds per network over 100 random networks
# (C-code with g++ -O3, GNU Octave 3.8.2 and MATLAB R2014a, one thread each).
PAPER_TABLE1 = {
    125: {"C-code": 1.05, "Octave": 0.50, "MATLAB": 0.13},
    250: {"C-code": 4.65, "Octave": 0.62, "MATLAB": 0.54},
    500: {"C-code": 32.73, "Octave": 2.82, "MATLAB": 2.61},
    1000: {"C-code": 241.51, "Octave": 15.82, "MATLAB": 15.06},
    2000: {"C-code": 1954.5, "Octave": 98.59, "MATLAB": 95.04},
}


def networks(n: int, count: int, torch, panda):
    """count normalised random W of size n x n on the device."""
    from . import inputs as I
    out = []
    for k in range(count):
        W0, _, _ = I.table1_priors(1000 * n + k, n)
        W = torch.from_numpy(np.ascontiguousarray(W0, dtype=np.float32)).cuda()
        panda.normalize(W)
        out.append(W)
    torch.cuda.synchronize()
    return out


def time_single(Ws, torch, panda, alpha=0.1, tol=1e-3, max_iter=200):
    n = Ws[0].shape[0]
    o = panda.default_options()
    ws = panda.workspace(panda.workspace_bytes(n, n, o))
    out = tuple(torch.empty((n, n), dtype=torch.float32, device="cuda") for _ in range(3))
    panda.run(Ws[0], None, None, alpha, tol, max_iter, o, ws, out)  # warm-up (code load)
    torch.cuda.synchronize()
    secs, iters = [], []
    for W in Ws:
        t0 = time.perf_counter()
        res = panda.run(W, None, None, alpha, tol, max_iter, o, ws, out)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
        iters.append(res.iters)
    return secs, iters


def time_batched(Ws, torch, panda):
    n = Ws[0].shape[0]
    b = panda.Batch([(n, n)] * len(Ws))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, W in enumerate(Ws):
        b.load(i, W)
    code, steps = b.run(graph=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    iters = [b.status(i)[1] for i in range(len(Ws))]
    b.close()
    return total, steps, iters


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--networks", type=int, default=100)
    ap.add_argument("--sizes", type=int, nargs="+", default=sorted(PAPER_TABLE1))
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args(argv)
    import torch

    from . import panda
    panda.load_library()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    rows = []
    for n in args.sizes:
        Ws = networks(n, args.networks, torch, panda)
        secs, iters = time_single(Ws, torch, panda)
        row = {"N": n, "networks": len(Ws),
               "single_s_per_network": statistics.mean(secs),
               "single_p10_p90": [float(np.percentile(secs, 10)), float(np.percentile(secs, 90))],
               "iterations_mean": statistics.mean(iters),
               "iterations_min_max": [min(iters), max(iters)],
               "paper_s_per_network": PAPER_TABLE1.get(n)}
        if not args.no_batched:
            total, steps, biters = time_batched(Ws, torch, panda)
            row["batched_s_per_network"] = total / len(Ws)
            row["batched_steps"] = steps
            row["batched_iterations_match"] = biters == iters
        print(f"N={n}: {row}", file=sys.stderr, flush=True)
        rows.append(row)
        del Ws
        torch.cuda.empty_cache()
    print(json.dumps({"experiment": "Table I: whole message passing per random network, "
                                    "Ne = Na = N, P = C = identity",
                      "alpha": 0.1, "tol": 1e-3, "max_iter": 200, "rows": rows}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
