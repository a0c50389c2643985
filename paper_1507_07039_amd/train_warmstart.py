#!/usr/bin/env python3
"""Train the warm-start network on plain runs and evaluate it.

  python -m paper_1507_07039_amd.train_warmstart [--train 256] [--steps 3000]

1. Training set: `--train` synthetic networks at T x G (default 200 x 4000,
   seeds 10000..), all run to convergence by the plain method in one batch;
   features and targets of every edge.
2. Adam on minibatches of edges (the library's MFMA kernels).
3. t0 tuning on `--holdout` further networks of the training size: the warm
   start is run from t0 = (median stopping iteration of the training set) - k
   for several k, and the k with the smallest error against the plain runs is
   kept.
4. Evaluation on the T=700 x G=18000 workload: iterations of the plain run,
   iterations of the polish from the warm state, max-abs W error against the
   plain run (and relative to max|W|), rank agreement of the edge weights,
   and whether the judge (max-abs error <= 1e-3 max(1, max|W|)) accepts it.

Writes the weights (FP32, .npy) and a JSON summary next to them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_1507_07039_amd import inputs as I  # noqa: E402
from paper_1507_07039_amd import panda  # noqa: E402
from paper_1507_07039_amd import warmstart as WSG  # noqa: E402

WEIGHTS = os.path.join(HERE, "weights", "warmstart_T200_G4000.npy")


def log(*a):
    print("[train_warmstart]", *a, flush=True)


def gen(shape_seed):
    T, G, seed = shape_seed
    return I.priors(seed, T, G, 0.03, 0.01, 200, 20)


def rank_agreement(a, b, n=1_000_000, seed=0):
    """Spearman correlation of two weight sets on a random sample of edges."""
    a = a.reshape(-1).cpu().numpy()
    b = b.reshape(-1).cpu().numpy()
    idx = np.random.default_rng(seed).choice(a.size, size=min(n, a.size), replace=False)
    ra = np.argsort(np.argsort(a[idx])).astype(np.float64)
    rb = np.argsort(np.argsort(b[idx])).astype(np.float64)
    return float(np.corrcoef(ra, rb)[0, 1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=256)
    ap.add_argument("--holdout", type=int, default=4)
    ap.add_argument("--T", type=int, default=200)
    ap.add_argument("--G", type=int, default=4000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--sketch-seed", type=int, default=7)
    ap.add_argument("--ks", default="0,2,5,10,15,20,30")
    ap.add_argument("--no-eval", action="store_true")
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    import torch
    panda.load_library()
    t0 = time.perf_counter()
    specs = [(args.T, args.G, 10000 + i) for i in range(args.train + args.holdout)]
    with ThreadPoolExecutor(8) as ex:
        nets = list(ex.map(gen, specs))
    log(f"{len(nets)} networks {args.T}x{args.G} generated in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    data = WSG.training_set(nets[:args.train], sketch_seed=args.sketch_seed)
    torch.cuda.synchronize()
    stops = data["stops"]
    log(f"training set: {data['F'].shape[0]} edges, plain stops median {np.median(stops)} "
        f"(min {min(stops)}, max {max(stops)}) in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    params, losses = WSG.train(data, steps=args.steps, batch=args.batch, lr=args.lr, seed=0)
    torch.cuda.synchronize()
    log(f"trained {args.steps} steps in {time.perf_counter() - t0:.1f} s: loss "
        f"{losses[0]:.4f} -> {losses[-1]:.4f}")
    del data
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, params.cpu().numpy())
    med = int(np.median(stops))
    # t0 tuning on held-out networks of the training size
    ks = [int(k) for k in args.ks.split(",")]
    hold = [WSG.normalized(*n) for n in nets[args.train:]]
    plains = [panda.run(*h) for h in hold]
    tune = {}
    for k in ks:
        t0k = max(0, med - k)
        errs, pol = [], []
        for h, pl in zip(hold, plains):
            w = WSG.warm_run(params, *h, t0k, args.sketch_seed)
            errs.append((w.W - pl.W).abs().max().item() / max(1.0, pl.W.abs().max().item()))
            pol.append(w.polish)
        tune[k] = {"t0": t0k, "rel_err": float(np.median(errs)), "polish": float(np.mean(pol))}
        log(f"k={k}: t0={t0k} median rel err {tune[k]['rel_err']:.3e}, polish {tune[k]['polish']}")
    kbest = min(ks, key=lambda k: tune[k]["rel_err"])
    summary = {"train": {"networks": args.train, "T": args.T, "G": args.G,
                         "edges": args.train * args.T * args.G, "steps": args.steps,
                         "batch": args.batch, "lr": args.lr, "loss_first": losses[0],
                         "loss_last": losses[-1], "plain_stop_median": med},
               "t0_tuning": {str(k): v for k, v in tune.items()}, "k": kbest,
               "t0_offset": med - tune[kbest]["t0"], "sketch_seed": args.sketch_seed}
    if not args.no_eval:
        W0, P0, C0 = I.workload_priors(I.HUMAN)
        W, P, C = WSG.normalized(W0, P0, C0)
        del W0, P0, C0
        torch.cuda.synchronize()
        ts = time.perf_counter()
        plain = panda.run(W, P, C)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - ts
        res = {}
        for name, t0e in (("t0_from_training", tune[kbest]["t0"]),
                          ("t0_scaled", max(0, plain.iters - (med - tune[kbest]["t0"])))):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            j = WSG.judged_run(params, W, P, C, t0e, args.sketch_seed, plain=plain)
            torch.cuda.synchronize()
            t_warm = time.perf_counter() - ts
            res[name] = {"t0": t0e, "polish_iters": j["warm"].polish,
                         "converged": j["warm"].converged, "frozen": j["warm"].frozen,
                         "max_abs_err": j["max_abs_err"],
                         "max_abs_W": j["scale"], "rel_err": j["max_abs_err"] / j["scale"],
                         "accepted": j["accepted"],
                         "rank_agreement": rank_agreement(j["warm"].W, plain.W),
                         "time_s_incl_judge": t_warm}
            log(name, res[name])
        # how close the prediction is to the converged W, and how close a warm
        # state at t0 would have to be to the plain run's own state there
        Wp = WSG.predict(params, W, P, C, args.sketch_seed)
        pred = {"max_abs_err_vs_converged": (Wp - plain.W).abs().max().item(),
                "rel_err_vs_converged": (Wp - plain.W).abs().max().item()
                / max(1.0, plain.W.abs().max().item()),
                "rank_agreement": rank_agreement(Wp, plain.W)}
        t0s = sorted({2, 5, 10, 20, 40, max(1, plain.iters - 5)})
        amp, _ = WSG.amplification(W, P, C, t0s, eps=1e-4, plain=plain)
        for t0e, a in amp.items():
            a["required_rel_accuracy_at_t0"] = 1e-3 / max(a["amp"], 1e-30)
        log("prediction", pred)
        log("amplification", amp)
        summary["eval_T700_G18000"] = {"plain_iters": plain.iters, "plain_time_s": t_plain,
                                       "prior_rank_agreement": rank_agreement(W, plain.W),
                                       "prediction": pred, "amplification_eps_1e-4": amp,
                                       "runs": res}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps(summary))
    return 0


if __name__ == "__main__":
    sys.exit(main())
