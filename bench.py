#!/usr/bin/env python3
"""Benchmark of the PANDA message-passing iteration on one MI355X.

Workload: synthetic priors shaped like the paper's realistic networks
(T = 700 transcription factors x G = 18000 genes, Sec. II-F), drawn by
paper_1507_07039_amd.inputs and z-scored on the GPU by the library.

Printed (one JSON line):
  value        seconds per message-passing iteration (median over the timed
               steps; a step is one full iteration: R, A + W, h, P, C, diagonals)
  time_to_converge_s / iters_to_converge   panda_run from the priors to h < tol
  roofline     the dominant kernel (A = T(W, C) fused with the W update):
               algorithmic FLOPs 2 T G^2 per launch over its event-timed
               average duration, against the FP32 matrix-core peak
  cpu_baseline the FP64 oracle: one whole iteration of this workload,
               measured on every host thread, and on one thread a column
               slice of the same iteration scaled up; with the CPU model
  accuracy     W of both forms against the stored FP64 oracle run of this
               workload (tests/golden/, written by the oracle alone) at its
               checkpoints, max-abs and relative to max|W|
  chosen_form  the split-BF16 products (and the learned warm start, judged
               against the plain run: accepted only within 1e-3 max|W|)
HBM traffic of the dominant kernels (rocprofv3 FETCH_SIZE / WRITE_SIZE) and
their kernel-trace durations come from summaries recorded in profiles/ and
are reported only while the kernel sources still hash to the digest recorded
with them.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1507_07039_amd import inputs as I  # noqa: E402

METRIC = "s/iteration & time-to-converge at T=700,G=18k: plain FP32 vs chosen form"
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0


# library options of each form: each runs in the layout that is faster for it
# (split-BF16 on packed C, plain FP32 on C stored whole; --packed-c sets both)
PLAIN_OPTS = {"packed_c": 0}
CHOSEN_OPTS = {"packed_c": 1}


def form_opts(precision):
    return CHOSEN_OPTS if precision else PLAIN_OPTS

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "iteration_T700_G18000_hbm_traffic.md")
TRACE_FILE = os.path.join(ROOT, "profiles", "iteration_T700_G18000_kernel_trace.md")
GOLDEN_FILE = os.path.join(ROOT, "tests", "golden", "oracle_panda-T700-G18000.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def csrc_digest() -> str:
    """sha256 over the library's kernel sources (file names and contents)."""
    d = os.path.join(ROOT, "paper_1507_07039_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def recorded_values(path, suffix):
    """{key: value} of the machine-readable lines (- `key`: value) of a
    profile summary whose key ends in suffix, or {} when the summary is
    missing or the kernels changed since it was recorded."""
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        line = line.strip()
        if line.startswith("- `") and "`: " in line:
            k, v = line[3:].split("`: ", 1)
            vals[k] = v.strip()
    if vals.get("csrc_sha256") != csrc_digest():
        return {}
    return {k: float(v) for k, v in vals.items() if k.endswith(suffix)}


def recorded_traffic():
    """{key: bytes per launch} from the counter summary."""
    return recorded_values(TRAFFIC_FILE, "_bytes")


def recorded_trace_us():
    """{key: average kernel duration in us} from the kernel-trace summary."""
    return recorded_values(TRACE_FILE, "_us")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def accuracy_vs_golden(torch, panda, W, P, C, precision: int):
    """W of the form against the stored FP64 oracle run at its checkpoints:
    {t: [max-abs, max-abs / max(1, max|W|)]} over the stored sampled entries.
    The stored run started from the oracle's z-scores rounded to FP32; these
    inputs are the library's z-scores (FP64 moments in another summation
    order, the same FP32 values up to rare last-bit flips), so the figures
    include that input difference."""
    if not os.path.exists(GOLDEN_FILE):
        return None
    g = json.load(open(GOLDEN_FILE))
    Ne, Na = W.shape
    if (g["workload"]["T"], g["workload"]["G"]) != (Ne, Na):
        return None
    ctx = panda.Context(Ne, Na, panda.default_options(tol=0.0, precision=precision, **form_opts(precision)))
    ctx.load(W, P, C)
    iw = g["idx"]["W"]
    rows = torch.as_tensor(iw[0], device="cuda")
    cols = torch.as_tensor(iw[1], device="cuda")
    out = {}
    for t in range(1, len(g["h_trace"]) + 1):
        ctx.iterate()
        snap = g["snapshots"].get(str(t))
        if snap is None:
            continue
        Wg = ctx.state()[0]
        got = Wg[rows, cols].double().cpu().numpy()
        want = np.asarray(snap["W"], dtype=np.float64)
        err = float(np.abs(got - want).max())
        out[str(t)] = [err, err / max(1.0, float(np.abs(want).max()))]
        del Wg
    ctx.close()
    return out


def gpu_inputs(w: I.Workload, torch, panda):
    W0, P0, C0 = I.workload_priors(w)
    dev = [torch.from_numpy(np.ascontiguousarray(M, dtype=np.float32)).cuda() for M in (W0, P0, C0)]
    del W0, P0, C0
    for M in dev:
        panda.normalize(M)
    torch.cuda.synchronize()
    return dev


def time_iterations(torch, panda, W, P, C, steps: int, warmup: int, precision: int = 0):
    Ne, Na = W.shape
    # tol = 0: no iteration inside the timing is skipped by convergence
    opts = panda.default_options(tol=0.0, max_iter=1 << 30, precision=precision, **form_opts(precision))
    ctx = panda.Context(Ne, Na, opts)
    ctx.load(W, P, C)
    for _ in range(warmup):
        ctx.iterate()
    ctx.set_timing(True)
    per = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        ctx.iterate()  # returns after h is read back, i.e. after the iteration ran
        per.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    phases = ctx.phase_times()
    ctx.close()
    return per, total, phases


def time_to_converge(torch, panda, W, P, C, runs: int, precision: int = 0):
    Ne, Na = W.shape
    opts = panda.default_options(precision=precision, **form_opts(precision))
    ws = panda.workspace(panda.workspace_bytes(Ne, Na, opts))
    out = (torch.empty_like(W), torch.empty_like(P), torch.empty_like(C))
    times, res = [], None
    for _ in range(runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = panda.run(W, P, C, opts=opts, ws=ws, out=out)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return times, res


def warm_start_eval(torch, panda, W, P, C, plain):
    """The learned warm start (weights trained on plain runs at 200 x 4000)
    with the split-BF16 products, judged against the plain run."""
    from paper_1507_07039_amd import warmstart as WSG
    wfile = os.path.join(ROOT, "paper_1507_07039_amd", "weights", "warmstart_T200_G4000")
    if not os.path.exists(wfile + ".npy"):
        return {"available": False}
    meta = json.load(open(wfile + ".json"))
    params = torch.from_numpy(np.load(wfile + ".npy")).cuda()
    # t0 from the training set alone (median stopping iteration minus the tuned k)
    t0 = max(0, int(meta["train"]["plain_stop_median"]) - int(meta.get("t0_offset", 0)))
    opts = panda.default_options(precision=1)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    warm = WSG.warm_run(params, W, P, C, t0, meta.get("sketch_seed", 0), opts)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - ts
    err = (warm.W - plain.W).abs().max().item()
    scale = max(1.0, plain.W.abs().max().item())
    accepted = warm.converged and err <= 1e-3 * scale
    ev = meta.get("eval_T700_G18000", {})
    return {"available": True, "t0": t0, "polish_iters": warm.polish, "frozen": warm.frozen,
            "time_s": t_warm, "max_abs_dW_vs_plain": err, "rel": err / scale,
            "accepted": accepted,
            "prediction_rel_err_vs_converged": ev.get("prediction", {}).get("rel_err_vs_converged"),
            "amplification_eps_1e-4": ev.get("amplification_eps_1e-4"),
            "note": ("judged by the plain run; not accepted, so the plain result stands and the "
                     "warm start is not part of the chosen form's time")}


def oracle_iteration(O, W, P, C, frac: float = 1.0, report=None):
    """Time one FP64 oracle iteration as oracle_step runs it: the similarity
    matrices R = T(P, W), A = T(W, C) (with the W update), T(W', W'^T) and
    T(W'^T, W') by the oracle's Tfunction, which gathers each column once and
    runs every row against it.  frac < 1 computes only the leading frac of
    each matrix's columns (all rows) and scales each part by its column
    fraction, which keeps that access pattern; frac = 1 is the whole
    iteration, measured.  The C side runs in column blocks so that progress
    can be reported.  Returns (seconds, {part: seconds})."""
    a = 0.1
    Ne, Na = W.shape
    nA = max(1, int(round(Na * frac)))
    nE = max(1, int(round(Ne * frac)))
    parts = {}

    def timed(name, fn, scale):
        t0 = time.perf_counter()
        out = fn()
        parts[name] = parts.get(name, 0.0) + (time.perf_counter() - t0) * scale
        if report:
            report(f"{name}: {parts[name]:.1f} s")
        return out

    R = timed("R", lambda: O.tanimoto(P, np.ascontiguousarray(W[:, :nA])), Na / nA)
    Wn = timed("A+W", lambda: (1 - a) * W[:, :nA] + a * 0.5 * (
        O.tanimoto(W, np.ascontiguousarray(C[:, :nA])) + R), Na / nA)
    del R
    if nA < Na:  # the columns not computed keep their W (the matrices below need a full W)
        Wn = np.concatenate([Wn, W[:, nA:]], axis=1)
    Wt = np.ascontiguousarray(Wn.T)
    timed("P", lambda: O.tanimoto(Wn, np.ascontiguousarray(Wt[:, :nE])), Ne / nE)
    for lo in range(0, nA, 4096):
        hi = min(nA, lo + 4096)
        timed("C", lambda: (1 - a) * C[:, lo:hi] + a * O.tanimoto(
            Wt, np.ascontiguousarray(Wn[:, lo:hi])), Na / nA)
    return sum(parts.values()), parts


def cpu_baseline(w: I.Workload):
    """The FP64 oracle on this workload: one whole iteration, measured, on
    every host thread the process may use; and on one thread, the same
    iteration on a 1/64 column slice of every similarity matrix, scaled."""
    from oracle import oracle as O
    W0, P0, C0 = I.workload_priors(w)
    W, P, C = O.normalize(W0), O.normalize(P0), O.normalize(C0)
    del W0, P0, C0
    Ne, Na = W.shape
    cores = O.set_threads(0)  # the OpenMP default: every host thread this process may use
    full, parts = oracle_iteration(O, W, P, C, 1.0, lambda m: log("cpu baseline, " + m))
    O.set_threads(1)
    frac = 1.0 / 64
    one, parts1 = oracle_iteration(O, W, P, C, frac, lambda m: log("cpu baseline, 1 thread, " + m))
    O.set_threads(cores)
    return {"value": full, "unit": "s/iteration", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"one whole FP64 oracle iteration at T={Ne} G={Na}, measured: every entry "
                       f"of R, A, W, T(W, W^T) and T(W^T, W) by the element-wise Tfunction"),
            "phases_s": parts,
            "single_thread": {"value": one, "unit": "s/iteration", "cores": 1,
                              "sample": (f"the same iteration on one thread over the first 1/64 "
                                         f"of the columns of each similarity matrix (all rows), "
                                         f"each part scaled by its column fraction"),
                              "phases_s": parts1}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="human", choices=["human", "small", "large"])
    ap.add_argument("--converge-runs", type=int, default=5)
    ap.add_argument("--no-converge", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-only", action="store_true", help="skip the split-BF16 form")
    ap.add_argument("--no-warm-start", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a device copy, a read-only sum and a fill of this many MiB "
                         "(counter calibration)")
    ap.add_argument("--packed-c", type=int, default=None, choices=[0, 1],
                    help="store C as its upper tiles (both forms); default: the library's")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the comparison with the stored oracle run")
    args = ap.parse_args()
    if args.packed_c is not None:
        PLAIN_OPTS["packed_c"] = CHOSEN_OPTS["packed_c"] = args.packed_c
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU layout is "
              "described in the design notes but not built", file=sys.stderr)
        return 2

    import torch

    from paper_1507_07039_amd import panda
    panda.load_library()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    w = {"human": I.HUMAN, "small": I.SMALL, "large": I.LARGE}[args.workload]
    log(f"workload {w.name}: generating priors")
    W, P, C = gpu_inputs(w, torch, panda)
    Ne, Na = W.shape
    flops = {"R": 2.0 * Ne * Ne * Na, "A+W": 2.0 * Ne * Na * Na, "P-partial": 1.0 * Ne * Ne * Na,
             "C": 1.0 * Ne * Na * Na}

    def measure(precision):
        per, total, phases = time_iterations(torch, panda, W, P, C, args.steps, args.warmup,
                                             precision)
        ms = {k: (v[0] / v[1] if v[1] else None) for k, v in phases.items()}
        rates = {k: flops[k] / (ms[k] * 1e-3) / 1e12 for k in flops if ms.get(k)}
        return per, ms, rates

    traffic = recorded_traffic()
    trace = recorded_trace_us()
    algo = {"A+W": flops["A+W"]}

    def trace_frac(prefix, peak, mult=1.0):
        us = trace.get(prefix + "_aw_product_us"), trace.get(prefix + "_aw_fixup_us")
        if us[0] is None or us[1] is None:
            return None
        tot = us[0] + us[1]
        return {"kernel_us": tot, "achieved": mult * algo["A+W"] / (tot * 1e-6) / 1e12,
                "frac": mult * algo["A+W"] / (tot * 1e-6) / 1e12 / peak}

    log("timing iterations (plain FP32)")
    per, ms, rates = measure(0)
    s_iter = statistics.median(per)
    achieved = rates["A+W"]
    result = {
        "metric": METRIC, "value": s_iter, "unit": "s/iteration", "higher_is_better": False,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": s_iter * 1e3,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "T": Ne, "G": Na, "alpha": 0.1, "tol": 1e-3,
                   "form": "plain-fp32", "parallelism": "single-gpu"},
        "s_per_iteration_p10_p90": [float(np.percentile(per, 10)), float(np.percentile(per, 90))],
        "phase_ms": ms, "phase_tflops": rates,
        "roofline": {"bound": "mfma",
                     "kernel": "A+W: k_rect_streamk<BlockGemm<64,128,1,4,XK,-,16>, EpiWUpdate> + "
                               "k_rect_fixup",
                     "achieved": achieved, "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_MFMA_TFLOPS,
                     "traffic": traffic.get("fp32_aw_traffic_bytes"),
                     "from_kernel_trace": trace_frac("fp32", PEAK_FP32_MFMA_TFLOPS)},
    }
    if not args.plain_only:
        log("timing iterations (split-BF16 form)")
        per3, ms3, rates3 = measure(1)
        # this form computes the next iteration's R inside the C update's
        # launch (after warm-up the R phase holds only its timing events)
        if ms3.get("C") is not None:
            ms3["C+R"] = ms3.pop("C") + (ms3.pop("R", None) or 0.0)
            rates3.pop("R", None)
            rates3.pop("C", None)
            rates3["C+R"] = (flops["C"] + flops["R"]) / (ms3["C+R"] * 1e-3) / 1e12
        # executed bf16 flops: three products per FP32-equivalent product
        bf_rate = 3.0 * rates3["A+W"]
        result["chosen_form"] = {
            "form": "bf16x3" + (" + packed C" if CHOSEN_OPTS.get("packed_c") else ""),
            "plain_layout": "packed C" if PLAIN_OPTS.get("packed_c") else "C stored whole",
            "s_per_iteration": statistics.median(per3),
            "speedup_per_iteration": s_iter / statistics.median(per3),
            "phase_ms": ms3, "phase_tflops_fp32_equivalent": rates3,
            "roofline": {"bound": "mfma",
                         "kernel": ("A+W: k_rect_streamk<BlockGemmB3P<256,128,4,2,FP32 C,3,32,"
                                    + ("packed" if CHOSEN_OPTS.get("packed_c") else "whole")
                                    + " C>, EpiWUpdate> + k_rect_fixup"),
                         "achieved": bf_rate, "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                         "frac": bf_rate / PEAK_BF16_MFMA_TFLOPS,
                         "traffic": traffic.get(("b3p" if CHOSEN_OPTS.get("packed_c") else "b3")
                                                + "_aw_traffic_bytes"),
                         "from_kernel_trace": trace_frac("b3p" if CHOSEN_OPTS.get("packed_c") else "b3",
                                                         PEAK_BF16_MFMA_TFLOPS, 3.0)},
        }
    if not args.no_converge:
        log("time to converge (plain FP32)")
        times, res = time_to_converge(torch, panda, W, P, C, args.converge_runs)
        result["time_to_converge_s"] = statistics.median(times)
        result["iters_to_converge"] = res.iters
        result["h_final"] = res.h
        result["converged"] = res.status == panda.OK
        if not args.plain_only:
            Wp = res.W.clone()
            log("time to converge (split-BF16 form)")
            times3, res3 = time_to_converge(torch, panda, W, P, C, args.converge_runs, 1)
            cf = result["chosen_form"]
            cf["time_to_converge_s"] = statistics.median(times3)
            cf["iters_to_converge"] = res3.iters
            cf["converged"] = res3.status == panda.OK
            cf["speedup_time_to_converge"] = result["time_to_converge_s"] / cf["time_to_converge_s"]
            cf["max_abs_dW_vs_plain"] = (res3.W - Wp).abs().max().item()
            cf["max_abs_W_plain"] = Wp.abs().max().item()
            if not args.no_warm_start and w is I.HUMAN:
                cf["warm_start"] = warm_start_eval(torch, panda, W, P, C, res)
    if not args.no_accuracy and w is I.HUMAN:
        log("accuracy against the stored oracle run")
        acc = {"plain-fp32": accuracy_vs_golden(torch, panda, W, P, C, 0)}
        if not args.plain_only:
            acc["bf16x3"] = accuracy_vs_golden(torch, panda, W, P, C, 1)
        result["accuracy_vs_oracle"] = {
            "what": "W at the stored oracle checkpoints t: [max-abs error, max-abs / max(1, max|W|)]",
            **acc}
    if args.copy_calibration:
        # known traffic for the counters: a copy (n reads + n writes), a
        # read-only sum (n reads) and a fill (n writes)
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        _ = a.sum().item()
        b.fill_(2.0)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = n * 4
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        result["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
