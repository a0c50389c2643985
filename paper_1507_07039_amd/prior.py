"""The co-expression prior of Sec. II-A on one MI355X: time panda_pearson
(the Pearson correlation between the genes of an expression matrix, genes x
samples) and place it on its roofline.

The correlations are one FP32 MFMA product of the centred, normalised rows
with their transpose, taken on the upper triangle of tiles and mirrored:
S G (G + 1) flops algorithmic (2 S per distinct entry, diagonal included,
unpadded sizes) against FP32 MFMA's 157.3 TFLOP/s; the output, 4 G^2 bytes,
is the bulk of the HBM traffic.  The input
is the synthetic expression matrix of the T=700, G=18000 workload (inputs.py:
200 samples, 20 latent factors) unless sizes are given.  Prints one JSON line.

    python -m paper_1507_07039_amd.prior [--genes 18000] [--samples 200] [--reps 20]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

FP32_MFMA_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


def measure(G: int, S: int, reps: int = 20, torch=None, panda=None) -> dict:
    from . import inputs as I
    if (G, S) == (I.HUMAN.G, I.HUMAN.S):
        E = I.workload_expression(I.HUMAN)
    else:
        E = I.expression(G, 1, G, 0.0, 0.0, S, 20)
    Ed = torch.from_numpy(np.ascontiguousarray(E, dtype=np.float32)).cuda()
    lib = panda.load_library()
    ws = panda.workspace(lib.panda_pearson_workspace_bytes(G, S))
    C = torch.empty((G, G), dtype=torch.float32, device="cuda")
    import ctypes as ct
    args = (ct.c_void_p(Ed.data_ptr()), G, S, S, ct.c_void_p(C.data_ptr()), G,
            ct.c_void_p(ws.data_ptr()), ws.numel(), panda._stream())

    def call():
        st = lib.panda_pearson(*args)
        if st != panda.OK:
            raise panda.PandaError(st, lib.panda_last_error().decode())

    for _ in range(3):
        call()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        call()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    flops = float(S) * G * (G + 1)
    tf = flops / (ms * 1e-3) / 1e12
    out_gbs = 4.0 * G * G / (ms * 1e-3) / 1e9
    return {"what": "Pearson co-expression prior (panda_pearson)", "genes": G, "samples": S,
            "ms": ms, "reps": reps,
            "roofline": {"bound": "mfma", "achieved": tf, "peak": FP32_MFMA_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tf / FP32_MFMA_PEAK_TFLOPS,
                         "flops": flops},
            "output_write_GBs": out_gbs, "output_write_frac_of_hbm": out_gbs / HBM_PEAK_GBS}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--genes", type=int, default=18000)
    ap.add_argument("--samples", type=int, default=200)
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args(argv)
    import torch

    from . import panda
    panda.load_library()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    print(json.dumps(measure(args.genes, args.samples, args.reps, torch, panda)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
