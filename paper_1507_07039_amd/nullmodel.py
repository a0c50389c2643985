"""Permutation null of the PANDA edges on one MI355X (node-label randomisation
on input, an option of the paper's C implementation, Sec. III).

Times panda_null on the T=700, G=18000 workload (inputs.py; priors z-scored
on the device): K null instances, each relabelling the genes of the
co-expression prior with its own permutation (numpy PCG64, seed 1000 + k) and
running the message passing to convergence, in the split-BF16 form (default)
or plain FP32.  Reports seconds per null instance, the iterations of each
instance, and the relabelling kernel (panda_permute_sym) on its own: 8 N_a^2
bytes moved per call (read and write of C) against 8 TB/s.  Prints one JSON
line.

    python -m paper_1507_07039_amd.nullmodel [--instances 4] [--fp32]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--instances", type=int, default=4)
    ap.add_argument("--fp32", action="store_true")
    args = ap.parse_args(argv)
    import torch

    from . import inputs as I
    from . import panda
    panda.load_library()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    W0, P0, C0 = I.workload_priors(I.HUMAN)
    W, P, C = (torch.from_numpy(np.ascontiguousarray(M, dtype=np.float32)).cuda()
               for M in (W0, P0, C0))
    del W0, P0, C0
    for M in (W, P, C):
        panda.normalize(M)
    Ne, Na = W.shape
    K = args.instances
    gp = torch.from_numpy(np.stack([np.random.default_rng(1000 + k).permutation(Na)
                                    for k in range(K)]).astype(np.int32)).cuda()
    o = panda.default_options(precision=0 if args.fp32 else 1)
    ws = panda.workspace(panda.load_library().panda_null_workspace_bytes(Ne, Na, o))

    # the relabelling kernel alone
    out = torch.empty_like(C)
    for _ in range(2):
        panda.permute_sym(C, gp[0])
    torch.cuda.synchronize()
    reps = 10
    lib = panda.load_library()
    import ctypes as ct
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    perm_ms = []
    for r in range(reps):  # the host check of each call synchronises, so time calls one by one
        a.record()
        st = lib.panda_permute_sym(ct.c_void_p(C.data_ptr()), Na, Na, ct.c_void_p(gp[r % K].data_ptr()),
                                   ct.c_void_p(out.data_ptr()), Na, panda._stream())
        b.record()
        torch.cuda.synchronize()
        if st != panda.OK:
            raise panda.PandaError(st, lib.panda_last_error().decode())
        perm_ms.append(a.elapsed_time(b))
    pm = float(np.median(perm_ms))
    gbs = 8.0 * Na * Na / (pm * 1e-3) / 1e9

    panda.null(W, P, C, gene_perm=gp[:1].contiguous(), opts=o, ws=ws)  # warm-up (code load)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = panda.null(W, P, C, gene_perm=gp, opts=o, ws=ws)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    print(json.dumps({
        "what": "permutation null (panda_null): genes of C relabelled per instance",
        "workload": I.HUMAN.name, "form": "fp32" if args.fp32 else "bf16x3", "instances": K,
        "s_per_instance": total / K, "iterations": res.iters, "status": res.status,
        "permute_sym_ms": pm, "permute_sym_GBs": gbs,
        "permute_sym_frac_of_hbm": gbs / HBM_PEAK_GBS,
        "null_sd_median": float(res.sd.median().item())}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
