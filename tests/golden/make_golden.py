"""Write the oracle's reference trajectories used by the parity tests.

Calls only the FP64 oracle (``oracle/``) and the seeded input generators; no
value here comes from the GPU library.  Usage:

    python tests/golden/make_golden.py small     # seconds
    python tests/golden/make_golden.py human     # about an hour on 8 cores

Shared starting point for both paths: the raw priors are z-scored by the
oracle in FP64 and rounded to FP32 (round-to-nearest-even).  The GPU path
starts from those FP32 arrays and the oracle from the same values in FP64, so
input rounding is not counted as error.  The SHA-256 of the FP32 bytes is
stored so that a test can tell when its regenerated inputs differ.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1507_07039_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def normalized_f32(w: I.Workload):
    W0, P0, C0 = I.workload_priors(w)
    out = []
    for M in (W0, P0, C0):
        out.append(np.ascontiguousarray(O.normalize(M).astype(np.float32)))
    return tuple(out)


def digest(*arrs) -> str:
    h = hashlib.sha256()
    for a in arrs:
        h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
    return h.hexdigest()


def sample_idx(seed: int, rows: int, cols: int, n: int, symmetric_offdiag: bool = False):
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.integers(0, rows, size=n)
    c = rng.integers(0, cols, size=n)
    if symmetric_offdiag:
        same = r == c
        c[same] = (c[same] + 1) % cols
    return r, c


def main(which: str):
    w = {"small": I.SMALL, "human": I.HUMAN}[which]
    checkpoints = {1, 2, 5, 10, 20}
    nsamp = 2048 if which == "human" else 256
    t0 = time.time()
    Wf, Pf, Cf = normalized_f32(w)
    W, P, C = (x.astype(np.float64) for x in (Wf, Pf, Cf))
    opts = O.Options()
    Ne, Na = W.shape
    rw, cw = sample_idx(1, Ne, Na, nsamp)
    rp, cp = sample_idx(2, Ne, Ne, nsamp, True)
    rc, cc = sample_idx(3, Na, Na, nsamp, True)
    dp = np.arange(Ne) if Ne <= nsamp else sample_idx(4, Ne, 1, nsamp)[0]
    dc = np.arange(Na) if Na <= nsamp else sample_idx(5, Na, 1, nsamp)[0]
    snaps = {}
    hs = []
    t = 0
    conv = False
    while t < opts.max_iter and not conv:
        t += 1
        W, P, C, h, conv = O.step(W, P, C, t, opts)
        hs.append(h)
        print(f"[{which}] t={t} h={h:.6e} ({time.time() - t0:.0f}s)", flush=True)
        if t in checkpoints or conv:
            snaps[str(t)] = {
                "W": W[rw, cw].tolist(), "P": P[rp, cp].tolist(), "C": C[rc, cc].tolist(),
                "Pdiag": P[dp, dp].tolist(), "Cdiag": C[dc, dc].tolist(),
                "W_absmax": float(np.abs(W).max()),
            }
    doc = {
        "what": "oracle trajectory from oracle-normalised FP32-rounded priors",
        "workload": w.__dict__, "readings": opts.__dict__,
        "inputs_sha256_f32": digest(Wf, Pf, Cf),
        "iters": t, "converged": bool(conv), "h_trace": hs,
        "idx": {"W": [rw.tolist(), cw.tolist()], "P": [rp.tolist(), cp.tolist()],
                "C": [rc.tolist(), cc.tolist()], "Pdiag": dp.tolist(), "Cdiag": dc.tolist()},
        "snapshots": snaps,
        "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(HERE, f"oracle_{w.name}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(doc, f)
    os.replace(path + ".tmp", path)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "small")
