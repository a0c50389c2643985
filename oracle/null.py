"""FP64 oracle of the permutation null (node-label randomisation on input, an
option of the paper's C implementation, Sec. III).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product library never does.

Instance k relabels the genes of C0 with permutation sigma_k (C_k[i][j] =
C0[sigma_k(i)][sigma_k(j)]) and the TFs of P0 with tau_k, keeps W0, and runs the
message passing (the C oracle's run) to convergence; the null of edge (i, j)
is the mean and the population standard deviation of W_k[i][j] over the K
instances, taken here with numpy over the stacked results.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def permute_sym(M, perm) -> np.ndarray:
    """The network with its nodes relabelled: out[i][j] = M[perm[i]][perm[j]]."""
    M = np.asarray(M, dtype=np.float64)
    perm = np.asarray(perm, dtype=np.int64)
    if M.ndim != 2 or M.shape[0] != M.shape[1] or perm.shape != (M.shape[0],):
        raise ValueError("square matrix and one permutation of its size")
    if not np.array_equal(np.sort(perm), np.arange(M.shape[0])):
        raise ValueError("not a permutation")
    return M[np.ix_(perm, perm)]


def null_runs(W0, P0, C0, gene_perms=None, tf_perms=None, opts: O.Options | None = None):
    """The K relabelled runs (oracle RunResult each).  P0 and C0 are arrays
    (a normalised identity where no prior exists)."""
    perms = [p for p in (gene_perms, tf_perms) if p is not None]
    K = len(perms[0]) if perms else 1
    out = []
    for k in range(K):
        Pk = P0 if tf_perms is None else permute_sym(P0, tf_perms[k])
        Ck = C0 if gene_perms is None else permute_sym(C0, gene_perms[k])
        out.append(O.run(W0, Pk, Ck, opts))
    return out


def null_stats(W0, P0, C0, gene_perms=None, tf_perms=None, opts: O.Options | None = None):
    """(mean, sd, iterations, statuses) of the null over the K instances."""
    runs = null_runs(W0, P0, C0, gene_perms, tf_perms, opts)
    Ws = np.stack([r.W for r in runs])
    return (Ws.mean(axis=0), Ws.std(axis=0), [r.iters for r in runs],
            [r.status for r in runs])


def zscore(W, mean, sd) -> np.ndarray:
    """(W - mean) / sd per edge, 0 where the null has no spread."""
    W, mean, sd = (np.asarray(a, dtype=np.float64) for a in (W, mean, sd))
    z = np.zeros_like(W)
    ok = sd > 0
    z[ok] = (W[ok] - mean[ok]) / sd[ok]
    return z
