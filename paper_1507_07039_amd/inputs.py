"""Seeded synthetic priors shaped like the paper's workloads.

This module holds no arithmetic of the message-passing method: it only draws
the raw seed networks that the method starts from (Sec. II-A: a motif prior W,
a TF-TF interaction prior P and a gene co-expression prior C built as the
Pearson correlation of an expression matrix).  Normalisation and everything
after it belong to the library and, independently, to the oracle.  Both sides
receive the same arrays from here.

Draw order for ``priors(seed, T, G, pW, pP, S, K)`` (numpy PCG64):
  1. W0 = [U(0,1)^{T x G} < pW]                     binary motif prior
  2. U  = [U(0,1)^{T x T} < pP], strict upper part; P0 = U + U^T + I
  3. L ~ N(0, 0.5^2)^{G x K}; F ~ N(0, 1)^{K x S}; E = L F + N(0, 1)^{G x S}
  4. C0 = Pearson correlation between the rows (genes) of E
A gene whose expression row is constant gets correlation 0 with every other
gene and 1 with itself.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    T: int      # transcription factors (effector nodes, N_e)
    G: int      # genes (affected nodes, N_a)
    pW: float   # motif-prior density
    pP: float   # TF-TF interaction density
    S: int      # expression samples
    K: int      # latent expression factors


# Small case the oracle finishes in seconds, and the realistic-size case
# (TFs a few percent of ~20k genes, Sec. II-F) that the benchmark times.
SMALL = Workload("panda-T40-G400", 1507, 40, 400, 0.05, 0.03, 30, 8)
HUMAN = Workload("panda-T700-G18000", 7039, 700, 18000, 0.03, 0.01, 200, 20)
LARGE = Workload("panda-T1000-G30000", 30000, 1000, 30000, 0.03, 0.01, 300, 25)


def pearson_rows(E: np.ndarray) -> np.ndarray:
    """Pearson correlation between the rows of E (genes x samples), FP64."""
    E = np.asarray(E, dtype=np.float64)
    Z = E - E.mean(axis=1, keepdims=True)
    nrm = np.sqrt(np.einsum("ij,ij->i", Z, Z))
    const = nrm == 0.0
    nrm[const] = 1.0
    Z = Z / nrm[:, None]
    C = Z @ Z.T
    C[const, :] = 0.0
    C[:, const] = 0.0
    np.fill_diagonal(C, 1.0)
    C = 0.5 * (C + C.T)  # exact symmetry regardless of the product's summation order
    return C


def _draw(seed: int, T: int, G: int, pW: float, pP: float, S: int, K: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    W0 = (rng.random((T, G)) < pW).astype(np.float64)
    U = np.triu((rng.random((T, T)) < pP).astype(np.float64), k=1)
    P0 = U + U.T + np.eye(T)
    L = rng.normal(0.0, 0.5, size=(G, K))
    F = rng.normal(0.0, 1.0, size=(K, S))
    E = L @ F + rng.normal(0.0, 1.0, size=(G, S))
    return W0, P0, E


def priors(seed: int, T: int, G: int, pW: float, pP: float, S: int, K: int):
    """Raw (un-normalised) FP64 priors (W0, P0, C0) in the documented order."""
    W0, P0, E = _draw(seed, T, G, pW, pP, S, K)
    return W0, P0, pearson_rows(E)


def workload_priors(w: Workload):
    return priors(w.seed, w.T, w.G, w.pW, w.pP, w.S, w.K)


def expression(seed: int, T: int, G: int, pW: float, pP: float, S: int, K: int) -> np.ndarray:
    """The expression matrix E (G x S, FP64) that C0 of priors(...) is built
    from (step 3 of the draw order)."""
    return _draw(seed, T, G, pW, pP, S, K)[2]


def workload_expression(w: Workload) -> np.ndarray:
    return expression(w.seed, w.T, w.G, w.pW, w.pP, w.S, w.K)


def random_dense(seed: int, shape, low: float = -1.0, high: float = 1.0) -> np.ndarray:
    """Uniform random FP64 matrix (kernel-level parity inputs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(low, high, size=shape)


def random_symmetric(seed: int, n: int) -> np.ndarray:
    """Symmetric FP64 matrix with N(0,1) entries."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.normal(0.0, 1.0, size=(n, n))
    return np.triu(A) + np.triu(A, 1).T


def table1_priors(seed: int, n: int):
    """Table I workload: a random square W with P = C = identity.

    The paper does not say how its random W were drawn; U(0,1) entries are
    used here.  Returns raw (W0, P0, C0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W0 = rng.random((n, n))
    return W0, np.eye(n), np.eye(n)


def batched_shapes(master_seed: int = 48, n: int = 48, t_range=(50, 700), g_range=(1000, 18000)):
    """Shapes (T, G) and instance seeds for a set of independent networks."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    Ts = rng.integers(t_range[0], t_range[1] + 1, size=n)
    Gs = rng.integers(g_range[0], g_range[1] + 1, size=n)
    return [(int(Ts[i]), int(Gs[i]), 4800 + i) for i in range(n)]


def to_f32(*arrs):
    """Round FP64 arrays to FP32 (round-to-nearest-even), C-contiguous."""
    return tuple(np.ascontiguousarray(a, dtype=np.float32) for a in arrs)


def sketch_matrices(seed: int, Ne: int, Na: int, k: int = 6):
    """Gaussian sketch matrices (Ne x k, Na x k, FP32) of the warm-start features."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (np.ascontiguousarray(rng.standard_normal((Ne, k)), dtype=np.float32),
            np.ascontiguousarray(rng.standard_normal((Na, k)), dtype=np.float32))
