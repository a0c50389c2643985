"""FP64 oracle of the learned warm start (not in the paper).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product library never does.

The warm start predicts the converged W of a PANDA run (Sec. II-B) from
per-edge features of the normalised priors with a small MLP, then rebuilds a
state (W, P, C, t0) from which the message passing (Eq. 2-7) is polished to
h < tol.  Everything here is plain numpy FP64 written from these definitions:

Features of edge (i, j), 16 per edge (P0, C0, W0 already z-scored):
  g0  = W0_ij
  g1  = sum_j' W0_ij'                 (TF out-degree)
  g2  = sum_i' W0_i'j                 (gene in-degree)
  g3..g8   = a_k[i] * b_k[j], k < 6: a_k = column k of the orthonormal basis
             of P0 (P0 Omega_P) by Cholesky QR, b_k = W0^T (P0 a_k)
             (rank-1 pieces of the projection of P0 W0 onto a sketch of
             P0's dominant subspace; randomised range finder with one power
             step, Omega_P a given Gaussian N_e x 6 matrix)
  g9..g14  = c_k[i] * d_k[j]: d_k = basis column of C0 (C0 Omega_C),
             c_k = W0 (C0 d_k) (the same for W0 C0)
  g15 = (R0_ij + A0_ij) / 2 with R0 = T(P0, W0), A0 = T(W0, C0) (Eq. 1-4)
Each feature is z-scored over the N_e N_a edges (population std; a constant
feature becomes 0).

MLP 16 -> 64 -> 64 -> 1 with ReLU; parameters packed as
  W1[64][16], b1[64], W2[64][64] (out, in), b2[64], w3[64], b3.
Its output is the converged change of W in units of the one-step change:
  W* - W0 = y * tau,  tau = std over edges of (S - W0), S = (R0 + A0) / 2.
Loss: mean squared error of y against (W* - W0) / tau over a batch.

The GPU computes the products with bf16 weights and bf16 activations on
matrix cores (FP32 accumulation); forward(..., bf16=True) rounds the same
values at the same points (round to nearest even) so the two can be compared
tightly; bf16=False is the exact FP64 network used for gradient checks.

Warm state: W = W_pred; off-diagonals P_im = T(W_i., W_m.), C_kj = T(W_.k,
W_.j) (the fixed point of Eq. 5 for this W); diagonals from the closed form of
the Eq. 6 recursion over t0 iterations with sigma held at the std of the
rebuilt off-diagonal row:
  d(t0) = (1 - a)^t0 d(0) + f N sigma sum_{tau=1..t0} (1 - a)^(t0 - tau) e^(2 a tau)
(f = a under the default reading, N = N_a for P and N_e for C).
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

NFEAT = 16
NH = 64
NSKETCH = 6
NPARAM = NH * NFEAT + NH + NH * NH + NH + NH + 1  # 5313

# offsets of the packed parameter vector
_OFF = {}
_o = 0
for _name, _n in (("W1", NH * NFEAT), ("b1", NH), ("W2", NH * NH), ("b2", NH), ("w3", NH),
                  ("b3", 1)):
    _OFF[_name] = (_o, _o + _n)
    _o += _n
assert _o == NPARAM


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    g = {k: p[a:b] for k, (a, b) in _OFF.items()}
    return (g["W1"].reshape(NH, NFEAT), g["b1"], g["W2"].reshape(NH, NH), g["b2"], g["w3"],
            g["b3"][0])


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def init_params(seed: int = 0):
    """He-uniform initial weights (FP32-representable), zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (NH, NFEAT)) * np.sqrt(6.0 / NFEAT)
    W2 = rng.uniform(-1, 1, (NH, NH)) * np.sqrt(6.0 / NH)
    w3 = rng.uniform(-1, 1, NH) * np.sqrt(3.0 / NH)
    p = pack(W1, np.zeros(NH), W2, np.zeros(NH), w3, 0.0)
    return p.astype(np.float32).astype(np.float64)


# ----------------------------------------------------------------- bf16 ---

def bf16(x):
    """Round to bfloat16 (nearest even) through FP32, returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ------------------------------------------------------------- features ---

PIVOT_REL = 1e-10  # Cholesky pivots below this fraction of max diag(Y^T Y) end the basis


def sketch_basis(M, Omega):
    """Orthonormal basis of Y = M (M Omega) by Cholesky QR: Q = Y L^-T with
    L L^T = Y^T Y.  The factorisation stops at the first pivot L_kk^2 <=
    PIVOT_REL * max diag(Y^T Y) (Y of rank k, e.g. fewer rows than columns);
    columns k.. of Q are then zero."""
    Y = M @ (M @ Omega)
    G = Y.T @ Y
    n = G.shape[0]
    L = np.zeros_like(G)
    thr = PIVOT_REL * max(float(np.max(np.diag(G))), 0.0)
    k = n
    for j in range(n):
        piv = G[j, j] - L[j, :j] @ L[j, :j]
        if not piv > thr:
            k = j
            break
        L[j, j] = np.sqrt(piv)
        for i in range(j + 1, n):
            L[i, j] = (G[i, j] - L[i, :j] @ L[j, :j]) / L[j, j]
    Q = np.zeros_like(Y)
    if k:
        Q[:, :k] = np.linalg.solve(L[:k, :k], Y[:, :k].T).T
    return Q


def raw_vectors(W0, P0, C0, OmegaP, OmegaC):
    """The per-row / per-column vectors behind features g1..g14."""
    W0, P0, C0 = (np.asarray(M, dtype=np.float64) for M in (W0, P0, C0))
    a = sketch_basis(P0, np.asarray(OmegaP, dtype=np.float64))   # Ne x 6
    b = W0.T @ (P0 @ a)                                             # Na x 6
    d = sketch_basis(C0, np.asarray(OmegaC, dtype=np.float64))   # Na x 6
    c = W0 @ (C0 @ d)                                               # Ne x 6
    return W0.sum(axis=1), W0.sum(axis=0), a, b, c, d


def one_step(W0, P0, C0):
    """S = (T(P0, W0) + T(W0, C0)) / 2 (Eq. 3, 4 at t = 1)."""
    return 0.5 * (O.tanimoto(P0, W0) + O.tanimoto(W0, C0))


def _z(col):
    m = col.mean()
    s = np.sqrt(((col - m) ** 2).mean())
    return (col - m) / s if s > 0 else np.zeros_like(col)


def features(W0, P0, C0, OmegaP, OmegaC):
    """Ne*Na x 16 feature matrix (row i*Na + j = edge (i, j)), z-scored columns."""
    W0 = np.asarray(W0, dtype=np.float64)
    Ne, Na = W0.shape
    dr, dc, a, b, c, d = raw_vectors(W0, P0, C0, OmegaP, OmegaC)
    S = one_step(W0, P0, C0)
    G = np.empty((Ne, Na, NFEAT))
    G[:, :, 0] = W0
    G[:, :, 1] = dr[:, None]
    G[:, :, 2] = dc[None, :]
    for k in range(NSKETCH):
        G[:, :, 3 + k] = np.outer(a[:, k], b[:, k])
        G[:, :, 9 + k] = np.outer(c[:, k], d[:, k])
    G[:, :, 15] = S
    G = G.reshape(Ne * Na, NFEAT)
    return np.stack([_z(G[:, f]) for f in range(NFEAT)], axis=1)


def target_scale(W0, S):
    """tau = population std over edges of S - W0."""
    D = np.asarray(S, dtype=np.float64) - np.asarray(W0, dtype=np.float64)
    return float(np.sqrt(((D - D.mean()) ** 2).mean()))


# ------------------------------------------------------------------ MLP ---

def forward(p, X, bf16_mode=False):
    """y for every row of X; returns (y, cache)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    r = bf16 if bf16_mode else (lambda v: v)
    if bf16_mode:
        W1, W2, w3 = r(W1), r(W2), r(w3)
        X = r(X)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    h1q = r(h1)
    z2 = h1q @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (X, z1, h1q, z2, h2, W1, W2, w3)


def loss_grad(p, X, target, bf16_mode=False):
    """Mean squared error over the batch and its gradient (FP64).  In bf16
    mode dz2 and dz1 enter the matrix products (dW2, dh1, dW1) rounded to
    bf16, as on the GPU; the bias gradients and dw3 use them unrounded."""
    y, (Xq, z1, h1q, z2, h2, W1, W2, w3) = forward(p, X, bf16_mode)
    r = bf16 if bf16_mode else (lambda v: v)
    n = y.shape[0]
    e = y - np.asarray(target, dtype=np.float64)
    loss = float((e * e).mean())
    dy = 2.0 * e / n
    dw3 = h2.T @ dy
    db3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)
    dz2q = r(dz2)
    dW2 = dz2q.T @ h1q
    db2 = dz2.sum(axis=0)
    dh1 = dz2q @ W2
    dz1 = dh1 * (z1 > 0)
    dW1 = r(dz1).T @ Xq
    db1 = dz1.sum(axis=0)
    return loss, pack(dW1, db1, dW2, db2, dw3, db3)


def adam(p, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1), step counted from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------- warm state ---

def diag_schedule(d0, sigma, N, t0, alpha=0.1, diag_alpha=True):
    """Closed form of Eq. 6 after t0 steps with sigma held fixed."""
    f = alpha if diag_alpha else 1.0
    acc = sum((1 - alpha) ** (t0 - tau) * np.exp(2 * alpha * tau) for tau in range(1, t0 + 1))
    return (1 - alpha) ** t0 * np.asarray(d0, dtype=np.float64) + f * N * np.asarray(sigma) * acc


def warm_state(Wp, P0, C0, t0, alpha=0.1):
    """(W, P, C) from which the polish starts at iteration t0 (see above)."""
    Wp = np.asarray(Wp, dtype=np.float64)
    Ne, Na = Wp.shape
    P = O.tanimoto(Wp, np.ascontiguousarray(Wp.T))
    C = O.tanimoto(np.ascontiguousarray(Wp.T), Wp)

    def off_std(M):
        n = M.shape[0]
        if n < 2:
            return np.zeros(n)
        off = M[~np.eye(n, dtype=bool)].reshape(n, n - 1)
        return off.std(axis=1)

    sP, sC = off_std(P), off_std(C)
    dP = diag_schedule(np.diag(P0), sP, Na, t0, alpha)
    dC = diag_schedule(np.diag(C0), sC, Ne, t0, alpha)
    np.fill_diagonal(P, dP)
    np.fill_diagonal(C, dC)
    return Wp, P, C
