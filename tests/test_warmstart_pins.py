"""Pins of the warm-start oracle (oracle/warmstart.py) against mathematics
that does not depend on it: central finite differences, the projection
identity behind the sketch features, brute force on tiny inputs, the bf16
bit patterns, Adam's first steps in closed form and the Eq. 6 recursion."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import warmstart as WS


def tiny(seed, Ne=5, Na=9):
    rng = np.random.default_rng(seed)
    W = rng.normal(size=(Ne, Na))
    A = rng.normal(size=(Ne, Ne))
    B = rng.normal(size=(Na, Na))
    return W, A + A.T, B + B.T, rng.normal(size=(Ne, 6)), rng.normal(size=(Na, 6))


def test_param_layout():
    assert WS.NPARAM == 5313
    p = np.arange(WS.NPARAM, dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = WS.unpack(p)
    assert W1.shape == (64, 16) and W2.shape == (64, 64) and w3.shape == (64,)
    assert W1[1, 0] == 16 and b1[0] == 1024 and W2[0, 1] == 1024 + 64 + 1 and b3 == 5312
    assert np.array_equal(WS.pack(W1, b1, W2, b2, w3, b3), p)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = WS.init_params(1) + rng.normal(scale=0.05, size=WS.NPARAM)
    X = rng.normal(size=(37, 16))
    tgt = rng.normal(size=37)
    loss, g = WS.loss_grad(p, X, tgt)
    idx = rng.choice(WS.NPARAM, size=300, replace=False)
    idx = np.concatenate([idx, [WS.NPARAM - 1, 0, 1024, 1024 + 64, 5312 - 64]])
    h = 1e-6
    for k in idx:
        e = np.zeros(WS.NPARAM)
        e[k] = h
        fd = (WS.loss_grad(p + e, X, tgt)[0] - WS.loss_grad(p - e, X, tgt)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * (1 + abs(g[k])), (k, fd, g[k])


def test_forward_closed_form_single_unit():
    # one active path: y = w3_0 * relu(W2_00 * relu(W1_00 x0 + b1_0) + b2_0) + b3
    W1 = np.zeros((64, 16)); W1[0, 0] = 2.0
    b1 = np.zeros(64); b1[0] = -1.0
    W2 = np.zeros((64, 64)); W2[0, 0] = 3.0
    b2 = np.zeros(64); b2[0] = 0.5
    w3 = np.zeros(64); w3[0] = -4.0
    p = WS.pack(W1, b1, W2, b2, w3, 0.25)
    X = np.zeros((3, 16)); X[:, 0] = [0.0, 1.0, 2.0]
    y, _ = WS.forward(p, X)
    want = [-4.0 * (3.0 * 0.0 + 0.5) + 0.25, -4.0 * (3.0 * 1.0 + 0.5) + 0.25,
            -4.0 * (3.0 * 3.0 + 0.5) + 0.25]
    assert np.allclose(y, want, rtol=0, atol=1e-12)


def test_bf16_rounding_bit_cases():
    cases = {1.0: 1.0, 1.0 + 2 ** -8: 1.0, 1.0 + 3 * 2 ** -8: 1.0 + 2 ** -6,
             1.0 + 2 ** -7: 1.0 + 2 ** -7, 1.0 + 2 ** -7 + 2 ** -8: 1.0 + 2 ** -6,
             -3.0: -3.0, 0.0: 0.0, 65280.0: 65280.0, 1.0 + 2 ** -8 + 2 ** -20: 1.0 + 2 ** -7}
    for x, want in cases.items():
        assert WS.bf16(np.array([x]))[0] == want, (x, WS.bf16(np.array([x]))[0], want)
    v = np.random.default_rng(0).normal(size=10000)
    r = WS.bf16(v)
    assert np.all(np.abs(r - v) <= 2 ** -8 * np.abs(v) * (1 + 1e-6))


def test_forward_bf16_mode_close_to_exact():
    rng = np.random.default_rng(4)
    p = WS.init_params(2)
    X = rng.normal(size=(200, 16))
    y, _ = WS.forward(p, X)
    yq, _ = WS.forward(p, X, bf16_mode=True)
    assert np.abs(yq - y).max() <= 3e-2 * (np.abs(y).max() + 1)
    assert not np.array_equal(yq, y)


def test_adam_closed_form_steps():
    rng = np.random.default_rng(5)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50); v = np.zeros(50)
    p1, m1, v1 = WS.adam(p, m, v, g, 1, lr=0.01, eps=0.0)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-15)
    # constant gradient: the bias-corrected moments stay g and g^2
    p2, _, _ = WS.adam(p1, m1, v1, g, 2, lr=0.01, eps=0.0)
    assert np.allclose(p2, p1 - 0.01 * np.sign(g), atol=1e-12)


def test_sketch_basis_is_orthonormal_and_spans_the_sketch():
    W, P, C, Op, Oc = tiny(6, 7, 11)
    for M, Om in ((P, Op), (C, Oc)):
        Q = WS.sketch_basis(M, Om)
        assert np.allclose(Q.T @ Q, np.eye(6), atol=1e-10)
        Y = M @ (M @ Om)
        assert np.allclose(Q @ (Q.T @ Y), Y, atol=1e-8 * np.abs(Y).max())
        # Cholesky QR: Q^T Y is upper-triangular with a positive diagonal
        R = Q.T @ Y
        assert np.allclose(np.tril(R, -1), 0, atol=1e-8 * np.abs(R).max())
        assert np.all(np.diag(R) > 0)


def test_rank_deficient_sketch_stops_the_basis():
    rng = np.random.default_rng(11)
    A = rng.normal(size=(4, 4))
    Q = WS.sketch_basis(A + A.T, rng.normal(size=(4, 6)))  # rank 4 < 6 columns
    assert np.allclose(Q[:, :4].T @ Q[:, :4], np.eye(4), atol=1e-8)
    assert np.all(Q[:, 4:] == 0)


def test_feature_definitions_brute_force():
    W, P, C, Op, Oc = tiny(7, 7, 11)
    Ne, Na = W.shape
    dr, dc, a, b, c, d = WS.raw_vectors(W, P, C, Op, Oc)
    # projection identity: sum_k a_k b_k^T = (a a^T) P W, sum_k c_k d_k^T = W C (d d^T)
    assert np.allclose(a @ b.T, a @ a.T @ P @ W, atol=1e-10)
    assert np.allclose(c @ d.T, W @ C @ d @ d.T, atol=1e-10)
    F = WS.features(W, P, C, Op, Oc)
    S = np.array([[0.5 * (O.T(P[i], W[:, j]) + O.T(W[i], C[:, j])) for j in range(Na)]
                  for i in range(Ne)])
    raw = np.empty((Ne * Na, 16))
    for i in range(Ne):
        for j in range(Na):
            e = i * Na + j
            raw[e, 0] = W[i, j]
            raw[e, 1] = sum(W[i, jj] for jj in range(Na))
            raw[e, 2] = sum(W[ii, j] for ii in range(Ne))
            for k in range(6):
                raw[e, 3 + k] = a[i, k] * b[j, k]
                raw[e, 9 + k] = c[i, k] * d[j, k]
            raw[e, 15] = S[i, j]
    for f in range(16):
        col = raw[:, f]
        z = (col - col.mean()) / col.std()
        assert np.allclose(F[:, f], z, atol=1e-9), f
    assert np.allclose(F.mean(axis=0), 0, atol=1e-12)
    assert np.allclose(F.std(axis=0), 1, atol=1e-12)


def test_constant_feature_becomes_zero():
    W, P, C, Op, Oc = tiny(8, 7, 9)
    W = np.ones_like(W)  # degrees constant
    F = WS.features(W, P, C, Op, Oc)
    assert np.all(F[:, 0] == 0) and np.all(F[:, 1] == 0) and np.all(F[:, 2] == 0)


def test_diag_schedule_is_eq6_iterated():
    rng = np.random.default_rng(9)
    d0 = rng.normal(size=4)
    sig = rng.uniform(0.5, 2, size=4)
    for alpha, da in ((0.1, True), (0.3, False)):
        d = d0.copy()
        f = alpha if da else 1.0
        for t in range(1, 13):
            d = (1 - alpha) * d + f * 50 * sig * np.exp(2 * alpha * t)
            assert np.allclose(WS.diag_schedule(d0, sig, 50, t, alpha, da), d, rtol=1e-12)
    assert np.array_equal(WS.diag_schedule(d0, sig, 50, 0), d0)


def test_warm_state_structure():
    W, P0, C0, _, _ = tiny(10, 7, 9)
    Wp, P, C = WS.warm_state(W, P0, C0, 12)
    Ne, Na = W.shape
    assert np.array_equal(P, P.T) and np.array_equal(C, C.T)
    for i in range(Ne):
        for m in range(Ne):
            if i != m:
                assert abs(P[i, m] - O.T(W[i], W[m])) <= 1e-14 * (1 + abs(P[i, m]))
    for k in range(Na):
        for j in range(Na):
            if k != j:
                assert abs(C[k, j] - O.T(W[:, k], W[:, j])) <= 1e-14 * (1 + abs(C[k, j]))
    sP = np.array([np.delete(P[i], i).std() for i in range(Ne)])
    assert np.allclose(np.diag(P), WS.diag_schedule(np.diag(P0), sP, Na, 12), rtol=1e-13)


def test_target_scale_is_the_population_std():
    # S - W0 = (0, 0, 0, 4): mean 1, population variance 3 (the sample
    # variance would be 4), so tau = sqrt(3)
    W0 = np.array([[1.0, -2.0], [0.5, 3.0]])
    S = W0 + np.array([[0.0, 0.0], [0.0, 4.0]])
    assert WS.target_scale(W0, S) == pytest.approx(np.sqrt(3.0), rel=1e-15)
    # one entry differs from all others equally: D = (5, 0, 0, 0, 0, 0, 0, 0),
    # population std = 5 sqrt(7) / 8
    D = np.zeros((2, 4)); D[0, 0] = 5.0
    assert WS.target_scale(np.zeros((2, 4)), D) == pytest.approx(5 * np.sqrt(7) / 8, rel=1e-15)


def _rounding_net():
    """A network whose output depends on every bf16 rounding point of the
    GPU's forward pass; all values are exact binary fractions.
      X  = (1, 2^-9, 1 + 2^-8 + 2^-9, 1): X_2 rounds up to 1 + 2^-7
      z1_0 = X_0 + X_1 = 1 + 2^-9                -> h1 rounds it to 1
      z1_1 = X_2 - X_3 = 2^-7 (X rounded), 3 2^-9 if X were not rounded
      z1_2 = W1_20 X_0 - X_3, W1_20 = 1 + 2^-8 + 2^-9 rounds to 1 + 2^-7:
             2^-7 (W1 rounded), 3 2^-9 if not
      z2_0 = W2_00 h1_0 + 2^-3 h1_1 + 2^-5 h1_2, W2_00 = 1 + 2^-9 rounds to 1
      z2_1 = 2^-9 h1_0
      y    = w3_0 h2_0 + h2_1 + 1/4, w3_0 = 1 + 2^-9 rounds to 1."""
    W1 = np.zeros((64, 16)); b1 = np.zeros(64)
    W2 = np.zeros((64, 64)); b2 = np.zeros(64)
    w3 = np.zeros(64)
    W1[0, 0] = 1.0; W1[0, 1] = 1.0
    W1[1, 2] = 1.0; W1[1, 3] = -1.0
    W1[2, 0] = 1 + 2.0 ** -8 + 2.0 ** -9; W1[2, 3] = -1.0
    W2[0, 0] = 1 + 2.0 ** -9; W2[0, 1] = 2.0 ** -3; W2[0, 2] = 2.0 ** -5
    W2[1, 0] = 2.0 ** -9
    w3[0] = 1 + 2.0 ** -9; w3[1] = 1.0
    p = WS.pack(W1, b1, W2, b2, w3, 0.25)
    X = np.zeros((1, 16)); X[0, :4] = [1.0, 2.0 ** -9, 1 + 2.0 ** -8 + 2.0 ** -9, 1.0]
    return p, X


def test_forward_bf16_rounding_points_bit_exact():
    """Inputs, weights and the first hidden layer are rounded to bf16; the
    second layer's pre-activations and the output are not.  Leaving out any
    rounding, or adding one after the second layer, changes y."""
    p, X = _rounding_net()
    y, (Xq, z1, h1q, z2, h2, W1q, W2q, w3q) = WS.forward(p, X, bf16_mode=True)
    assert h1q[0, :3].tolist() == [1.0, 2.0 ** -7, 2.0 ** -7]
    assert z2[0, :2].tolist() == [1 + 2.0 ** -10 + 2.0 ** -12, 2.0 ** -9]
    assert y[0] == 1.25 + 2.0 ** -9 + 2.0 ** -10 + 2.0 ** -12
    # the exact network differs at every one of those points
    ye, (_, z1e, _, _, _, _, _, _) = WS.forward(p, X)
    assert z1e[0, :3].tolist() == [1 + 2.0 ** -9, 3 * 2.0 ** -9, 3 * 2.0 ** -9]
    z2e0 = (1 + 2.0 ** -9) ** 2 + 3 * 2.0 ** -9 * 2.0 ** -3 + 3 * 2.0 ** -9 * 2.0 ** -5
    assert ye[0] == z2e0 * (1 + 2.0 ** -9) + (1 + 2.0 ** -9) * 2.0 ** -9 + 0.25


def test_gradient_bf16_rounding_points_bit_exact():
    """In the backward pass dz2 and dz1 enter the weight and input-gradient
    products rounded to bf16 (with the rounded h1, X and W2 of the forward
    pass), while the bias gradients and dw3 take them unrounded.  The target
    makes dy = 1 + 2^-9, so dz2_0 = dz2_1 = 1 + 2^-9 (rounds to 1) and
    dh1_0 = dz2q_0 W2q_00 + dz2q_1 W2q_10 = 1 + 2^-9 (rounds to 1)."""
    p, X = _rounding_net()
    y = 1.25 + 2.0 ** -9 + 2.0 ** -10 + 2.0 ** -12
    target = np.array([y - (0.5 + 2.0 ** -10)])  # e = (1 + 2^-9) / 2, n = 1
    loss, g = WS.loss_grad(p, X, target, bf16_mode=True)
    assert loss == (0.5 + 2.0 ** -10) ** 2
    dW1, db1, dW2, db2, dw3, db3 = WS.unpack(g)
    dy = 1 + 2.0 ** -9
    assert db3 == dy
    assert dw3[:2].tolist() == [(1 + 2.0 ** -10 + 2.0 ** -12) * dy, 2.0 ** -9 * dy]
    assert db2[:2].tolist() == [dy, dy]                                  # unrounded dz2
    assert dW2[0, :3].tolist() == [1.0, 2.0 ** -7, 2.0 ** -7]          # bf16(dz2) h1q
    assert dW2[1, :3].tolist() == [1.0, 2.0 ** -7, 2.0 ** -7]
    # dh1 = bf16(dz2) W2q: unit 0 gets 1 + 2^-9, units 1 and 2 get 2^-3, 2^-5
    assert db1[:3].tolist() == [1 + 2.0 ** -9, 2.0 ** -3, 2.0 ** -5]   # unrounded dz1
    assert dW1[0, :4].tolist() == [1.0, 2.0 ** -9, 1 + 2.0 ** -7, 1.0]  # bf16(dz1) Xq
    assert dW1[1, :4].tolist() == [2.0 ** -3, 2.0 ** -12, 2.0 ** -3 * (1 + 2.0 ** -7), 2.0 ** -3]
    assert np.count_nonzero(dW1[3:]) == 0 and np.count_nonzero(dW2[2:]) == 0
