"""The learned warm start on the GPU against its FP64 oracle
(oracle/warmstart.py): features, MLP forward and gradient (bf16 matrix-core
products emulated by the oracle at the same rounding points), Adam, the
warm state and the polish iterations from it, and a small training run that
must beat the trivial predictor on held-out networks.

Tolerances.  Features are z-scored O(1) values computed in FP64 from FP32
inputs except the one-step similarity (FP32 products): max-abs 1e-4.  MLP
output: one bf16 ulp (2^-8 relative) of any hidden activation may round
the other way when the GPU's FP32 pre-activation and the oracle's FP64 one
straddle a rounding boundary, so the bound per edge is
2^-7 sum_n |w3_n| sum_k |W2_nk| |h1_k| plus FP32 accumulation (1e-5 of the
magnitudes).  Gradients: relative L2 error 1e-2 per parameter block (the same
ulp flips, summed over the batch).  Adam: relative 1e-5 (FP32 arithmetic).
"""
import numpy as np
import pytest

from oracle import warmstart as WS
from paper_1507_07039_amd import inputs as I
from test_gpu_parity import compare_state, cuda, f32r, host, prep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def pd(torch):
    from paper_1507_07039_amd import panda
    panda.load_library()
    return panda


def loaded_ctx(torch, pd, W, P, C):
    ctx = pd.Context(*W.shape)
    ctx.load(cuda(torch, W), cuda(torch, P), cuda(torch, C))
    return ctx


@pytest.mark.parametrize("case", ["small", "ragged", "tiny"])
def test_features_match_oracle(torch, pd, oracle, case):
    if case == "small":
        W, P, C = prep(oracle, *I.workload_priors(I.SMALL))
    else:
        Ne, Na = (65, 300) if case == "ragged" else (3, 11)
        rng = np.random.default_rng(Ne + Na)
        W = f32r(rng.normal(size=(Ne, Na)))
        P = f32r(I.random_symmetric(Ne + 9, Ne))
        C = f32r(I.random_symmetric(Na + 9, Na))
    Ne, Na = W.shape
    Op, Oc = I.sketch_matrices(Ne * 7 + Na, Ne, Na)
    ctx = loaded_ctx(torch, pd, W, P, C)
    F, tau = ctx.features(cuda(torch, Op), cuda(torch, Oc))
    want = WS.features(W, P, C, Op.astype(np.float64), Oc.astype(np.float64))
    err = np.abs(host(F) - want)
    assert err.max() <= 1e-4, (case, err.max(axis=0))
    S = WS.one_step(W, P, C)
    assert abs(tau - WS.target_scale(W, S)) <= 1e-5 * WS.target_scale(W, S)
    # the state is untouched: the next iteration still matches the oracle
    Wo, Po, Co, _, _ = oracle.step(W, P, C, 1, oracle.Options(tol=0.0))
    ctx.iterate()
    Wg, Pg, Cg, _, _ = ctx.state()
    compare_state(host(Wg), host(Pg), host(Cg), Wo, Po, Co, what=case)


def fwd_bound(p, X):
    W1, b1, W2, b2, w3, b3 = WS.unpack(p)
    _, (Xq, z1, h1q, z2, h2, W1q, W2q, w3q) = WS.forward(p, X, bf16_mode=True)
    flip = 2.0 ** -7 * (np.abs(h1q) @ np.abs(W2q).T) @ np.abs(w3q)
    acc = 1e-5 * (np.abs(h2) @ np.abs(w3q) + np.abs(b3) + (np.abs(Xq) @ np.abs(W1q).T).sum(1))
    return flip + acc + 1e-6


@pytest.mark.parametrize("n", [1, 37, 4096])
def test_mlp_forward_matches_oracle(torch, pd, n):
    rng = np.random.default_rng(n)
    p = f32r(WS.init_params(3) + rng.normal(scale=0.05, size=WS.NPARAM))
    X = f32r(rng.normal(size=(n, 16)))
    y = host(pd.mlp_forward(cuda(torch, p), cuda(torch, X)))
    want, _ = WS.forward(p, X, bf16_mode=True)
    err = np.abs(y - want)
    assert np.all(err <= fwd_bound(p, X)), (err.max(), (err / fwd_bound(p, X)).max())


def blocks(g):
    W1, b1, W2, b2, w3, b3 = WS.unpack(g)
    return {"W1": W1, "b1": b1, "W2": W2, "b2": b2, "w3": w3, "b3": np.array([b3])}


@pytest.mark.parametrize("n,use_idx", [(1000, False), (777, True), (20000, True)])
def test_mlp_gradient_matches_oracle(torch, pd, n, use_idx):
    rng = np.random.default_rng(n + use_idx)
    p = f32r(WS.init_params(4) + rng.normal(scale=0.05, size=WS.NPARAM))
    rows = n + 100 if use_idx else n
    X = f32r(rng.normal(size=(rows, 16)))
    t = f32r(rng.normal(size=rows))
    idx = rng.permutation(rows)[:n] if use_idx else np.arange(n)
    g, loss = pd.mlp_grad(cuda(torch, p), cuda(torch, X), cuda(torch, t),
                          torch.from_numpy(idx.astype(np.int64)).cuda() if use_idx else None, n)
    lw, gw = WS.loss_grad(p, X[idx], t[idx], bf16_mode=True)
    assert abs(loss.item() - lw) <= 1e-4 * lw
    got, want = blocks(host(g)), blocks(gw)
    for k in want:
        rel = np.linalg.norm(got[k] - want[k]) / max(np.linalg.norm(want[k]), 1e-30)
        assert rel <= 1e-2, (k, rel)
    # and against the exact FP64 network (bf16 effects only): looser
    _, ge = WS.loss_grad(p, X[idx], t[idx])
    assert np.linalg.norm(host(g) - ge) <= 0.05 * np.linalg.norm(ge)


def test_adam_matches_oracle(torch, pd):
    rng = np.random.default_rng(8)
    p = f32r(rng.normal(size=WS.NPARAM))
    m = np.zeros(WS.NPARAM)
    v = np.zeros(WS.NPARAM)
    pg, mg, vg = (cuda(torch, a) for a in (p, m, v))
    for step in range(1, 4):
        g = f32r(rng.normal(size=WS.NPARAM))
        pd.mlp_adam(pg, mg, vg, cuda(torch, g), step, lr=1e-2)
        p, m, v = WS.adam(p, m, v, g, step, lr=1e-2)
        assert np.abs(host(pg) - p).max() <= 1e-5 * 1e-2 * step + 1e-6 * np.abs(p).max()


def test_warm_state_and_polish_match_oracle(torch, pd, oracle):
    W0, P0, C0 = prep(oracle, *I.workload_priors(I.SMALL))
    ref = oracle.run(W0, P0, C0)
    Wp = f32r(ref.W + np.random.default_rng(2).normal(scale=0.05, size=ref.W.shape))
    t0 = 20
    ctx = loaded_ctx(torch, pd, W0, P0, C0)
    ctx.ws_init(cuda(torch, Wp), t0)
    Wg, Pg, Cg, _, tg = ctx.state()
    assert tg == t0
    Wo, Po, Co = WS.warm_state(Wp, P0, C0, t0)
    compare_state(host(Wg), host(Pg), host(Cg), Wo, Po, Co, what="warm state")
    for t in range(t0 + 1, t0 + 4):
        Wo, Po, Co, ho, _ = oracle.step(Wo, Po, Co, t, oracle.Options(tol=0.0))
        h, tt = ctx.iterate()
        assert tt == t
        Wg, Pg, Cg, _, _ = ctx.state()
        compare_state(host(Wg), host(Pg), host(Cg), Wo, Po, Co, what=f"polish t={t}")


def test_training_beats_the_trivial_predictor(torch, pd, oracle):
    """Train on plain runs of 12 small networks (batched form), evaluate on 2
    held-out ones: the predicted converged W is closer to the plain result
    than the prior is."""
    from paper_1507_07039_amd import warmstart as WSG
    nets = [I.priors(100 + s, 40, 400, 0.05, 0.03, 30, 8) for s in range(14)]
    data = WSG.training_set(nets[:12], sketch_seed=5)
    params, hist = WSG.train(data, steps=300, batch=4096, lr=3e-3, seed=1)
    assert hist[-1] < 0.5 * hist[0], hist[::50]
    for raw in nets[12:]:
        W, P, C = WSG.normalized(*raw)
        Wp = WSG.predict(params, W, P, C, sketch_seed=5)
        plain = pd.run(W, P, C)
        e_pred = (Wp - plain.W).norm().item()
        e_prior = (W - plain.W).norm().item()
        print(f"held-out: |Wpred - W*| = {e_pred:.3f}, |W0 - W*| = {e_prior:.3f}")
        assert e_pred < e_prior
