"""Learned warm start (not in the paper): orchestration of the library's
warm-start kernels.

Every computation runs in libpanda.so (features, MLP forward / gradient /
Adam, targets, predictions, warm state, message passing); this module draws
the random inputs (sketch matrices, initial weights, minibatch indices),
moves tensors between calls and keeps the training loop.

  training_set   plain runs of many networks in one batch (grouped launches),
                 then the features of each network's priors and its target
                 (W* - W0) / tau
  train          Adam on random minibatches of edges
  predict        W_pred = W0 + tau * MLP(features)
  warm_run       W_pred -> warm state at t0 -> message passing to h < tol
  judged_run     warm_run checked against the plain run from the priors (the
                 reference and the fallback)
  amplification  how much a small change of W at iteration t0 of the plain
                 run grows by the end of the run (what a warm state at t0
                 would have to be accurate to)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import inputs as I
from . import panda

MLP_PARAMS = panda.MLP_PARAMS


def _torch():
    import torch
    return torch


def normalized(W0, P0, C0):
    """Device copies of raw priors, z-scored by the library."""
    torch = _torch()
    dev = [torch.from_numpy(np.ascontiguousarray(M, dtype=np.float32)).cuda() for M in (W0, P0, C0)]
    for M in dev:
        panda.normalize(M)
    return dev


def features(W, P, C, sketch_seed: int, opts=None):
    """(F, tau) of normalised device priors."""
    torch = _torch()
    Ne, Na = W.shape
    Op, Oc = I.sketch_matrices(sketch_seed, Ne, Na)
    ctx = panda.Context(Ne, Na, opts)
    ctx.load(W, P, C)
    F, tau = ctx.features(torch.from_numpy(Op).cuda(), torch.from_numpy(Oc).cuda())
    ctx.close()
    return F, tau


def training_set(nets, sketch_seed: int = 0, opts=None):
    """Features and targets of raw priors [(W0, P0, C0), ...] from their plain
    runs (all networks in one batch, graph replays)."""
    torch = _torch()
    dev = [normalized(*n) for n in nets]
    batch = panda.Batch([d[0].shape for d in dev], opts)
    for i, d in enumerate(dev):
        batch.load(i, *d)
    batch.run(graph=True)
    Fs, Ys, stops, taus = [], [], [], []
    for i, (W, P, C) in enumerate(dev):
        F, tau = features(W, P, C, sketch_seed)
        Wstar, _, _, _, t = batch.state(i)
        Fs.append(F)
        Ys.append(panda.ws_target(W, Wstar, tau).reshape(-1))
        stops.append(t)
        taus.append(tau)
    batch.close()
    return {"F": torch.cat(Fs), "Y": torch.cat(Ys), "stops": stops, "taus": taus}


def init_params(seed: int = 0):
    """He-uniform weights, zero biases (FP32, device)."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    nh, nf = 64, panda.WS_FEATURES
    parts = [rng.uniform(-1, 1, nh * nf) * np.sqrt(6.0 / nf), np.zeros(nh),
             rng.uniform(-1, 1, nh * nh) * np.sqrt(6.0 / nh), np.zeros(nh),
             rng.uniform(-1, 1, nh) * np.sqrt(3.0 / nh), np.zeros(1)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == MLP_PARAMS
    return torch.from_numpy(p).cuda()


def train(data, steps: int = 2000, batch: int = 65536, lr: float = 1e-3, seed: int = 0,
          params=None, log_every: int = 10):
    """Adam on minibatches of edges drawn uniformly; returns (params, losses)."""
    torch = _torch()
    F, Y = data["F"], data["Y"]
    n = F.shape[0]
    p = init_params(seed) if params is None else params.clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    ws = panda.workspace(panda.load_library().panda_mlp_grad_workspace_bytes(batch))
    rng = np.random.default_rng(seed + 1)
    losses = []
    for step in range(1, steps + 1):
        idx = torch.from_numpy(rng.integers(0, n, size=batch, dtype=np.int64)).cuda()
        g, loss = panda.mlp_grad(p, F, Y, idx, batch, ws=ws)
        panda.mlp_adam(p, m, v, g, step, lr=lr)
        if step % log_every == 0 or step == 1:
            losses.append(loss.item())
    return p, losses


def predict(params, W, P, C, sketch_seed: int = 0):
    """W_pred of normalised device priors."""
    F, tau = features(W, P, C, sketch_seed)
    y = panda.mlp_forward(params, F)
    return panda.ws_predict(W, y.reshape(W.shape), tau)


@dataclass
class WarmResult:
    W: object
    P: object
    C: object
    t: int            # final iteration number (t0 + polish iterations)
    polish: int       # iterations run from the warm state
    h: float
    converged: bool   # h < tol after more than one polish iteration
    frozen: bool      # h < tol at once: the warm state did not move


def warm_run(params, W, P, C, t0: int, sketch_seed: int = 0, opts=None, max_polish: int = 200):
    """Prediction, warm state at t0, then iterations until h < tol."""
    Ne, Na = W.shape
    Wp = predict(params, W, P, C, sketch_seed)
    ctx = panda.Context(Ne, Na, opts)
    ctx.load(W, P, C)
    ctx.ws_init(Wp, t0)
    t = t0
    h = float("inf")
    for _ in range(max_polish):
        h, t2 = ctx.iterate()
        if t2 == t:
            break
        t = t2
    Wf, Pf, Cf, h, t = ctx.state()
    o = opts or panda.default_options()
    ctx.close()
    # a warm state whose first iteration already has h < tol did not move:
    # that is not a converged run of the method, and the judge rejects it
    frozen = h < o.tol and t - t0 <= 1
    return WarmResult(Wf, Pf, Cf, t, t - t0, h, h < o.tol and not frozen, frozen)


def judged_run(params, W, P, C, t0: int, sketch_seed: int = 0, opts=None, rel_tol: float = 1e-3,
               plain=None):
    """Warm run judged by the plain run: accepted when max|W_warm - W_plain| <=
    rel_tol * max(1, max|W_plain|); otherwise the plain result stands."""
    warm = warm_run(params, W, P, C, t0, sketch_seed, opts)
    if plain is None:
        plain = panda.run(W, P, C, opts=opts)
    err = (warm.W - plain.W).abs().max().item()
    scale = max(1.0, plain.W.abs().max().item())
    ok = warm.converged and err <= rel_tol * scale
    return {"accepted": ok, "warm": warm, "plain": plain, "max_abs_err": err, "scale": scale,
            "result_W": warm.W if ok else plain.W}


def amplification(W, P, C, t0s, eps: float = 1e-4, seed: int = 0, opts=None, plain=None):
    """For each t0: run the plain method to iteration t0, multiply every entry
    of W by (1 + eps u), u ~ U(-1, 1), resume from there (a stored state
    resumes exactly) and run to h < tol.  Returns {t0: {"amp": max|dW| /
    max(1, max|W|) / eps at the end, "iters": stopping iteration}} and the
    plain run.  A warm state at t0 is accepted only if its own W is within
    about 1e-3 / amp of the plain run's W at t0."""
    torch = _torch()
    Ne, Na = W.shape
    if plain is None:
        plain = panda.run(W, P, C, opts=opts)
    scale = max(1.0, plain.W.abs().max().item())
    g = torch.Generator(device="cuda").manual_seed(seed)
    out = {}
    for t0 in t0s:
        ctx = panda.Context(Ne, Na, opts)
        ctx.load(W, P, C)
        t = 0
        while t < t0:
            _, t2 = ctx.iterate()
            if t2 == t:
                break
            t = t2
        Wt, Pt, Ct, _, tt = ctx.state()
        ctx.close()
        u = torch.rand(Wt.shape, generator=g, device="cuda") * 2 - 1
        Wp = (Wt.double() * (1 + eps * u.double())).float()
        ctx = panda.Context(Ne, Na, opts)
        ctx.load(Wp, Pt, Ct, t=tt)
        t = tt
        while True:
            _, t2 = ctx.iterate()
            if t2 == t:
                break
            t = t2
        Wf = ctx.state()[0]
        ctx.close()
        out[int(t0)] = {"amp": (Wf - plain.W).abs().max().item() / scale / eps, "iters": int(t)}
    return out, plain
