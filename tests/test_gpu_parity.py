"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Both sides start from the same arrays: the seeded raw priors are z-scored by
the oracle in FP64 and rounded to FP32; the GPU receives the FP32 values and
the oracle the same values widened to FP64, so input rounding is not counted.

Tolerances.  W: max-abs 1e-4 (the plain FP32 target).  Single similarity
matrices: a first-order bound of FP32 accumulation over K terms,
|dT| <= 2 K u sum_k |x_k y_k| / sqrt(den) + 4 u |T| with u = 2^-24.
P and C off-diagonals: max-abs 1e-4.  Diagonals of P and C grow like
exp(2 alpha t), so they are compared relative to their size (1e-5).
"""
import numpy as np
import pytest

from paper_1507_07039_amd import inputs as I

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


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


def f32r(a):
    """Round to FP32 and widen back to FP64 (keeps the array shape)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def cuda(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def prep(oracle, W0, P0, C0):
    """Oracle z-score in FP64, then FP32 rounding: the shared start."""
    return tuple(f32r(oracle.normalize(M)) for M in (W0, P0, C0))


def t_bound(X, Y, T):
    K = X.shape[1]
    absdot = np.abs(X) @ np.abs(Y)
    den = (X ** 2).sum(1)[:, None] + (Y ** 2).sum(0)[None, :] - np.abs(X @ Y)
    with np.errstate(divide="ignore", invalid="ignore"):
        b = np.where(den > 0, 2 * K * U * absdot / np.sqrt(np.maximum(den, 1e-300)), 0.0)
    return b + 4 * U * np.abs(T) + 1e-30


# ------------------------------------------------------------- Tfunction ---

@pytest.mark.parametrize("M,K,N", [(1, 1, 1), (3, 5, 7), (64, 16, 256), (65, 17, 257),
                                   (70, 333, 300), (130, 700, 513), (40, 400, 400)])
def test_tanimoto_matches_oracle(torch, pd, oracle, M, K, N):
    X = f32r(I.random_dense(M * 7 + K, (M, K)))
    Y = f32r(I.random_dense(N * 5 + K, (K, N), -2.0, 2.0))
    got = host(pd.tanimoto(cuda(torch, X), cuda(torch, Y)))
    want = oracle.tanimoto(X, Y)
    err = np.abs(got - want)
    bound = t_bound(X, Y, want)
    assert np.all(err <= bound), (err.max(), (err / bound).max())


@pytest.mark.parametrize("sx,sy", [(1e18, 1e18), (1e-18, 1e-18), (1e18, 1.0), (1.0, 1e-17)])
def test_tanimoto_extreme_magnitudes(torch, pd, oracle, sx, sy):
    # squared norms far outside FP32's range (as the diagonals of P and C reach
    # late in long runs): the denominator must not overflow or flush to zero
    X = f32r(sx * I.random_dense(11, (33, 50)))
    Y = f32r(sy * I.random_dense(12, (50, 70), -2.0, 2.0))
    got = host(pd.tanimoto(cuda(torch, X), cuda(torch, Y)))
    want = oracle.tanimoto(X, Y)
    assert np.all(np.isfinite(got))
    err = np.abs(got - want)
    bound = t_bound(X, Y, want)
    assert np.all(err <= bound), (err.max(), (err / bound).max())


def test_tanimoto_zero_vectors(torch, pd, oracle):
    X = np.zeros((5, 9))
    X[2] = 1.0
    Y = np.zeros((9, 4))
    Y[:, 1] = -1.0
    got = host(pd.tanimoto(cuda(torch, X), cuda(torch, Y)))
    np.testing.assert_array_equal(got, oracle.tanimoto(X, Y))


# ------------------------------------------------------------- z-score -----

def test_normalize_matches_oracle(torch, pd, oracle):
    W0, P0, C0 = I.workload_priors(I.SMALL)
    for M in (W0, P0, C0, I.random_dense(3, (17, 33), 5.0, 9.0)):
        M32 = f32r(M)
        t = cuda(torch, M32)
        pd.normalize(t)
        want = oracle.normalize(M32)
        assert np.abs(host(t) - want).max() <= 2e-7 * max(1.0, np.abs(want).max())


def test_normalize_errors(torch, pd):
    t = torch.full((8, 8), 3.0, device="cuda")
    with pytest.raises(pd.PandaError) as e:
        pd.normalize(t)
    assert e.value.code == pd.ERR_DEGENERATE
    assert torch.all(t == 3.0)
    t[3, 4] = float("nan")
    with pytest.raises(pd.PandaError) as e:
        pd.normalize(t)
    assert e.value.code == pd.ERR_NONFINITE


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("ddof", [0, 1])
def test_normalize_ex_matches_oracle(torch, pd, oracle, mode, ddof):
    """Every scope and normaliser of the z-score against the oracle's, on
    the small workload's priors, a ragged dense matrix, one-row and one-column
    shapes (where the scope allows them) and the identity."""
    W0, P0, C0 = I.workload_priors(I.SMALL)
    cases = [W0, P0, C0, I.random_dense(3, (17, 33), 5.0, 9.0), np.eye(130)]
    if mode == 0:
        cases += [I.random_dense(4, (1, 9), 1.0, 2.0), I.random_dense(5, (7, 1), 1.0, 2.0)]
    if mode == 1:
        cases += [I.random_dense(4, (1, 9), 1.0, 2.0), I.random_dense(6, (300, 2), 1.0, 2.0)]
    for M in cases:
        M32 = f32r(M)
        t = cuda(torch, M32)
        try:
            want = oracle.normalize_ex(M32, mode, ddof)
        except oracle.OracleError as e:  # e.g. W0 has empty columns: both sides refuse
            with pytest.raises(pd.PandaError) as g:
                pd.normalize(t, mode=mode, ddof=ddof)
            assert g.value.code == e.code == pd.ERR_DEGENERATE
            continue
        pd.normalize(t, mode=mode, ddof=ddof)
        # one FP32 rounding of an FP64 value (the moments agree to FP64 rounding)
        err = np.abs(host(t) - want).max()
        assert err <= 2e-7 * max(1.0, np.abs(want).max()), (M.shape, err)


def test_normalize_ex_errors(torch, pd):
    rng = np.random.default_rng(11)
    M = rng.normal(size=(6, 9)).astype(np.float32)
    M[2] = 1.5  # constant row
    t = cuda(torch, M)
    pd.normalize(t, mode=pd.ZSCORE_GLOBAL, ddof=1)  # fine for the global scope
    for mode in (pd.ZSCORE_ROW, pd.ZSCORE_ROWCOL):
        t = cuda(torch, M)
        with pytest.raises(pd.PandaError) as e:
            pd.normalize(t, mode=mode)
        assert e.value.code == pd.ERR_DEGENERATE
        assert np.array_equal(host(t), M.astype(np.float64))  # untouched
    M = rng.normal(size=(6, 9)).astype(np.float32)
    M[:, 4] = -2.0  # constant column: only the row + column scope fails
    pd.normalize(cuda(torch, M), mode=pd.ZSCORE_ROW)
    with pytest.raises(pd.PandaError) as e:
        pd.normalize(cuda(torch, M), mode=pd.ZSCORE_ROWCOL)
    assert e.value.code == pd.ERR_DEGENERATE
    with pytest.raises(pd.PandaError) as e:  # one entry per row, sample std
        pd.normalize(cuda(torch, M[:, :1].copy()), mode=pd.ZSCORE_ROW, ddof=1)
    assert e.value.code == pd.ERR_DEGENERATE
    M[3, 3] = np.nan
    for mode in (0, 1, 2):
        with pytest.raises(pd.PandaError) as e:
            pd.normalize(cuda(torch, M), mode=mode, ddof=1)
        assert e.value.code == pd.ERR_NONFINITE
    with pytest.raises(pd.PandaError) as e:
        pd.normalize(cuda(torch, M), mode=3)
    assert e.value.code == pd.ERR_ARG


# ------------------------------------------------------------ iterations ---

def compare_state(W, P, C, Wo, Po, Co, what=""):
    eW = np.abs(W - Wo).max()
    off_p = ~np.eye(P.shape[0], dtype=bool)
    off_c = ~np.eye(C.shape[0], dtype=bool)
    eP = np.abs(P - Po)[off_p].max() if P.shape[0] > 1 else 0.0
    eC = np.abs(C - Co)[off_c].max() if C.shape[0] > 1 else 0.0
    dP = np.abs(np.diag(P) - np.diag(Po)) / np.maximum(1.0, np.abs(np.diag(Po)))
    dC = np.abs(np.diag(C) - np.diag(Co)) / np.maximum(1.0, np.abs(np.diag(Co)))
    assert eW <= 1e-4, (what, "W", eW)
    assert eP <= 1e-4, (what, "P", eP)
    assert eC <= 1e-4, (what, "C", eC)
    assert dP.max() <= 1e-5, (what, "diag P", dP.max())
    assert dC.max() <= 1e-5, (what, "diag C", dC.max())
    assert np.array_equal(P, P.T) and np.array_equal(C, C.T), what


def run_matched(torch, pd, oracle, W, P, C, opts_kw=None, steps=None, pass_identity=False):
    """Step GPU and oracle side by side; compare after every iteration."""
    opts_kw = opts_kw or {}
    o = oracle.Options(**opts_kw)
    po = pd.default_options(**{k: int(v) if isinstance(v, bool) else v for k, v in opts_kw.items()})
    Ne, Na = W.shape
    ctx = pd.Context(Ne, Na, po)
    if pass_identity:
        ctx.load(cuda(torch, W))
    else:
        ctx.load(cuda(torch, W), cuda(torch, P), cuda(torch, C))
    Wo, Po, Co = W.copy(), P.copy(), C.copy()
    t = 0
    n = steps or o.max_iter
    conv = False
    while t < n and not conv:
        t += 1
        Wo, Po, Co, ho, conv = oracle.step(Wo, Po, Co, t, o)
        hg, tg = ctx.iterate()
        assert tg == t
        # h is a mean of |dW| over FP32 entries: relative 1e-5 (FP32 sums of
        # many terms with cancellation lose a few more bits than one ulp)
        assert abs(hg - ho) <= 1e-5 * ho + 1e-9, (t, hg, ho)
        Wg, Pg, Cg, _, _ = ctx.state()
        compare_state(host(Wg), host(Pg), host(Cg), Wo, Po, Co, what=f"t={t}")
    return t, ctx


def test_small_workload_matched_iterations(torch, pd, oracle):
    W, P, C = prep(oracle, *I.workload_priors(I.SMALL))
    t, ctx = run_matched(torch, pd, oracle, W, P, C)
    assert 20 <= t <= 60
    # converged state is frozen
    h1, t1 = ctx.iterate()
    assert t1 == t


@pytest.mark.parametrize("kw", [{"diag_alpha": False}, {"sigma_from_T": True}, {"n_own": True},
                                {"h_undamped": True}, {"update_last": True}, {"sigma_ddof": 1},
                                {"sigma_ddof": 1, "sigma_from_T": True},
                                {"alpha": 0.3, "tol": 1e-4}])
def test_readings_flags(torch, pd, oracle, kw):
    W, P, C = prep(oracle, *I.workload_priors(I.SMALL))
    run_matched(torch, pd, oracle, W, P, C, opts_kw=kw, steps=12)


@pytest.mark.parametrize("Ne,Na", [(1, 1), (1, 7), (3, 1), (2, 5), (65, 300), (70, 257)])
def test_ragged_shapes(torch, pd, oracle, Ne, Na):
    rng = np.random.default_rng(Ne * 1000 + Na)
    W = f32r(rng.normal(size=(Ne, Na)))
    P = f32r(I.random_symmetric(Ne + 1, Ne))
    C = f32r(I.random_symmetric(Na + 2, Na))
    run_matched(torch, pd, oracle, W, P, C, steps=6)


def test_identity_defaults(torch, pd, oracle):
    """NULL P0 / C0 mean identity networks, z-scored like any other."""
    W0, _, _ = I.workload_priors(I.SMALL)
    W = f32r(oracle.normalize(W0))
    Ne, Na = W.shape
    # the GPU builds the identities and z-scores them in FP64 before storing
    # FP32; the oracle gets the same FP32-rounded values
    P = f32r(oracle.normalize(np.eye(Ne)))
    C = f32r(oracle.normalize(np.eye(Na)))
    ctx = pd.Context(Ne, Na)
    ctx.load(cuda(torch, W))
    _, Pg, Cg, _, t0 = ctx.state()
    assert t0 == 0
    assert np.abs(host(Pg) - P).max() <= 2e-7 * np.abs(P).max()
    assert np.abs(host(Cg) - C).max() <= 2e-7 * np.abs(C).max()
    run_matched(torch, pd, oracle, W, P, C, steps=5, pass_identity=True)


@pytest.mark.parametrize("mode,ddof", [(1, 0), (2, 1), (0, 1)])
def test_identity_defaults_other_scopes(torch, pd, oracle, mode, ddof):
    """The identity default is z-scored with the context's scope and
    normaliser; the run from it follows the oracle with the same sigma rule."""
    W0, _, _ = I.workload_priors(I.SMALL)
    W = f32r(oracle.normalize(W0))
    Ne, Na = W.shape
    P = f32r(oracle.normalize_ex(np.eye(Ne), mode, ddof))
    C = f32r(oracle.normalize_ex(np.eye(Na), mode, ddof))
    ctx = pd.Context(Ne, Na, pd.default_options(zscore_mode=mode, sigma_ddof=ddof))
    ctx.load(cuda(torch, W))
    _, Pg, Cg, _, _ = ctx.state()
    assert np.abs(host(Pg) - P).max() <= 2e-7 * np.abs(P).max()
    assert np.abs(host(Cg) - C).max() <= 2e-7 * np.abs(C).max()
    run_matched(torch, pd, oracle, W, P, C, opts_kw={"sigma_ddof": ddof}, steps=5)


def test_run_entry_point(torch, pd, oracle):
    W, P, C = prep(oracle, *I.workload_priors(I.SMALL))
    ref = oracle.run(W, P, C)
    res = pd.run(cuda(torch, W), cuda(torch, P), cuda(torch, C))
    assert res.status == pd.OK
    assert res.iters == ref.iters
    # h (Eq. 7) is a mean of differences of FP32-rounded W entries: its error
    # is a few FP32 ulps of those entries, not of h itself
    assert abs(res.h - ref.h) <= 8 * U * np.abs(ref.W).mean()
    compare_state(host(res.W), host(res.P), host(res.C), ref.W, ref.P, ref.C, "run")
    # max_iter exhaustion returns NOT_CONVERGED with the state of that step
    short = pd.run(cuda(torch, W), cuda(torch, P), cuda(torch, C), max_iter=5)
    assert short.status == pd.NOT_CONVERGED and short.iters == 5
    ref5 = oracle.run(W, P, C, oracle.Options(max_iter=5))
    compare_state(host(short.W), host(short.P), host(short.C), ref5.W, ref5.P, ref5.C, "max_iter")


def test_run_poll_every_and_determinism(torch, pd, oracle):
    W, P, C = prep(oracle, *I.workload_priors(I.SMALL))
    a = pd.run(cuda(torch, W), cuda(torch, P), cuda(torch, C))
    b = pd.run(cuda(torch, W), cuda(torch, P), cuda(torch, C), opts=pd.default_options(poll_every=7))
    assert a.iters == b.iters and a.h == b.h
    assert torch.equal(a.W, b.W) and torch.equal(a.P, b.P) and torch.equal(a.C, b.C)


@pytest.mark.parametrize("precision", [0, 1])
def test_run_one_iteration_ahead_equals_stepwise(torch, pd, oracle, precision):
    # panda_run keeps the next iteration queued while it checks h of the last
    # one; the iteration it queues after convergence runs gated.  The result
    # must be that of a context stepped one synchronous iteration at a time,
    # also when the cap falls on the converging iteration or just before it.
    W, P, C = prep(oracle, *I.workload_priors(I.SMALL))
    Ne, Na = W.shape
    opts = pd.default_options(precision=precision)
    ctx = pd.Context(Ne, Na, opts)
    ctx.load(cuda(torch, W), cuda(torch, P), cuda(torch, C))
    for _ in range(200):
        h, t = ctx.iterate()
        if h < 1e-3:
            break
    Ws, Ps, Cs, hs, ts = ctx.state()
    ctx.close()
    for cap in (ts + 3, ts, ts - 1, 1):
        r = pd.run(cuda(torch, W), cuda(torch, P), cuda(torch, C), max_iter=cap, opts=opts)
        if cap >= ts:
            assert r.status == pd.OK and r.iters == ts and r.h == hs
            assert torch.equal(r.W, Ws) and torch.equal(r.P, Ps) and torch.equal(r.C, Cs)
        else:
            assert r.status == pd.NOT_CONVERGED and r.iters == cap


@pytest.mark.parametrize("precision,packed", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_resume_equals_straight_run(torch, pd, oracle, precision, packed):
    """A state stored after 9 iterations and loaded into a new context runs to
    the same result bit for bit (split-BF16: R after the load comes from its
    own launch, later R from the C update's launch, with the same arithmetic)."""
    W, P, C = prep(oracle, *I.workload_priors(I.SMALL))
    opts = pd.default_options(precision=precision, packed_c=packed)
    straight = pd.run(cuda(torch, W), cuda(torch, P), cuda(torch, C), opts=opts)
    ctx = pd.Context(*W.shape, opts)
    ctx.load(cuda(torch, W), cuda(torch, P), cuda(torch, C))
    for _ in range(9):
        ctx.iterate()
    Wk, Pk, Ck, hk, tk = ctx.state()
    assert tk == 9
    ctx2 = pd.Context(*W.shape, opts)
    ctx2.load(Wk, Pk, Ck, t=tk)
    t = tk
    while True:
        h, t2 = ctx2.iterate()
        if t2 == t:
            break
        t = t2
    Wr, Pr, Cr, hr, tr = ctx2.state()
    assert tr == straight.iters
    assert torch.equal(Wr, straight.W) and torch.equal(Cr, straight.C) and torch.equal(Pr, straight.P)


def test_diagonals_past_fp32_range(torch, pd, oracle):
    """At alpha = 1 the Eq. 6 diagonals pass FLT_MAX near t = 40 (they reach
    ~1e55 by t = 60).  They stay FP64 on the GPU, so W and the off-diagonal
    entries keep following the FP64 oracle; a stored diagonal past the FP32
    range reads +inf, every other one matches."""
    W, P, C = prep(oracle, *I.workload_priors(I.SMALL))
    kw = dict(alpha=1.0, tol=0.0, max_iter=60)
    ref = oracle.run(W, P, C, oracle.Options(**kw))
    assert ref.status == oracle.NOT_CONVERGED and np.diag(ref.P).max() > 1e50
    res = pd.run(cuda(torch, W), cuda(torch, P), cuda(torch, C), **kw)
    assert res.status == pd.NOT_CONVERGED and res.iters == 60
    Wg, Pg, Cg = host(res.W), host(res.P), host(res.C)
    assert np.abs(Wg - ref.W).max() <= 1e-4
    for G, R in ((Pg, ref.P), (Cg, ref.C)):
        off = ~np.eye(G.shape[0], dtype=bool)
        assert np.abs(G - R)[off].max() <= 1e-4
        dg, dr = np.diag(G), np.diag(R)
        big = np.abs(dr) > np.finfo(np.float32).max
        assert big.any() and np.all(dg[big] == np.inf)
        assert np.all(np.abs(dg[~big] - dr[~big]) <= 1e-5 * np.abs(dr[~big]))


# ------------------------------------------------------- packed C storage --

@pytest.mark.parametrize("precision", [0, 1])
def test_packed_c_runs_like_full_storage(torch, pd, oracle, precision):
    """C stored as its upper 128 x 128 tiles: the products read the same values
    in the same order, so every iteration equals the full-storage one bit for
    bit (W, P, C, h), on the small workload and on ragged shapes that leave
    partial tiles, and both follow the oracle."""
    cases = [prep(oracle, *I.workload_priors(I.SMALL))]
    for Ne, Na in ((1, 7), (3, 1), (65, 300), (70, 257), (9, 129)):
        rng = np.random.default_rng(Ne * 1000 + Na)
        cases.append((f32r(rng.normal(size=(Ne, Na))), f32r(I.random_symmetric(Ne + 1, Ne)),
                      f32r(I.random_symmetric(Na + 2, Na))))
    for W, P, C in cases:
        Ne, Na = W.shape
        ctx = {k: pd.Context(Ne, Na, pd.default_options(precision=precision, packed_c=k, tol=0.0))
               for k in (0, 1)}
        for k in (0, 1):
            ctx[k].load(cuda(torch, W), cuda(torch, P), cuda(torch, C))
        Wo, Po, Co = W, P, C
        for t in range(1, 7):
            h0, _ = ctx[0].iterate()
            h1, _ = ctx[1].iterate()
            assert h0 == h1, (W.shape, t)
            s0, s1 = ctx[0].state(), ctx[1].state()
            for a, b in zip(s0[:3], s1[:3]):
                assert torch.equal(a, b), (W.shape, t)
            if precision == 0:  # the split-BF16 form has its own bounds (test_gpu_precision)
                Wo, Po, Co, _, _ = oracle.step(Wo, Po, Co, t, oracle.Options(tol=0.0))
                compare_state(host(s1[0]), host(s1[1]), host(s1[2]), Wo, Po, Co, f"packed t={t}")


def test_packed_c_identity_default_and_run(torch, pd, oracle):
    """The identity default of a packed context (its z-score in closed form)
    against the oracle's z-scored identity, then panda_run from it."""
    W0, _, _ = I.workload_priors(I.SMALL)
    W = f32r(oracle.normalize(W0))
    Ne, Na = W.shape
    for mode, ddof in ((0, 0), (2, 1)):
        opts = pd.default_options(packed_c=1, zscore_mode=mode, sigma_ddof=ddof)
        ctx = pd.Context(Ne, Na, opts)
        ctx.load(cuda(torch, W))
        _, Pg, Cg, _, _ = ctx.state()
        C = oracle.normalize_ex(np.eye(Na), mode, ddof)
        assert np.abs(host(Cg) - C).max() <= 2e-7 * np.abs(C).max()
        P = oracle.normalize_ex(np.eye(Ne), mode, ddof)
        assert np.abs(host(Pg) - P).max() <= 2e-7 * np.abs(P).max()
    res = pd.run(cuda(torch, W), None, None, opts=pd.default_options(packed_c=1))
    ref = oracle.run(W, f32r(oracle.normalize(np.eye(Ne))), f32r(oracle.normalize(np.eye(Na))))
    assert res.iters == ref.iters
    compare_state(host(res.W), host(res.P), host(res.C), ref.W, ref.P, ref.C, "packed identity")
