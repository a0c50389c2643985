"""Pins of the permutation-null oracle (node-label randomisation, Sec. III)
against relabelling identities and closed forms."""
import numpy as np
import pytest

from oracle import null as N
from paper_1507_07039_amd import inputs as I

RNG = np.random.default_rng(178)


@pytest.fixture(scope="module")
def small(oracle):
    W0, P0, C0 = I.priors(4321, 12, 60, 0.1, 0.1, 20, 4)
    return tuple(oracle.normalize(M) for M in (W0, P0, C0))


def inv(p):
    q = np.empty_like(p)
    q[p] = np.arange(p.size)
    return q


def test_permute_sym_group_laws():
    M = RNG.normal(size=(9, 9))
    a, b = RNG.permutation(9), RNG.permutation(9)
    assert np.array_equal(N.permute_sym(N.permute_sym(M, a), b), N.permute_sym(M, a[b]))
    assert np.array_equal(N.permute_sym(N.permute_sym(M, a), inv(a)), M)
    assert np.array_equal(N.permute_sym(M, np.arange(9)), M)
    S = M + M.T
    assert np.array_equal(N.permute_sym(S, a), N.permute_sym(S, a).T)
    with pytest.raises(ValueError):
        N.permute_sym(M, np.array([0, 0, 1, 2, 3, 4, 5, 6, 7]))


def test_identity_relabelling_is_the_plain_run(oracle, small):
    W0, P0, C0 = small
    ident = np.tile(np.arange(60), (3, 1))
    mean, sd, iters, _ = N.null_stats(W0, P0, C0, gene_perms=ident)
    ref = oracle.run(W0, P0, C0)
    np.testing.assert_allclose(mean, ref.W, rtol=1e-13, atol=1e-13)
    assert np.all(sd <= 1e-12 * np.abs(ref.W).max())
    assert iters == [ref.iters] * 3


def test_gene_relabelling_equals_relabelled_motif_prior(oracle, small):
    # Relabelling genes in C only is the plain run from W0 with its columns
    # relabelled the inverse way, read back in the new labels:
    # PANDA(W, P, C[s][s]) = PANDA(W[:, s^-1], P, C)[:, s].
    W0, P0, C0 = small
    s = RNG.permutation(60)
    (r,) = N.null_runs(W0, P0, C0, gene_perms=[s])
    ref = oracle.run(W0[:, inv(s)], P0, C0)
    assert r.iters == ref.iters
    np.testing.assert_allclose(r.W, ref.W[:, s], rtol=0, atol=1e-9 * np.abs(ref.W).max())


def test_tf_relabelling_equals_relabelled_motif_prior(oracle, small):
    W0, P0, C0 = small
    t = RNG.permutation(12)
    (r,) = N.null_runs(W0, P0, C0, tf_perms=[t])
    ref = oracle.run(W0[inv(t), :], P0, C0)
    assert r.iters == ref.iters
    np.testing.assert_allclose(r.W, ref.W[t, :], rtol=0, atol=1e-9 * np.abs(ref.W).max())


def test_two_instances_closed_form(oracle, small):
    W0, P0, C0 = small
    g = np.stack([RNG.permutation(60), RNG.permutation(60)])
    mean, sd, _, _ = N.null_stats(W0, P0, C0, gene_perms=g)
    W1 = oracle.run(W0, P0, C0[np.ix_(g[0], g[0])]).W
    W2 = oracle.run(W0, P0, C0[np.ix_(g[1], g[1])]).W
    np.testing.assert_allclose(mean, 0.5 * (W1 + W2), rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(sd, 0.5 * np.abs(W1 - W2), rtol=1e-12, atol=1e-12)


def test_zscore_closed_form():
    W = np.array([[3.0, 1.0], [2.0, 5.0]])
    mean = np.array([[1.0, 1.0], [4.0, 5.0]])
    sd = np.array([[2.0, 0.0], [0.5, 1.0]])
    assert np.array_equal(N.zscore(W, mean, sd), np.array([[1.0, 0.0], [-4.0, 0.0]]))
