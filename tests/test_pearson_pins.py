"""Pins of the oracle's co-expression prior (Sec. II-A: Pearson correlation
between pairs of genes across all samples) against a library routine and the
properties a correlation has by definition."""
import numpy as np
import pytest

from paper_1507_07039_amd import inputs as I

RNG = np.random.default_rng(1507)


def test_matches_numpy_corrcoef(oracle):
    for G, S in ((1, 2), (5, 2), (37, 3), (120, 50)):
        E = RNG.normal(size=(G, S)) * RNG.uniform(0.1, 10, size=(G, 1)) + RNG.normal(size=(G, 1))
        C = oracle.pearson(E)
        assert C.shape == (G, G)
        np.testing.assert_allclose(C, np.atleast_2d(np.corrcoef(E)), rtol=0, atol=1e-13)


def test_constant_row_gets_zero_and_unit_diagonal(oracle):
    E = RNG.normal(size=(9, 14))
    E[3] = 2.5
    E[7] = 0.0
    C = oracle.pearson(E)
    for r in (3, 7):
        assert np.all(np.delete(C[r], r) == 0.0) and np.all(np.delete(C[:, r], r) == 0.0)
    assert np.all(np.diag(C) == 1.0)
    keep = [i for i in range(9) if i not in (3, 7)]
    np.testing.assert_allclose(C[np.ix_(keep, keep)], np.corrcoef(E[keep]), atol=1e-13)


def test_identical_and_negated_rows(oracle):
    x = RNG.normal(size=40)
    E = np.stack([x, x, -x, 3.0 * x + 7.0, -0.5 * x - 1.0])
    C = oracle.pearson(E)
    sign = np.array([1, 1, -1, 1, -1], dtype=np.float64)
    np.testing.assert_allclose(C, np.outer(sign, sign), rtol=0, atol=1e-14)


def test_affine_row_invariance_and_symmetry(oracle):
    E = RNG.normal(size=(30, 25))
    a = RNG.uniform(0.01, 100.0, size=(30, 1))
    b = RNG.normal(scale=50.0, size=(30, 1))
    C1 = oracle.pearson(E)
    C2 = oracle.pearson(a * E + b)
    np.testing.assert_allclose(C2, C1, rtol=0, atol=1e-12)
    assert np.array_equal(C1, C1.T)
    assert np.all(np.abs(C1) <= 1.0 + 1e-15)


def test_two_samples_is_sign(oracle):
    # With two samples every non-constant centred row is +-(d, -d): r = +-1.
    E = RNG.normal(size=(12, 2))
    C = oracle.pearson(E)
    s = np.sign(E[:, 0] - E[:, 1])
    np.testing.assert_allclose(C, np.outer(s, s), atol=1e-15)


def test_positive_semidefinite(oracle):
    # A correlation matrix is a Gram matrix of unit vectors: PSD, rank <= S - 1.
    E = RNG.normal(size=(60, 9))
    w = np.linalg.eigvalsh(oracle.pearson(E))
    assert w.min() > -1e-12
    assert np.sum(w > 1e-9) == 8


def test_entries_match_full_matrix(oracle):
    E = RNG.normal(size=(50, 17))
    E[4] = 1.0
    C = oracle.pearson(E)
    r = RNG.integers(0, 50, size=200)
    c = RNG.integers(0, 50, size=200)
    assert np.array_equal(oracle.pearson_entries(E, r, c), C[r, c])


def test_workload_prior_is_the_pearson_of_its_expression(oracle):
    _, _, C0 = I.workload_priors(I.SMALL)
    E = I.workload_expression(I.SMALL)
    np.testing.assert_allclose(oracle.pearson(E), C0, rtol=0, atol=1e-13)


def test_bad_arguments(oracle):
    with pytest.raises(Exception):
        oracle.pearson(np.ones((4, 1)))
    with pytest.raises(Exception):
        oracle.pearson_entries(np.ones((4, 3)), [0, 4], [0, 0])
