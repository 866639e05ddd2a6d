"""The KGC's selection (Algorithm 2) and mask plaintexts, product code
against the oracle's independent implementation and against the paper's
worked example; runs on the CPU."""
import pathlib

import numpy as np
import pytest

from paper_2408_06197_amd import robust


def test_selection_matches_oracle(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(11)
    for _ in range(300):
        n = int(rng.integers(3, 30))
        c = int(rng.integers(0, max(1, (n - 3) // 2) + 1))
        vals = rng.integers(0, 6, size=n * (n - 1) // 2).astype(float)  # many ties
        D = robust.distance_matrix(vals, n)
        assert np.array_equal(D, O.distance_matrix(vals, n))
        assert np.allclose(robust.krum_scores(D, c), O.krum_scores(D, c))
        for rule in robust.RULES:
            l = int(rng.integers(1, n + 1))
            assert robust.select(rule, D, c, l) == O.select(rule, D, c, l), (rule, n, c, l)


def test_byzantine_outliers_not_selected():
    rng = np.random.default_rng(3)
    n, c, dim = 12, 3, 500
    w = rng.normal(0, 0.01, (n, dim))
    w[-c:] = rng.normal(0, 0.1, (c, dim))  # the last c clients are far from the rest
    vals = [np.sum((w[i] - w[j]) ** 2) for i in range(n) for j in range(i + 1, n)]
    D = robust.distance_matrix(vals, n)
    for rule in robust.RULES:
        chosen = robust.select(rule, D, c, l=n - c)
        assert chosen and all(i < n - c for i in chosen), rule


def test_multikrum_stopping_rule():
    n, c = 10, 3
    D = robust.distance_matrix(np.arange(n * (n - 1) // 2, dtype=float), n)
    assert len(robust.select("multikrum", D, c, l=10)) == n - (2 * c + 2)   # n - |psi| > 2c + 2
    assert len(robust.select("multikrum", D, c, l=1)) == 1


def test_paper_example_mask_rows():
    """The 5-client example of Masked-based Encrypted Sorting
    (tests/golden/permutation_mask_5clients.txt): clients 1, 3, 5 (1-based)
    used, two zero rows; here as weights and constant plaintexts."""
    P = np.loadtxt(pathlib.Path(__file__).parent / "golden" / "permutation_mask_5clients.txt", comments="#")
    chosen = [int(j) for j in np.nonzero(P.any(axis=0))[0]]
    assert chosen == [0, 2, 4]
    w = robust.weights("multikrum", chosen, 5)
    assert np.allclose(w, [1 / 3, 0, 1 / 3, 0, 1 / 3])
    m = robust.mask_plaintexts(w, 16, 2.0 ** 40)
    assert m.shape == (5, 16) and np.all(m[:, 1:] == 0)
    assert list(m[:, 0]) == [round(2 ** 40 / 3), 0, round(2 ** 40 / 3), 0, round(2 ** 40 / 3)]
    assert np.allclose(robust.weights("krum", [3], 5), [0, 0, 0, 1, 0])


def test_bad_rule():
    with pytest.raises(ValueError):
        robust.select("trimmed", np.zeros((3, 3)), 0)
