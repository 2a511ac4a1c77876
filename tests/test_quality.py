"""Host reductions of the quality readout (no GPU): misclassification from
confusion counts and the trade-off cost of eq (11), checked on cases worked
by hand."""
import numpy as np

from paper_2002_01981_amd.quality import (best_map_misclassification, misclassification,
                                          tradeoff_cost)


def test_misclassification_by_hand():
    counts = [[50, 5, 0], [10, 30, 5], [0, 0, 100]]
    assert misclassification(counts) == 1.0 - 180.0 / 200.0
    assert misclassification(np.eye(4) * 7) == 0.0


def test_best_map_finds_the_permutation():
    counts = np.array([[0, 40, 1], [30, 0, 2], [3, 0, 50]])
    # identity: 0 + 0 + 50; best: 0->1, 1->0, 2->2 = 40 + 30 + 50
    assert misclassification(counts) == 1.0 - 50.0 / 126.0
    assert abs(best_map_misclassification(counts) - (1.0 - 120.0 / 126.0)) < 1e-15


def test_tradeoff_cost_by_hand():
    # two algorithms, two images
    incS = [[0.10, 0.20], [0.30, 0.40]]
    S = [[1.0, 10.0], [3.0, 30.0]]
    # normalised: incS -> [[0, 0], [1, 1]]; S -> [[0, 0], [1, 1]]
    for a in (0.0, 0.3, 1.0):
        assert np.allclose(tradeoff_cost(incS, S, a), [0.0, 1.0])
    incS = [[0.10, 0.40], [0.30, 0.20]]   # -> [[0, 1], [1, 0]]
    S = [[2.0, 5.0], [1.0, 5.0]]          # -> [[1, 0], [0, 0]] (equal on image 2)
    J = tradeoff_cost(incS, S, 0.25)
    assert np.allclose(J, [(0.25 * 0 + 0.75 * 1 + 0.25 * 1 + 0.75 * 0) / 2,
                           (0.25 * 1 + 0.75 * 0 + 0.25 * 0 + 0.75 * 0) / 2])


def test_tradeoff_cost_limits():
    rng = np.random.default_rng(0)
    incS, S = rng.random((3, 5)), rng.random((3, 5))
    j1 = tradeoff_cost(incS, S, 1.0)
    j0 = tradeoff_cost(incS, S, 0.0)
    jh = tradeoff_cost(incS, S, 0.5)
    assert np.allclose(jh, 0.5 * (j0 + j1))     # linear in alpha
    assert np.all((j0 >= 0) & (j0 <= 1) & (j1 >= 0) & (j1 <= 1))
