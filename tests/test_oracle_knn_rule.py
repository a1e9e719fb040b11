"""Pins for the corrected k-NN object-pair pruning rule (Algorithm 6)."""
import json
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(__file__), "golden", "knn_fig13.json")


def _run_story(orc):
    g = json.load(open(GOLD))
    names = {"UNDECIDED": orc.UNDECIDED, "CONFIRMED": orc.CONFIRMED, "REMOVED": orc.REMOVED}
    status = np.zeros(4, np.int64)
    ids = np.asarray(g["ids"])
    for st in g["stages"]:
        k_left = g["k"] - int(np.sum(status == orc.CONFIRMED))
        status = orc.knn_prune(np.asarray(st["lb"]), np.asarray(st["ub"]), ids, status, k_left)
        assert [int(x) for x in status] == [names[e] for e in st["expect"]], st["name"]
    return status


def test_fig13_story(orc):
    final = _run_story(orc)
    assert sorted(np.nonzero(final == orc.CONFIRMED)[0].tolist()) == [0, 3]  # {O1, O4}


def _printed_rule_confirms(lb, ub, m, k_left):
    """The rule as printed: confirm if N - farther < kLeft."""
    N = len(lb)
    farther = sum(1 for n in range(N) if n != m and ub[m] <= lb[n])
    return N - farther < k_left


def test_clear_nearest_neighbour_k1(orc):
    lb, ub, ids = np.array([1.0, 3.0]), np.array([2.0, 4.0]), np.array([0, 1])
    # the printed rule never confirms the obvious nearest neighbour ...
    assert not _printed_rule_confirms(lb, ub, 0, 1)
    # ... the corrected one does, and drops the other
    st = orc.knn_prune(lb, ub, ids, np.zeros(2, np.int64), 1)
    assert st.tolist() == [orc.CONFIRMED, orc.REMOVED]


def test_exact_ties_broken_by_id(orc):
    lb = np.zeros(3)
    ub = np.zeros(3)
    ids = np.array([5, 3, 9])
    st = orc.knn_prune(lb, ub, ids, np.zeros(3, np.int64), 1)
    assert st.tolist() == [orc.REMOVED, orc.CONFIRMED, orc.REMOVED]
    st = orc.knn_prune(lb, ub, ids, np.zeros(3, np.int64), 2)
    assert st.tolist() == [orc.CONFIRMED, orc.CONFIRMED, orc.REMOVED]


def test_rule_never_contradicts_truth(orc):
    """Random true distances inside random intervals: confirmed candidates
    are always in the true top-k of (d, id), removed ones never are."""
    rng = np.random.default_rng(0)
    for _ in range(2000):
        n = int(rng.integers(1, 9))
        k = int(rng.integers(1, 5))
        d = np.round(rng.uniform(0, 5, n), 1)
        ids = rng.permutation(n)
        lb = d - np.round(rng.uniform(0, 1, n), 1) * rng.integers(0, 2, n)
        ub = d + np.round(rng.uniform(0, 1, n), 1) * rng.integers(0, 2, n)
        truth = set(np.lexsort((ids, d))[:k].tolist())
        st = orc.knn_prune(lb, ub, ids, np.zeros(n, np.int64), k)
        for m in range(n):
            if st[m] == orc.CONFIRMED:
                assert m in truth
            if st[m] == orc.REMOVED:
                assert m not in truth
        # with exact intervals every candidate is decided
        st = orc.knn_prune(d, d, ids, np.zeros(n, np.int64), k)
        assert not np.any(st == orc.UNDECIDED)
        assert set(np.nonzero(st == orc.CONFIRMED)[0].tolist()) == truth
