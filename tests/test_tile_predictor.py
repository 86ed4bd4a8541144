"""The tile predictor (nearest neighbour, k = 1) against the CPU 1-NN of oracle.knn, and that
1-NN pinned to an independent implementation and to the paper's Table I.  No GPU needed:
wf_tile_predict is host code."""
import os

import numpy as np
import pytest

from oracle import knn
from paper_2510_27351_amd import _lib

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table(name):
    rows = [list(map(float, line.split())) for line in open(os.path.join(GOLDEN, name))
            if line.strip() and not line.startswith("#")]
    return np.array(rows)


def test_oracle_1nn_matches_scikit_learn():
    """Independent pin: scikit-learn's 1-nearest-neighbour classifier, on points drawn so that
    no query is equally near two training points."""
    from sklearn.neighbors import KNeighborsClassifier
    rng = np.random.default_rng(7)
    x = rng.normal(size=(60, 2))
    y = rng.integers(0, 4, size=60)
    q = rng.normal(size=(200, 2))
    ref = KNeighborsClassifier(n_neighbors=1, algorithm="brute").fit(x, y).predict(q)
    assert np.array_equal(knn.predict(x, y, q), ref)


def test_oracle_ties_go_to_the_earlier_point():
    assert knn.predict([[0.0], [2.0]], [5, 7], [[1.0]])[0] == 5
    assert knn.predict([[2.0], [0.0]], [7, 5], [[1.0]])[0] == 7


def _loo_1d_sorted(x, y):
    """Leave-one-out 1-NN accuracy for points sorted along one axis, counted a second way: the
    nearest other point is the left or the right neighbour, the left one on a tie (it comes
    earlier in the table)."""
    hits = 0
    for i in range(len(x)):
        left = x[i] - x[i - 1] if i > 0 else np.inf
        right = x[i + 1] - x[i] if i + 1 < len(x) else np.inf
        hits += y[i - 1 if left <= right else i + 1] == y[i]
    return hits / len(x)


def test_paper_table_one():
    """Table I: the corrected labels follow the trend the paper describes (the sizes fall into
    intervals with one optimum each), so 1-NN on the size predicts them better than the raw
    labels.  Leave-one-out over all 37 sizes (the paper's own split is not printed), checked
    against a count by adjacent neighbours, which is exact in one dimension."""
    t = _table("table1_opt_subsystem.txt")
    assert t.shape == (37, 3)
    assert np.all(np.diff(t[:, 0]) > 0)
    x = np.log10(t[:, 0])
    raw, corrected = t[:, 1].astype(int), t[:, 2].astype(int)
    for y in (raw, corrected):
        assert knn.loo_accuracy(x, y) == pytest.approx(_loo_1d_sorted(x, y))
    loo_raw, loo_cor = knn.loo_accuracy(x, raw), knn.loo_accuracy(x, corrected)
    assert loo_cor > loo_raw
    # the corrected optimum never decreases with N and changes at five sizes: a miss needs a
    # nearest neighbour across one of those boundaries, so at most two misses per boundary
    assert np.all(np.diff(corrected) >= 0)
    boundaries = int(np.count_nonzero(np.diff(corrected)))
    assert boundaries == 5
    assert (1 - loo_cor) * 37 <= 2 * boundaries + 1e-9
    # null accuracy: always predicting the most frequent label (corrected: 32, 12 of 37;
    # raw: 4 and 64, 9 of 37 each)
    assert knn.null_accuracy(corrected) == pytest.approx(12 / 37)
    assert knn.null_accuracy(raw) == pytest.approx(9 / 37)


def test_paper_label_correction_is_the_interval_rule():
    """The corrected column of Table I is the trend of the paper's interval list applied to
    N, and it differs from the measured optimum in exactly the 8 of 37 cases the paper
    counts."""
    t = _table("table1_opt_subsystem.txt")
    N, raw, corrected = t[:, 0], t[:, 1].astype(int), t[:, 2].astype(int)
    assert [knn.interval_rule(v) for v in N] == list(corrected)
    assert int(np.count_nonzero(raw != corrected)) == 8
    # interval ends themselves: closed above
    assert knn.interval_rule(4.5e3) == 4 and knn.interval_rule(4.5e3 + 1) == 8
    assert knn.interval_rule(1e7) == 32 and knn.interval_rule(1e8) == 64
    with pytest.raises(ValueError):
        knn.interval_rule(2e8)


def test_paper_1nn_reproduces_the_interval_rule_between_boundaries():
    """1-NN fitted on all 37 corrected rows predicts the interval rule for every size except
    those lying between the last table size of one interval and the first of the next (there
    the nearest table size can sit on either side of the boundary)."""
    t = _table("table1_opt_subsystem.txt")
    N, corrected = t[:, 0], t[:, 2].astype(int)
    rng = np.random.default_rng(11)
    queries = 10 ** rng.uniform(2, 8, size=400)
    straddle = [(N[i], N[i + 1]) for i in range(len(N) - 1) if corrected[i] != corrected[i + 1]]
    pred = knn.predict(np.log10(N), corrected, np.log10(queries))
    checked = 0
    for q, p in zip(queries, pred):
        if any(lo < q < hi for lo, hi in straddle):
            continue
        assert p == knn.interval_rule(q), q
        checked += 1
    assert checked > 300


def test_paper_split_accuracies_are_reachable():
    """The paper's scores (0.7 with the measured labels, 1.0 with the corrected ones, on a
    shuffled 3:1 split whose training part holds every label) come from one split it does not
    print.  Both occur among such splits (test part: 10 sizes), 1.0 only on a minority of them,
    since a test size next to an interval boundary is often missed."""
    from sklearn.model_selection import train_test_split
    t = _table("table1_opt_subsystem.txt")
    x, raw, corrected = np.log10(t[:, 0]), t[:, 1].astype(int), t[:, 2].astype(int)
    seen = {"raw": [], "corrected": []}
    for seed in range(300):
        tr, te = train_test_split(np.arange(len(x)), test_size=0.25, shuffle=True, random_state=seed)
        assert len(te) == 10
        for name, y in (("raw", raw), ("corrected", corrected)):
            if set(y[tr]) == set(y):
                seen[name].append(float(np.mean(knn.predict(x[tr], y[tr], x[te]) == y[te])))
    r, c = np.array(seen["raw"]), np.array(seen["corrected"])
    assert np.any(np.isclose(r, 0.7)) and np.any(c == 1.0)
    assert 0.0 < np.mean(c == 1.0) < 0.5
    assert c.mean() > r.mean()


def test_mi355x_table_accuracy():
    """Leave-one-out accuracy of the 1-NN rule on the MI355X tile table against the null
    accuracy, per column (the figures the design notes report)."""
    t = _table("mi355x_tile_table.txt")
    assert t.shape == (49, 6)
    x = np.log2(t[:, :2])
    expect = {2: (45, 34), 3: (41, 30), 4: (41, 25), 5: (42, 26)}  # column: (LOO hits, modal count)
    for col, (hits, modal) in expect.items():
        y = t[:, col].astype(int)
        assert knn.loo_accuracy(x, y) == pytest.approx(hits / 49), col
        assert knn.null_accuracy(y) == pytest.approx(modal / 49), col


def test_mi355x_holdout():
    """The rule's purpose, checked on shapes it did not see: fitted on the 4 x 4 sub-grid of
    even powers of four (256, 1024, 4096, 16384), it is scored on the other 33 shapes of the
    table."""
    t = _table("mi355x_tile_table.txt")
    x = np.log2(t[:, :2])
    seen = np.isin(t[:, 0], [256, 1024, 4096, 16384]) & np.isin(t[:, 1], [256, 1024, 4096, 16384])
    assert seen.sum() == 16
    for col, hits in {2: 30, 3: 30, 4: 27, 5: 30}.items():
        y = t[:, col].astype(int)
        pred = knn.predict(x[seen], y[seen], x[~seen])
        assert int(np.sum(pred == y[~seen])) == hits, col


COLUMNS = ((_lib.WF_F32, 0, 2), (_lib.WF_F32, 1, 3), (_lib.WF_F64, 0, 4), (_lib.WF_F64, 1, 5),
           (_lib.WF_I32, 0, 2))  # (dtype, reverse, table column); int32 reads the float32 forward column


def test_library_predictor_equals_oracle_1nn():
    lib = _lib.load()
    t = _table("mi355x_tile_table.txt")
    x = np.log2(t[:, :2])
    rng = np.random.default_rng(3)
    queries = [(int(m), int(n)) for m, n in t[:, :2]]
    queries += [(int(2 ** a), int(2 ** b)) for a, b in rng.uniform(0, 17, size=(300, 2))]
    checked = 0
    for m, n in queries:
        q = np.log2([max(m, 1), max(n, 1)])
        d = np.sort(((x - q) ** 2).sum(axis=1))
        if len(d) > 1 and d[1] - d[0] < 1e-9 and d[0] > 0:
            continue  # equally near two shapes: rounding of log2 may decide either way
        for dtype, rev, col in COLUMNS:
            want = int(knn.predict(x, t[:, col].astype(int), [q])[0])
            assert lib.wf_tile_predict(dtype, max(m, 1), max(n, 1), rev) == want, (m, n, dtype, rev)
        checked += 1
    assert checked > 250


def test_library_predictor_arguments():
    lib = _lib.load()
    assert lib.wf_tile_predict(_lib.WF_F32, 0, 5, 0) == _lib.WF_E_ARG
    assert lib.wf_tile_predict(_lib.WF_F32, 5, 0, 1) == _lib.WF_E_ARG
    assert lib.wf_tile_predict(_lib.WF_F64, 5, 5, 2) == _lib.WF_E_ARG
    assert lib.wf_tile_predict(7, 5, 5, 0) == _lib.WF_E_ARG
    assert lib.wf_tile_predict(_lib.WF_I32, 5, 5, 1) == _lib.WF_E_UNSUPPORTED
    assert lib.wf_tile_predict(_lib.WF_F32, 16384, 16384, 0) == 64
    assert lib.wf_tile_predict(_lib.WF_F32, 16384, 16384, 1) == 32
    assert lib.wf_tile_predict(_lib.WF_F64, 16384, 16384, 1) == 64
    # extreme shapes still land on a row of the table
    for m, n in ((1, 1), (1, 1 << 31), (1 << 40, 1), (1 << 40, 1 << 31)):
        for dtype, rev, _ in COLUMNS:
            assert lib.wf_tile_predict(dtype, m, n, rev) in (16, 32, 64), (m, n, dtype, rev)
    assert lib.wf_tile_predict(_lib.WF_F32, 1, 1, 0) == 64  # nearest: 256 x 256
    assert lib.wf_tile_predict(_lib.WF_F64, 1 << 40, 1, 1) == 16  # nearest: 16384 x 256


def test_python_predict_tile():
    import torch
    import paper_2510_27351_amd as wf
    assert wf.predict_tile(16384, 16384) == 64
    assert wf.predict_tile(16384, 16384, reverse=True) == 32
    assert wf.predict_tile(16384, 16384, reverse=True, dtype=torch.float64) == 64
    assert wf.predict_tile(300, 200, dtype=torch.int32) == 64
    with pytest.raises(wf.WfError):
        wf.predict_tile(0, 5)
    with pytest.raises(wf.WfError):
        wf.predict_tile(5, 5, reverse=True, dtype=torch.int32)
    with pytest.raises(wf.WfError):
        wf.predict_tile(5, 5, dtype=torch.float16)
