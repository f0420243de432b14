"""Host-side planner logic on hand-made label records (no GPU): the generator's parameter
ranges, label loading (torn lines skipped, seed filter, seed order), the robust training
label among near-ties and the best single class."""
import json
import math

import numpy as np

from paper_2407_00829_amd import planner


def test_matrix_params_cover_the_stated_range():
    ns, rls = [], []
    for s in range(400):
        n, rl, pi = planner.matrix_params(s)
        ns.append(n)
        rls.append(rl)
        assert 1e4 <= n <= 1e6 and 4 <= rl <= 64
        assert abs(pi.sum() - 1.0) < 1e-12 and (pi >= 0).all()
    # log-uniform n: about half of the draws below the geometric midpoint 1e5
    assert 0.35 < np.mean(np.array(ns) < 1e5) < 0.65
    assert 0.35 < np.mean(np.array(rls) < 34) < 0.65
    a, b = planner.matrix_params(7), planner.matrix_params(7)  # seeded: the same matrix again
    assert a[:2] == b[:2] and np.array_equal(a[2], b[2])


def test_class_names_cover_lists_and_deltas():
    names = [planner.class_name(c) for c in range(planner.NCLASS)]
    assert len(set(names)) == planner.NCLASS
    assert names[0] == "CSR@0.5" and names[8] == "VBR+CSR@0.9" and names[14] == "VBR+VDIA+CSR@0.9"


def test_load_labels_skips_torn_lines_and_filters(tmp_path):
    p = tmp_path / "l.jsonl"
    recs = [{"seed": s, "times": [1.0] * planner.NCLASS} for s in (5, 2, 9)]
    p.write_text("\n".join(json.dumps(r) for r in recs) + "\n{\"seed\": 11, \"tim")
    got = planner.load_labels(str(p))
    assert [r["seed"] for r in got] == [2, 5, 9]
    assert [r["seed"] for r in planner.load_labels(str(p), {9, 2})] == [2, 9]


def _recs(rows):
    return [{"seed": i, "times": list(map(float, t))} for i, t in enumerate(rows)]


def test_robust_labels_pick_the_steadiest_class_among_near_ties():
    base = [10.0] * planner.NCLASS
    rows = []
    # class 3 is the fastest on every matrix by 1% or more, class 0 close behind on the first two
    for k in range(4):
        t = list(base)
        t[3] = 5.0
        t[0] = 5.05 if k < 2 else 9.0
        rows.append(t)
    recs = _recs(rows)
    # no tolerance: the argmin
    assert list(planner.robust_labels(recs, 0.0)) == [3, 3, 3, 3]
    # 2% tolerance: on the first two class 0 is within it, but class 3 has the lower mean regret
    assert list(planner.robust_labels(recs, 0.02)) == [3, 3, 3, 3]
    # make class 0 the steadier one: on the last two class 3 is far off
    rows[2][3] = rows[3][3] = 20.0
    rows[2][0] = rows[3][0] = 5.0
    recs = _recs(rows)
    assert list(planner.robust_labels(recs, 0.02)) == [0, 0, 0, 0]
    assert list(planner.robust_labels(recs, 0.0)) == [3, 3, 0, 0]


def test_best_constant_class_minimises_mean_regret():
    rng = np.random.default_rng(1)
    T = rng.uniform(1.0, 2.0, (50, planner.NCLASS))
    T[:, 6] = T.min(axis=1) * 1.01  # always within 1% of the fastest
    recs = _recs(T)
    assert planner.best_constant_class(recs) == 6
    R = T / T.min(axis=1, keepdims=True) - 1.0
    assert math.isclose(R[:, 6].mean(), R.mean(axis=0).min())
