"""Host-side logic of the learned policy's training and of the batch autotuner,
on the CPU: weight layout, regret labels, the fit itself, and the sub-batch
the autotuner times."""
import os

import numpy as np
import pytest

import oracle
from paper_2303_04934_amd import _native, policy_train


def test_weight_layout_round_trips_and_matches_the_abi():
    assert policy_train.n_params() == _native.POLICY_FLOATS
    rng = np.random.default_rng(1)
    w = rng.standard_normal(policy_train.n_params()).astype(np.float32)
    assert np.array_equal(policy_train.pack(*policy_train.unpack(w)), w)


def test_training_forward_is_the_oracle_forward():
    rng = np.random.default_rng(2)
    w = rng.standard_normal(policy_train.n_params()).astype(np.float32) * 0.3
    x = rng.standard_normal((17, 5)).astype(np.float32)
    got, _ = policy_train.forward(w, x)
    want = oracle.policy_forward(w, x)
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-5)


def test_shipped_weights_are_complete_and_finite():
    w = np.load(policy_train.WEIGHTS)
    assert w.dtype == np.float32 and w.shape == (policy_train.n_params(),)
    assert np.all(np.isfinite(w))


def test_regret_scores_favour_the_default_class_by_the_margin():
    # graph 0: class 3 is 1% faster than the default class 2 (inside the margin);
    # graph 1: class 0 is 20% faster (outside it)
    times = np.array([[1.10, 1.05, 1.00, 0.99], [0.80, 1.0, 1.0, 1.2]])
    sc = policy_train.scores_for([0, 1, 1], times)
    assert sc.shape == (3, 4)
    assert np.argmax(sc[0]) == policy_train.DEFAULT_CLASS
    assert np.argmax(sc[1]) == 0 and np.array_equal(sc[1], sc[2])
    # the best class of a graph scores 0 before the margin; the default class never loses it
    assert sc[0, policy_train.DEFAULT_CLASS] == pytest.approx(-np.log(1.00 / 0.99), abs=1e-6)
    assert sc[1, 0] == pytest.approx(-policy_train.MARGIN, abs=1e-6)


def test_fit_recovers_a_clear_winner():
    # two kinds of rounds (by frontier size): class 0 wins on the first, class 3 on the second
    rng = np.random.default_rng(3)
    n = 200
    rows = np.zeros((n, 12), np.float32)
    kind = rng.integers(0, 2, n)
    rows[:, 1] = np.where(kind == 0, 0.1, 0.9) + rng.normal(0, 0.01, n)
    rows[:, 2:6] = rng.normal(0, 0.01, (n, 4))
    scores = np.where(kind[:, None] == 0, [0.0, -0.3, -0.3, -0.3], [-0.3, -0.3, -0.3, 0.0]).astype(np.float32)
    w = policy_train.fit(rows, scores, steps=1500, verbose=False)
    out, _ = policy_train.forward(w, rows[:, 1:6])
    pick = np.argmax(out[:, 0::2], axis=1)
    assert np.mean(pick == np.where(kind == 0, 0, 3)) > 0.95


def test_autotune_subset_takes_whole_graphs():
    torch = pytest.importorskip("torch")
    from paper_2303_04934_amd import autotune
    # three graphs with local ids: sizes (n, m) = (2, 1), (3, 3), (1, 0)
    vb = np.array([0, 2, 5, 6])
    ab = np.array([0, 1, 4, 4])
    off = [np.array([0, 1, 1]), np.array([0, 1, 2, 3]), np.array([0, 0])]
    adj = [np.array([1]), np.array([1, 2, 0]), np.array([], np.int64)]
    cat = lambda xs: torch.from_numpy(np.concatenate(xs).astype(np.int32))
    arrays = (cat(off), cat(adj), cat(off), cat(adj))
    vb2, ab2, (oo, oa, io, ia) = autotune._subset(vb, ab, arrays, [0, 2])
    assert list(vb2) == [0, 2, 3] and list(ab2) == [0, 1, 1]
    assert oo.tolist() == [0, 1, 1, 0, 0] and oa.tolist() == [1]
    assert io.tolist() == oo.tolist() and ia.tolist() == oa.tolist()
    vb3, ab3, (oo3, oa3, _, _) = autotune._subset(vb, ab, arrays, [1])
    assert list(vb3) == [0, 3] and list(ab3) == [0, 3]
    assert oo3.tolist() == [0, 1, 2, 3] and oa3.tolist() == [1, 2, 0]


def test_autotune_sample_is_a_strict_subset_and_held_out_is_the_rest():
    import numpy as np

    from paper_2303_04934_amd import autotune
    for G, arcs_each in ((4096, 1000), (4097, 999), (7, 3), (2, 5)):
        vb = np.arange(G + 1, dtype=np.int64) * 10
        ab = np.arange(G + 1, dtype=np.int64) * arcs_each
        for seed in (0, 1, 5):
            idx, rest = autotune.split(vb, ab, seed=seed)
            assert len(idx) >= 1 and len(rest) >= 1, (G, seed)
            assert sorted(idx + rest) == list(range(G))
            assert len(set(idx) & set(rest)) == 0
            # every second graph: the sample keeps about half the batch
            assert abs(len(idx) - G / 2) <= 1


def test_class_and_mode_labels_train_dense_outputs_on_single_source_rows_only():
    import numpy as np

    from paper_2303_04934_amd import policy_train as pt
    rows = np.zeros((3, 12), np.float32)
    rows[:, 0] = [0, 1, 2]  # sparse single-source, dense single-source, multi-source
    times = np.array([[4.0, 3.0, 2.5, 2.0, 2.2, 1.0, 3.0, 3.5]])  # T(c, m), output 2c + m
    sc = pt.scores_for(np.zeros(3, np.int32), times, margin=0.0)
    x, mask, y = pt.dataset(rows, sc)
    assert mask[0].tolist() == [1] * 8 and mask[1].tolist() == [1] * 8
    assert mask[2].tolist() == [1, 0, 1, 0, 1, 0, 1, 0]
    assert np.argmax(y[0]) == 5  # the fastest setting scores 0, the others below
    # the margin lowers every setting but the default (class 2, pull allowed)
    sc2 = pt.scores_for(np.zeros(1, np.int32), times, margin=0.03)
    assert sc2[0, pt.DEFAULT_OUTPUT] == sc[0, pt.DEFAULT_OUTPUT] and sc2[0, 0] < sc[0, 0]


def test_autotune_choice_keeps_default_within_margin():
    from paper_2303_04934_amd import autotune
    assert autotune.choose([100.0, 98.0, 99.0]) == 0            # 2% better: noise, the default stays
    assert autotune.choose([100.0, 98.0, 96.0]) == 2            # 4% better: taken
    assert autotune.choose([100.0, 96.9, 96.0]) == 2            # the fastest of those beyond the margin
    assert autotune.choose([100.0, 120.0], margin=0.0) == 0
    assert autotune.choose([100.0, 99.0], margin=0.0) == 1
