"""Pins for the oracle's per-group feature selection and gather (CPU only).

Section 3 selects, per size group, the top-k opcodes by the normalised
malware-benign occurrence difference; section 4 trains and classifies each
group on those k features.  The pins: the hand-worked example
(tests/golden/select_worked_example.json, exact fractions), brute-force
ranking with exact fractions (a different route from the oracle's integer
cross-products), invariants of a normalised difference, and training on the
gathered columns.  The last test plants mistakes and checks that the pins
reject each one.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import nb, select
from tests import exact_nb

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold():
    with open(os.path.join(GOLD, "select_worked_example.json")) as fh:
        return json.load(fh)


def _fractions_top_k(counts, sums, k):
    """Rank by d_f = |T_1f / S_1 - T_0f / S_0| as exact fractions (phi = 0
    for an empty class), ties to the lower index; ascending output."""
    F = len(counts[0])
    phi = [[Fraction(int(counts[c][f]), int(sums[c])) if int(sums[c]) else Fraction(0)
            for f in range(F)] for c in range(2)]
    d = [abs(phi[1][f] - phi[0][f]) for f in range(F)]
    order = sorted(range(F), key=lambda f: (-d[f], f))
    return sorted(order[:k])


# ------------------------------------------------------------ worked example

@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_worked_example_selection(kind):
    g = _gold()
    ref = g[kind]
    m = nb.train(np.array(g["train_x"]), np.array(g["train_y"]), 2, kind)
    sums = select.class_sums(m.counts, m.Nc, kind)
    assert sums == ref["sums"]
    assert select.selection_keys(m.counts, sums) == ref["keys"]
    # the keys are d_f scaled by S_0 S_1
    for key, d in zip(ref["keys"], ref["d"]):
        assert Fraction(key, sums[0] * sums[1]) == Fraction(d)
    for k, idx in ref["top"].items():
        assert select.top_k(m.counts, sums, int(k)).tolist() == idx
        assert select.select_model_features(m, int(k)).tolist() == idx


@pytest.mark.parametrize("kind,k", [(nb.MULTINOMIAL, 2), (nb.MULTINOMIAL, 1), (nb.BERNOULLI, 2)])
def test_worked_example_k_feature_model(kind, k):
    g = _gold()
    ref = g[kind][f"k{k}_model"]
    m = nb.train(np.array(g["train_x"]), np.array(g["train_y"]), 2, kind)
    idx = select.select_model_features(m, k)
    mk = select.model_on_features(m, idx)
    assert mk.counts.tolist() == ref["counts"]
    np.testing.assert_allclose(np.exp(mk.log_theta), [[float(Fraction(t)) for t in r] for r in ref["theta"]],
                               rtol=1e-14)
    xk = select.gather(np.array([g["test_x"]]), idx)
    s = nb.joint_log_likelihood(mk, xk)[0]
    if "joint" in ref:
        np.testing.assert_allclose(s, [exact_nb.log_fraction(Fraction(j)) for j in ref["joint"]], rtol=1e-13)
    d = nb.decide(s[None, :])
    np.testing.assert_allclose(np.exp(d.log_post[0]), [float(Fraction(p)) for p in ref["posterior"]], rtol=1e-13)
    assert int(d.labels[0]) == ref["label"]


# ------------------------------------------------------------ exact fractions

@st.composite
def count_pair(draw):
    F = draw(st.integers(1, 9))
    hi = draw(st.sampled_from([0, 1, 3, 50, 10 ** 6, 2 ** 31 - 1]))
    cols = [draw(st.lists(st.integers(0, hi), min_size=F, max_size=F)) for _ in range(2)]
    if draw(st.booleans()):                       # force exact ties: repeat a column
        f = draw(st.integers(0, F - 1))
        g = draw(st.integers(0, F - 1))
        for c in range(2):
            cols[c][g] = cols[c][f]
    return np.array(cols, dtype=np.int64)


@settings(max_examples=300, deadline=None)
@given(count_pair())
def test_ranking_matches_exact_fractions(counts):
    sums = select.class_sums(counts)
    F = counts.shape[1]
    for k in range(1, F + 1):
        assert select.top_k(counts, sums, k).tolist() == _fractions_top_k(counts, sums, k)


def test_presence_model_normalises_by_files():
    # presence counts are normalised by the class's file count, not by the
    # sum of presence counts: here the two readings rank differently
    D = np.array([[2, 2], [2, 0]])
    Nc = np.array([2, 2])
    sums = select.class_sums(D, Nc, nb.BERNOULLI)
    assert sums == [2, 2]
    # by files: phi = (1, 1) and (1, 0), d = (0, 1) -> feature 1; by the
    # presence sums it would be (1/2, 1/2) and (1, 0), a tie -> feature 0
    assert select.top_k(D, sums, 1).tolist() == [1]
    assert _fractions_top_k(D, sums, 1) == [1]


def test_empty_class_keys_on_the_other_class():
    counts = np.array([[0, 0, 0, 0], [5, 9, 9, 1]])
    sums = select.class_sums(counts)
    assert sums == [0, 24]
    assert select.top_k(counts, sums, 2).tolist() == [1, 2]
    assert select.top_k(counts, sums, 3).tolist() == [0, 1, 2]
    assert select.top_k(np.zeros((2, 3), np.int64), [0, 0], 2).tolist() == [0, 1]


# ------------------------------------------------------------ invariants

def test_selection_invariants():
    rng = np.random.default_rng(5)
    for trial in range(40):
        F = int(rng.integers(1, 60))
        counts = rng.poisson(rng.gamma(0.5, 2.0, size=(2, F)) * 20).astype(np.int64)
        sums = select.class_sums(counts)
        for k in (1, max(1, F // 3), F):
            idx = select.top_k(counts, sums, k)
            # ascending, unique, in range, of length k
            assert idx.size == k and (np.diff(idx) > 0).all() and idx.min() >= 0 and idx.max() < F
            # swapping the classes keeps the set (an absolute difference)
            assert select.top_k(counts[::-1], sums[::-1], k).tolist() == idx.tolist()
            # scaling one class's counts by an integer keeps the set (normalised)
            sc = counts.copy()
            sc[1] *= 7
            assert select.top_k(sc, select.class_sums(sc), k).tolist() == idx.tolist()
            # every selected feature scores at least every unselected one
            key = select.selection_keys(counts, sums)
            rest = np.setdiff1d(np.arange(F), idx)
            if rest.size:
                assert min(key[f] for f in idx) >= max(key[f] for f in rest)
        assert select.top_k(counts, sums, F).tolist() == list(range(F))


def test_argument_errors():
    c = np.array([[1, 2], [3, 4]])
    with pytest.raises(ValueError):
        select.top_k(c, [3, 7], 0)
    with pytest.raises(ValueError):
        select.top_k(c, [3, 7], 3)
    with pytest.raises(ValueError):
        select.top_k(np.ones((3, 2), np.int64), [2, 2, 2], 1)
    with pytest.raises(ValueError):
        select.gather(np.ones((2, 2)), [0, 2])


# ------------------------------------------------------------ gathered training

@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_model_on_features_is_training_on_gathered_columns(kind):
    rng = np.random.default_rng(17)
    X = rng.poisson(rng.gamma(0.5, 2.0, size=60), size=(300, 60)).astype(np.uint8)
    X[rng.random(X.shape) < 0.7] = 0
    y = np.arange(300) % 2
    m = nb.train(X, y, 2, kind)
    for k in (1, 7, 60):
        idx = select.select_model_features(m, k)
        mk = select.model_on_features(m, idx)
        ref = nb.train(select.gather(X, idx), y, 2, kind)
        assert (mk.counts == ref.counts).all() and (mk.Nc == ref.Nc).all()
        np.testing.assert_array_equal(mk.log_theta, ref.log_theta)
        np.testing.assert_array_equal(mk.log_prior, ref.log_prior)
        if kind == nb.BERNOULLI:
            np.testing.assert_array_equal(mk.log_1m_theta, ref.log_1m_theta)
        # and against exact rationals on a few files
        ex = exact_nb.exact_model(select.gather(X, idx).tolist(), y.tolist(), 2, kind)
        for j in range(3):
            xj = select.gather(X[j:j + 1], idx)
            post = np.exp(nb.decide(nb.joint_log_likelihood(mk, xj)).log_post[0])
            want = [float(p) for p in exact_nb.exact_posterior(ex, xj[0].tolist())]
            np.testing.assert_allclose(post, want, rtol=1e-9)


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_expanded_model_scores_full_rows_as_the_k_model_scores_gathered_rows(kind):
    rng = np.random.default_rng(23)
    F = 50
    X = rng.poisson(rng.gamma(0.5, 2.0, size=F), size=(200, F)).astype(np.uint8)
    X[rng.random(X.shape) < 0.6] = 0
    y = np.arange(200) % 2
    m = nb.train(X, y, 2, kind)
    for k in (1, 9, F):
        idx = select.select_model_features(m, k)
        mk = select.model_on_features(m, idx)
        me = select.expanded_model(mk, idx, F)
        assert me.n_features == F and (me.Nc == mk.Nc).all()
        Xt = rng.poisson(1.5, size=(40, F)).astype(np.uint8)
        want = nb.joint_log_likelihood(mk, select.gather(Xt, idx))
        np.testing.assert_allclose(nb.joint_log_likelihood(me, Xt), want, rtol=1e-13, atol=1e-12)
        # the unselected columns do not matter
        rest = np.setdiff1d(np.arange(F), idx)
        Xr = Xt.copy()
        Xr[:, rest] = rng.integers(0, 200, size=(40, rest.size))
        np.testing.assert_allclose(nb.joint_log_likelihood(me, Xr), want, rtol=1e-13, atol=1e-12)
    with pytest.raises(ValueError):
        select.expanded_model(mk, idx[::-1], F)


def test_gather_is_column_selection():
    X = np.arange(24).reshape(4, 6)
    assert select.gather(X, [5, 0, 3]).tolist() == [[r[5], r[0], r[3]] for r in X.tolist()]


# ------------------------------------------------------------ planted mistakes

def _pins_fail():
    checks = [
        lambda: test_worked_example_selection(nb.MULTINOMIAL),
        lambda: test_worked_example_selection(nb.BERNOULLI),
        lambda: test_worked_example_k_feature_model(nb.MULTINOMIAL, 2),
        lambda: test_worked_example_k_feature_model(nb.BERNOULLI, 2),
        lambda: test_model_on_features_is_training_on_gathered_columns(nb.MULTINOMIAL),
        lambda: test_expanded_model_scores_full_rows_as_the_k_model_scores_gathered_rows(nb.BERNOULLI),
        test_presence_model_normalises_by_files,
        test_empty_class_keys_on_the_other_class,
        test_selection_invariants,
        test_ranking_matches_exact_fractions,
    ]
    failed = 0
    for chk in checks:
        try:
            chk()
        except Exception:
            failed += 1
    return failed


_orig_keys = select.selection_keys
_orig_top_k = select.top_k
_orig_sums = select.class_sums
_orig_model = select.model_on_features
_orig_expanded = select.expanded_model


def _unnormalised_keys(counts, sums):
    return [abs(int(counts[1, f]) - int(counts[0, f])) for f in range(counts.shape[1])]


def _signed_keys(counts, sums):
    return [int(counts[1, f]) * int(sums[0]) - int(counts[0, f]) * int(sums[1]) for f in range(counts.shape[1])]


def _swapped_normaliser(counts, sums):
    return [abs(int(counts[1, f]) * int(sums[1]) - int(counts[0, f]) * int(sums[0])) for f in range(counts.shape[1])]


def _ties_to_higher(counts, sums, k):
    keys = select.selection_keys(counts, sums)
    F = counts.shape[1]
    order = sorted(range(F), key=lambda f: (-keys[f], -f))
    return np.array(sorted(order[:k]), dtype=np.int32)


def _rank_order_output(counts, sums, k):
    keys = select.selection_keys(counts, sums)
    order = sorted(range(counts.shape[1]), key=lambda f: (-keys[f], f))
    return np.array(order[:k], dtype=np.int32)


def _presence_by_sum(counts, Nc=None, kind=nb.MULTINOMIAL):
    return _orig_sums(counts, None, nb.MULTINOMIAL)


def _full_normaliser_kept(m, idx):
    # keep the full model's S_c instead of the selected columns' sum
    idx = np.asarray(idx, dtype=np.int64)
    mk = _orig_model(m, idx)
    if m.kind == nb.MULTINOMIAL:
        T = np.asarray(mk.counts, dtype=np.float64)
        S = np.asarray(m.counts, dtype=np.float64).sum(axis=1, keepdims=True)
        mk.log_theta = np.log(T + m.alpha) - np.log(S + m.alpha * T.shape[1])
    return mk


def _expanded_one_off(mk, idx, F):
    # tables written one feature to the right of their own column
    return _orig_expanded(mk, np.minimum(np.asarray(idx) + 1, F - 1) if idx[-1] < F - 1 else idx, F)


def _expanded_unselected_presence_kept(mk, idx, F):
    # the presence model's log(1 - theta) left at log 1/2 outside the selection
    me = _orig_expanded(mk, idx, F)
    if me.log_1m_theta is not None:
        rest = np.setdiff1d(np.arange(F), np.asarray(idx))
        me.log_1m_theta[:, rest] = np.log(0.5)
    return me


SELECT_MUTATIONS = {
    "difference not normalised": ("selection_keys", _unnormalised_keys),
    "signed difference": ("selection_keys", _signed_keys),
    "normalisers swapped": ("selection_keys", _swapped_normaliser),
    "ties go to the higher index": ("top_k", _ties_to_higher),
    "list in rank order, not feature order": ("top_k", _rank_order_output),
    "presence normalised by presence sum": ("class_sums", _presence_by_sum),
    "k-feature model keeps the full normaliser": ("model_on_features", _full_normaliser_kept),
    "expanded tables one column off": ("expanded_model", _expanded_one_off),
    "expanded presence model scores unselected absences": ("expanded_model", _expanded_unselected_presence_kept),
}


def test_unmutated_selection_passes_all_pins():
    assert _pins_fail() == 0


@pytest.mark.parametrize("name", sorted(SELECT_MUTATIONS))
def test_planted_selection_mistake_is_caught(name, monkeypatch):
    attr, fn = SELECT_MUTATIONS[name]
    monkeypatch.setattr(select, attr, fn)
    assert _pins_fail() > 0, name
