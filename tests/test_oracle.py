"""Pins for the FP64 oracle (CPU only).

Each pin ties the oracle to something other than itself: the hand-worked
example (tests/golden/worked_example.json), exact rationals, scikit-learn's
Naive Bayes, closed forms and invariants of the method, and brute-force
counting.  tests/test_oracle_mutations.py plants mistakes in the oracle and
checks that these pins catch every one.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import nb, groups
from tests import exact_nb

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def _fr(s):
    return Fraction(s)


# ---------------------------------------------------------------- worked example

@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_worked_example(kind):
    g = _load("worked_example.json")
    X = np.array(g["train_x"])
    y = np.array(g["train_y"])
    m = nb.train(X, y, g["n_classes"], kind, alpha=g["alpha"])
    ref = g[kind]
    assert m.Nc.tolist() == g["class_totals"]
    assert m.counts.tolist() == ref["counts"]
    np.testing.assert_allclose(np.exp(m.log_prior), [float(_fr(p)) for p in g["prior"]], rtol=1e-14)
    np.testing.assert_allclose(np.exp(m.log_theta), [[float(_fr(t)) for t in r] for r in ref["theta"]],
                               rtol=1e-14)
    s = nb.joint_log_likelihood(m, np.array([g["test_x"]]))[0]
    np.testing.assert_allclose(s, [exact_nb.log_fraction(_fr(j)) for j in ref["joint"]], rtol=1e-13)
    d = nb.decide(s[None, :])
    np.testing.assert_allclose(np.exp(d.log_post[0]), [float(_fr(p)) for p in ref["posterior"]], rtol=1e-13)
    assert int(d.labels[0]) == ref["label"]


# ---------------------------------------------------------------- exact rationals

@st.composite
def tiny_problem(draw):
    C = draw(st.integers(2, 3))
    F = draw(st.integers(1, 4))
    per = [draw(st.integers(1, 3)) for _ in range(C)]
    y = [c for c in range(C) for _ in range(per[c])]
    X = [[draw(st.integers(0, 3)) for _ in range(F)] for _ in y]
    tests = [[draw(st.integers(0, 3)) for _ in range(F)] for _ in range(3)]
    return C, X, y, tests


@settings(max_examples=150, deadline=None)
@given(tiny_problem(), st.sampled_from([nb.MULTINOMIAL, nb.BERNOULLI]))
def test_exact_rational_posteriors(prob, kind):
    C, X, y, tests = prob
    ex = exact_nb.exact_model(X, y, C, kind)
    m = nb.train(np.array(X), np.array(y), C, kind)
    assert m.Nc.tolist() == ex["Nc"]
    assert m.counts.tolist() == ex["counts"]
    np.testing.assert_allclose(np.exp(m.log_theta), [[float(t) for t in r] for r in ex["theta"]], rtol=1e-14)
    s = nb.joint_log_likelihood(m, np.array(tests))
    d = nb.decide(s)
    for j, x in enumerate(tests):
        joint = exact_nb.exact_joint(ex, x)
        np.testing.assert_allclose(s[j], [exact_nb.log_fraction(v) for v in joint], rtol=1e-12, atol=1e-12)
        post = exact_nb.exact_posterior(ex, x)
        np.testing.assert_allclose(np.exp(d.log_post[j]), [float(p) for p in post], rtol=1e-12, atol=1e-15)
        if d.margin[j] > 1e-9:   # float ties are decided by the exact check below
            assert int(d.labels[j]) == exact_nb.exact_label(ex, x)


# ---------------------------------------------------------------- library cross-check

@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_sklearn_cross_check(kind):
    from sklearn.naive_bayes import BernoulliNB, MultinomialNB
    rng = np.random.default_rng(7)
    C, F = 3, 12
    y = rng.integers(0, C, 300)
    X = rng.poisson(rng.gamma(0.5, 2.0, size=(C, F))[y])
    Xt = rng.poisson(1.0, size=(50, F))
    sk = (MultinomialNB(alpha=1.0) if kind == nb.MULTINOMIAL else BernoulliNB(alpha=1.0, binarize=0.0))
    sk.fit(X, y)
    m = nb.train(X, y, C, kind)
    np.testing.assert_allclose(m.log_prior, sk.class_log_prior_, rtol=1e-13)
    np.testing.assert_allclose(m.log_theta, sk.feature_log_prob_, rtol=1e-13)
    s = nb.joint_log_likelihood(m, Xt)
    np.testing.assert_allclose(s, sk.predict_joint_log_proba(Xt), rtol=1e-12)
    d = nb.decide(s)
    np.testing.assert_allclose(np.exp(d.log_post), sk.predict_proba(Xt), rtol=1e-10, atol=1e-14)
    assert (d.labels == sk.predict(Xt)).all()


# ---------------------------------------------------------------- counts by brute force

def test_counts_brute_force_and_invariants():
    rng = np.random.default_rng(3)
    C, F, N = 4, 7, 97
    y = rng.integers(0, C, N)
    X = rng.poisson(2.0, size=(N, F)) * (rng.random((N, F)) > 0.5)
    T = nb.feature_counts(X, y, C, nb.MULTINOMIAL)
    D = nb.feature_counts(X, y, C, nb.BERNOULLI)
    Nc = nb.class_totals(y, C)
    Tb = np.zeros((C, F), dtype=np.int64)
    Db = np.zeros((C, F), dtype=np.int64)
    tok = np.zeros(C, dtype=np.int64)
    for i in range(N):
        for f in range(F):
            Tb[y[i], f] += X[i, f]
            Db[y[i], f] += X[i, f] > 0
            tok[y[i]] += X[i, f]
    assert (T == Tb).all() and (D == Db).all()
    assert (T.sum(axis=1) == tok).all()
    assert (T.sum(axis=0) == X.sum(axis=0)).all()
    assert Nc.sum() == N and (Nc == np.bincount(y, minlength=C)).all()
    assert (D <= Nc[:, None]).all() and (D <= T).all()


def test_bad_inputs_rejected():
    with pytest.raises(ValueError):
        nb.class_totals([0, 2], 2)
    with pytest.raises(ValueError):
        nb.feature_counts(np.array([[-1, 0]]), [0], 2)
    with pytest.raises(ValueError):
        nb.train(np.ones((2, 2)), [0, 1], 2, alpha=0.0)


# ---------------------------------------------------------------- invariants

def _problem(seed=11, C=3, F=20, N=400, n=64):
    rng = np.random.default_rng(seed)
    lam = rng.gamma(0.5, 2.0, size=(C, F))
    y = np.arange(N) % C
    X = rng.poisson(lam[y])
    Xt = rng.poisson(lam[np.arange(n) % C])
    return C, X, y, Xt


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_posteriors_normalised(kind):
    C, X, y, Xt = _problem()
    d = nb.classify(nb.train(X, y, C, kind), Xt)
    lse = np.log(np.exp(d.log_post).sum(axis=1))
    np.testing.assert_allclose(lse, 0.0, atol=1e-13)


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_feature_permutation_invariance(kind):
    C, X, y, Xt = _problem()
    p = np.random.default_rng(5).permutation(X.shape[1])
    s1 = nb.joint_log_likelihood(nb.train(X, y, C, kind), Xt)
    s2 = nb.joint_log_likelihood(nb.train(X[:, p], y, C, kind), Xt[:, p])
    np.testing.assert_allclose(s1, s2, rtol=1e-12)


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_class_relabel_equivariance(kind):
    C, X, y, Xt = _problem()
    perm = np.array([2, 0, 1])          # old class c becomes perm[c]
    s1 = nb.joint_log_likelihood(nb.train(X, y, C, kind), Xt)
    s2 = nb.joint_log_likelihood(nb.train(X, perm[y], C, kind), Xt)
    np.testing.assert_allclose(s2[:, perm], s1, rtol=1e-12)


def test_zero_file_posterior_is_prior():
    C, X, y, _ = _problem()
    y = np.where(np.arange(len(y)) % 5 == 0, 0, y)      # unbalance the classes
    m = nb.train(X, y, C, nb.MULTINOMIAL)
    d = nb.classify(m, np.zeros((1, X.shape[1]), dtype=np.int64))
    np.testing.assert_allclose(np.exp(d.log_post[0]), m.Nc / m.Nc.sum(), rtol=1e-13)


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_two_class_logistic_form(kind):
    C, X, y, Xt = _problem(C=2)
    m = nb.train(X, y, 2, kind)
    d = nb.classify(m, Xt)
    g = Xt if kind == nb.MULTINOMIAL else (Xt > 0).astype(np.float64)
    if kind == nb.MULTINOMIAL:
        logit = g @ (m.log_theta[1] - m.log_theta[0]) + m.log_prior[1] - m.log_prior[0]
    else:
        w = (m.log_theta - m.log_1m_theta)
        b = m.log_prior + m.log_1m_theta.sum(axis=1)
        logit = g @ (w[1] - w[0]) + b[1] - b[0]
    np.testing.assert_allclose(d.log_post[:, 1], -np.logaddexp(0.0, -logit), rtol=1e-11, atol=1e-13)


def test_bernoulli_weight_form_equals_textbook_form():
    C, X, y, Xt = _problem()
    m = nb.train(X, y, C, nb.BERNOULLI)
    W, b = nb.weight_form(m)
    np.testing.assert_allclose((Xt > 0) @ W.T + b, nb.joint_log_likelihood(m, Xt), rtol=1e-12)


def test_batch_composition_invariance():
    C, X, y, Xt = _problem()
    m = nb.train(X, y, C, nb.MULTINOMIAL)
    whole = nb.joint_log_likelihood(m, Xt)
    one = np.vstack([nb.joint_log_likelihood(m, Xt[j:j + 1]) for j in range(Xt.shape[0])])
    np.testing.assert_allclose(whole, one, rtol=1e-13)


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_symmetric_training_ties_go_to_benign(kind):
    rng = np.random.default_rng(2)
    half = rng.poisson(1.5, size=(30, 6))
    X = np.vstack([half, half])
    y = np.array([0] * 30 + [1] * 30)
    d = nb.classify(nb.train(X, y, 2, kind), rng.poisson(1.5, size=(40, 6)))
    assert (d.margin == 0).all()
    assert (d.labels == 0).all()


# ---------------------------------------------------------------- size groups

def test_group_fixture_routing():
    g = _load("size_groups.json")
    G = g["n_groups"]
    cc = np.full((G, 2), 50, dtype=np.int64)
    for k, grp in enumerate(g["untrained_1based"]):
        cc[grp - 1, k % 2] = g["min_files"] - 1
    cc[3, 0] = g["min_files"]           # exactly at the threshold is trained
    trained = groups.trained_mask(cc, g["min_files"])
    assert trained.sum() == G - len(g["untrained_1based"])
    r = groups.route(trained)
    for grp in range(1, G + 1):
        want = g["fallback_1based"].get(str(grp), grp)
        assert r[grp - 1] + 1 == want


def test_group_routing_edge_cases():
    assert groups.route([True]).tolist() == [0]
    assert groups.route([False, False, True]).tolist() == [2, 2, 2]
    assert groups.route([True, False, False]).tolist() == [0, 0, 0]
    with pytest.raises(ValueError):
        groups.route([False, False])
