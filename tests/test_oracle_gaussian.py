"""Pins for the oracle's Gaussian Naive Bayes variant (CPU only).

The paper does not name its Naive Bayes variant (section 4); the Gaussian
form over the occurrence counts is the third classical one.  Pins: the
hand-worked example (tests/golden/gaussian_worked_example.json, exact
fractions), scikit-learn's GaussianNB (run, not copied), the expanded
weight form against the textbook density, invariants of a Gaussian model,
and planted mistakes that the pins must reject."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import nb

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold():
    with open(os.path.join(GOLD, "gaussian_worked_example.json")) as fh:
        return json.load(fh)


def _fr(v):
    return Fraction(v)


def test_worked_example():
    g = _gold()
    X, y = np.array(g["train_x"]), np.array(g["train_y"])
    m = nb.train(X, y, 2, nb.GAUSSIAN)
    assert m.counts.tolist() == g["sums"] and m.sq.tolist() == g["square_sums"]
    eps = _fr(g["epsilon"])
    assert m.eps == pytest.approx(float(eps), rel=1e-15)
    assert float(max(_fr(v) for v in g["pooled_variance"])) * 1e-9 == pytest.approx(m.eps, rel=1e-15)
    for c in range(2):
        for f in range(3):
            assert m.mean[c, f] == float(_fr(g["mean"][c][f]))
            assert m.var[c, f] == pytest.approx(float(_fr(g["variance"][c][f]) + eps), rel=1e-15)
    # the joint log-likelihood of the test file from the exact moments
    x = g["test_x"]
    s = nb.joint_log_likelihood(m, np.array([x]))[0]
    prior = [Fraction(2, 5), Fraction(3, 5)]
    for c in range(2):
        v = [_fr(g["variance"][c][f]) + eps for f in range(3)]
        mu = [_fr(g["mean"][c][f]) for f in range(3)]
        want = math.log(prior[c]) - 0.5 * sum(math.log(2 * math.pi * float(vf)) for vf in v) \
            - 0.5 * sum(float((x[f] - mu[f]) ** 2 / v[f]) for f in range(3))
        assert s[c] == pytest.approx(want, rel=1e-13)
        # without the (tiny) floor the quadratic terms are the hand-worked ones
        q = [(x[f] - mu[f]) ** 2 / _fr(g["variance"][c][f]) for f in range(3)]
        assert [str(v) for v in q] == g["squared_deviation_over_variance_without_epsilon"][c]
    assert int(nb.decide(s[None, :]).labels[0]) == g["label"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sklearn_cross_check(seed):
    from sklearn.naive_bayes import GaussianNB
    rng = np.random.default_rng(seed)
    C = 2 + seed
    X = rng.poisson(rng.gamma(0.5, 2.0, size=30) * 3, size=(400, 30))
    X[rng.random(X.shape) < 0.6] = 0
    X[:, 3] = 7                                   # a constant feature: variance = epsilon
    y = np.arange(400) % C
    m = nb.train(X, y, C, nb.GAUSSIAN)
    ref = GaussianNB(var_smoothing=nb.VAR_SMOOTHING).fit(X, y)
    np.testing.assert_allclose(m.mean, ref.theta_, rtol=1e-14, atol=0)
    np.testing.assert_allclose(m.var, ref.var_, rtol=1e-9)
    assert m.eps == pytest.approx(ref.epsilon_, rel=1e-12)
    np.testing.assert_allclose(np.exp(m.log_prior), ref.class_prior_, rtol=1e-14)
    Xt = rng.poisson(2.0, size=(60, 30))
    np.testing.assert_allclose(nb.joint_log_likelihood(m, Xt), ref.predict_joint_log_proba(Xt), rtol=1e-9)
    d = nb.decide(nb.joint_log_likelihood(m, Xt))
    np.testing.assert_allclose(np.exp(d.log_post), ref.predict_proba(Xt), atol=1e-9)
    assert (d.labels == ref.predict(Xt)).all()


def test_weight_form_is_the_density():
    rng = np.random.default_rng(4)
    X = rng.poisson(3.0, size=(200, 12))
    y = np.arange(200) % 3
    m = nb.train(X, y, 3, nb.GAUSSIAN)
    Xt = rng.poisson(3.0, size=(40, 12)).astype(np.float64)
    W, b = nb.weight_form(m)
    s = np.concatenate([Xt, Xt * Xt], axis=1) @ W.T + b
    ref = nb.joint_log_likelihood(m, Xt)
    assert np.abs(s - ref).max() <= 1e-10 * np.abs(ref).max()


def test_score_form_is_the_expanded_form():
    # the density's own form and the expanded linear form agree
    rng = np.random.default_rng(8)
    X = rng.poisson(3.0, size=(200, 10))
    y = np.arange(200) % 2
    m = nb.train(X, y, 2, nb.GAUSSIAN)
    mean, h, bias = nb.gaussian_score_form(m)
    Xt = rng.poisson(3.0, size=(30, 10)).astype(np.float64)
    s = np.stack([bias[c] + (h[c][None, :] * (Xt - mean[c][None, :]) ** 2).sum(axis=1) for c in range(2)], axis=1)
    W, b = nb.weight_form(m)
    s2 = np.concatenate([Xt, Xt * Xt], axis=1) @ W.T + b
    assert np.abs(s - s2).max() <= 1e-10 * np.abs(s).max()
    assert (h < 0).all()


def test_invariants():
    rng = np.random.default_rng(6)
    X = rng.poisson(2.5, size=(300, 16)).astype(np.int64)
    y = (np.arange(300) % 2)
    Xt = rng.poisson(2.5, size=(50, 16)).astype(np.int64)
    m = nb.train(X, y, 2, nb.GAUSSIAN)
    d = nb.classify(m, Xt)
    np.testing.assert_allclose(np.exp(d.log_post).sum(axis=1), 1.0, rtol=1e-12)
    # translating a feature in training and test files moves only its means
    sh = np.zeros(16, dtype=np.int64)
    sh[5] = 40
    m2 = nb.train(X + sh, y, 2, nb.GAUSSIAN)
    np.testing.assert_allclose(m2.var, m.var, rtol=1e-12)
    np.testing.assert_allclose(nb.classify(m2, Xt + sh).log_post, d.log_post, atol=1e-9)
    # relabelling the classes permutes the scores
    m3 = nb.train(X, 1 - y, 2, nb.GAUSSIAN)
    np.testing.assert_allclose(nb.joint_log_likelihood(m3, Xt), nb.joint_log_likelihood(m, Xt)[:, ::-1],
                               rtol=1e-12)
    # a feature constant within a class has variance epsilon there
    X4 = X.copy()
    X4[y == 0, 2] = 3
    m4 = nb.train(X4, y, 2, nb.GAUSSIAN)
    assert m4.var[0, 2] == m4.eps and m4.eps > 0


# ------------------------------------------------------------ planted mistakes

def _pins_fail():
    checks = [test_worked_example, lambda: test_sklearn_cross_check(0), lambda: test_sklearn_cross_check(2),
              test_weight_form_is_the_density, test_score_form_is_the_expanded_form, test_invariants]
    failed = 0
    for chk in checks:
        try:
            chk()
        except Exception:
            failed += 1
    return failed


_orig_moments = nb.gaussian_moments
_orig_form = nb.weight_form


def _sample_variance(T, Q, Nc, var_smoothing=nb.VAR_SMOOTHING):
    mean, var, eps = _orig_moments(T, Q, Nc, var_smoothing)
    n = np.asarray(Nc, dtype=np.float64)[:, None]
    return mean, (var - eps) * n / np.maximum(n - 1, 1) + eps, eps


def _no_floor(T, Q, Nc, var_smoothing=nb.VAR_SMOOTHING):
    mean, var, eps = _orig_moments(T, Q, Nc, var_smoothing)
    return mean, var - eps, 0.0


def _floor_from_class_variances(T, Q, Nc, var_smoothing=nb.VAR_SMOOTHING):
    mean, var, eps = _orig_moments(T, Q, Nc, var_smoothing)
    e2 = var_smoothing * float((var - eps).max())
    return mean, var - eps + e2, e2


def _bias_without_mean_term(m):
    W, b = _orig_form(m)
    if m.kind == nb.GAUSSIAN:
        b = b + 0.5 * (m.mean * m.mean / m.var).sum(axis=1)
    return W, b


def _quadratic_sign(m):
    W, b = _orig_form(m)
    if m.kind == nb.GAUSSIAN:
        F = m.n_features
        W = W.copy()
        W[:, F:] = -W[:, F:]
    return W, b


_orig_sform = nb.gaussian_score_form


def _score_form_without_two_pi(m):
    mean, h, bias = _orig_sform(m)
    return mean, h, bias + 0.5 * m.n_features * np.log(2.0 * np.pi)


def _score_form_full_inverse(m):
    mean, h, bias = _orig_sform(m)
    return mean, 2.0 * h, bias


GAUSS_MUTATIONS = {
    "score form drops 2 pi": ("gaussian_score_form", _score_form_without_two_pi),
    "score form without the 1/2": ("gaussian_score_form", _score_form_full_inverse),
    "sample (n - 1) variance": ("gaussian_moments", _sample_variance),
    "no variance floor": ("gaussian_moments", _no_floor),
    "floor from class variances": ("gaussian_moments", _floor_from_class_variances),
    "weight form bias drops mean^2 / var": ("weight_form", _bias_without_mean_term),
    "weight form quadratic sign": ("weight_form", _quadratic_sign),
}


def test_unmutated_gaussian_passes_all_pins():
    assert _pins_fail() == 0


@pytest.mark.parametrize("name", sorted(GAUSS_MUTATIONS))
def test_planted_gaussian_mistake_is_caught(name, monkeypatch):
    attr, fn = GAUSS_MUTATIONS[name]
    monkeypatch.setattr(nb, attr, fn)
    assert _pins_fail() > 0, name
