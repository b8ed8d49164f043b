"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
of test_oracle.py reject every one of them.  A pin set that let a dropped
term, a wrong sign or a swapped index through would not pin anything."""
import numpy as np
import pytest

from oracle import nb
from tests import test_oracle as pins


def _pins_fail():
    checks = [
        lambda: pins.test_worked_example(nb.MULTINOMIAL),
        lambda: pins.test_worked_example(nb.BERNOULLI),
        lambda: pins.test_sklearn_cross_check(nb.MULTINOMIAL),
        lambda: pins.test_sklearn_cross_check(nb.BERNOULLI),
        pins.test_counts_brute_force_and_invariants,
        lambda: pins.test_symmetric_training_ties_go_to_benign(nb.MULTINOMIAL),
        lambda: pins.test_posteriors_normalised(nb.MULTINOMIAL),
        pins.test_zero_file_posterior_is_prior,
    ]
    failed = 0
    for chk in checks:
        try:
            chk()
        except Exception:
            failed += 1
    return failed


def _no_smoothing_mass(T, alpha):
    T = np.asarray(T, dtype=np.float64)
    return np.log(T + alpha) - np.log(T.sum(axis=1, keepdims=True))


def _transposed_total(T, alpha):
    T = np.asarray(T, dtype=np.float64)
    return np.log(T + alpha) - np.log(T.sum() / T.shape[0] + alpha * T.shape[1])


def _complement_unsmoothed(D, Nc, alpha):
    D = np.asarray(D, dtype=np.float64)
    N = np.asarray(Nc, dtype=np.float64)[:, None]
    den = np.log(N + 2 * alpha)
    with np.errstate(divide="ignore"):
        return np.log(D + alpha) - den, np.log(N - D) - den


def _uniform_prior(Nc):
    Nc = np.asarray(Nc, dtype=np.float64)
    return np.full(Nc.size, -np.log(Nc.size))


def _last_index_ties(s):
    s = np.asarray(s, dtype=np.float64)
    d = _orig_decide(s)
    d.labels = s.shape[1] - 1 - np.argmax(s[:, ::-1], axis=1)
    return d


def _no_normaliser(s):
    d = _orig_decide(s)
    d.log_post = np.asarray(s) - np.asarray(s).max(axis=1, keepdims=True)
    return d


def _bernoulli_counts_occurrences(X, y, C, kind=nb.MULTINOMIAL):
    return _orig_counts(X, y, C, nb.MULTINOMIAL)


def _shifted_class(X, y, C, kind=nb.MULTINOMIAL):
    return _orig_counts(X, (np.asarray(y) + 1) % C, C, kind)


_orig_decide = nb.decide
_orig_counts = nb.feature_counts

MUTATIONS = {
    "multinomial denominator drops alpha*F": ("multinomial_log_theta", _no_smoothing_mass),
    "multinomial total over the wrong axis": ("multinomial_log_theta", _transposed_total),
    "bernoulli complement loses smoothing": ("bernoulli_log_theta", _complement_unsmoothed),
    "class prior dropped": ("log_prior", _uniform_prior),
    "ties go to the highest class": ("decide", _last_index_ties),
    "posterior not normalised": ("decide", _no_normaliser),
    "presence counted as occurrences": ("feature_counts", _bernoulli_counts_occurrences),
    "counts credited to the wrong class": ("feature_counts", _shifted_class),
}


def test_unmutated_oracle_passes_all_pins():
    assert _pins_fail() == 0


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(nb, attr, fn)
    assert _pins_fail() > 0, name
