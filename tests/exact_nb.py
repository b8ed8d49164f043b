"""Exact-rational Naive Bayes on tiny inputs (test-side pin for the oracle).

Computes posteriors as exact ratios prior * prod_f P(a_f | c) / sum over
classes with fractions.Fraction, from plain Python loops: a different route
from the oracle's float64 log-space sums, so a dropped term, a wrong sign or a
transposed index in either shows up as a mismatch.
"""
from fractions import Fraction
import math


def exact_model(train_x, train_y, n_classes, kind, alpha=Fraction(1)):
    F = len(train_x[0])
    Nc = [0] * n_classes
    cnt = [[0] * F for _ in range(n_classes)]
    for row, c in zip(train_x, train_y):
        Nc[c] += 1
        for f, v in enumerate(row):
            cnt[c][f] += (1 if v > 0 else 0) if kind == "bernoulli" else v
    N = sum(Nc)
    prior = [Fraction(n, N) for n in Nc]
    theta = []
    for c in range(n_classes):
        if kind == "bernoulli":
            theta.append([(cnt[c][f] + alpha) / (Nc[c] + 2 * alpha) for f in range(F)])
        else:
            S = sum(cnt[c])
            theta.append([(cnt[c][f] + alpha) / (S + alpha * F) for f in range(F)])
    return {"Nc": Nc, "counts": cnt, "prior": prior, "theta": theta, "kind": kind}


def exact_joint(model, x):
    """prior_c * P(x | c) as exact fractions (multinomial coefficient omitted)."""
    out = []
    for c, pc in enumerate(model["prior"]):
        p = pc
        for f, v in enumerate(x):
            t = model["theta"][c][f]
            if model["kind"] == "bernoulli":
                p *= t if v > 0 else (1 - t)
            else:
                p *= t ** v
        out.append(p)
    return out


def exact_posterior(model, x):
    j = exact_joint(model, x)
    z = sum(j)
    return [v / z for v in j]


def exact_label(model, x):
    """Lowest class index among those with the largest joint probability."""
    j = exact_joint(model, x)
    best = max(j)
    return min(c for c, v in enumerate(j) if v == best)


def log_fraction(q: Fraction) -> float:
    return math.log(q.numerator) - math.log(q.denominator)
