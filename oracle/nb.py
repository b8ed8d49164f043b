"""FP64 Naive Bayes oracle (test infrastructure; see the package docstring).

Method (paper, section 4): a Naive Bayes classifier over per-file opcode
occurrence features a_1..a_n computes the class posterior
P(C | a_1..a_n) and labels a file malware when the malware posterior is the
higher one, otherwise benign.  With the features conditionally independent
given the class, the posterior is proportional to P(C) * prod_f P(a_f | C).

Readings where the paper is silent (each listed in the design notes):
  * variant: multinomial (occurrence counts) and Bernoulli (presence) NB;
  * smoothing: Laplace/Lidstone with alpha > 0 (default 1);
  * prior: the empirical class frequency N_c / N (the printed equation omits
    P(C); it is reinstated, and equals the literal formula for balanced data);
  * the multinomial coefficient is class-independent and omitted: "scores"
    are joint log-likelihoods log P(C) + sum_f x_f log theta_{C,f};
  * ties: "otherwise benign" -> the lowest class index wins an exact tie;
  * Bernoulli presence is x > 0;
  * a third variant, Gaussian NB over the occurrence counts: per class and
    feature the mean and the (population) variance of the counts, every
    variance increased by var_smoothing (1e-9) times the largest
    per-feature variance of all training files together (scikit-learn's
    GaussianNB convention, which keeps zero-variance features finite).

Everything is computed in float64 straight from the definitions, with no
blocking or fusion; large inputs are only split into row chunks.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

MULTINOMIAL = "multinomial"
BERNOULLI = "bernoulli"
GAUSSIAN = "gaussian"
VAR_SMOOTHING = 1e-9
CHUNK_ROWS = 65536


def _as_np(a):
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.asarray(a)


def class_totals(y, n_classes: int) -> np.ndarray:
    """N_c = number of training files with label c (int64[C])."""
    y = _as_np(y).astype(np.int64).reshape(-1)
    if y.size and (y.min() < 0 or y.max() >= n_classes):
        raise ValueError("label outside [0, C)")
    out = np.zeros(n_classes, dtype=np.int64)
    for c in range(n_classes):
        out[c] = np.count_nonzero(y == c)
    return out


def feature_counts(X, y, n_classes: int, kind: str = MULTINOMIAL) -> np.ndarray:
    """Per-class feature counts over the training files (int64[C, F]).

    multinomial: T[c, f] = sum over files of class c of x_f (occurrences)
    bernoulli:   D[c, f] = number of files of class c with x_f > 0
    """
    X = _as_np(X)
    y = _as_np(y).astype(np.int64).reshape(-1)
    if X.ndim != 2 or X.shape[0] != y.size:
        raise ValueError("X must be [N, F] with one label per row")
    if X.size and X.min() < 0:
        raise ValueError("occurrence counts must be non-negative")
    out = np.zeros((n_classes, X.shape[1]), dtype=np.int64)
    for c in range(n_classes):
        for r0 in range(0, X.shape[0], CHUNK_ROWS):
            xs = X[r0:r0 + CHUNK_ROWS][y[r0:r0 + CHUNK_ROWS] == c].astype(np.int64)
            out[c] += (xs > 0).sum(axis=0) if kind == BERNOULLI else xs.sum(axis=0)
    return out


def square_sums(X, y, n_classes: int) -> np.ndarray:
    """Q[c, f] = sum over files of class c of x_f^2 (int64[C, F])."""
    X = _as_np(X)
    y = _as_np(y).astype(np.int64).reshape(-1)
    out = np.zeros((n_classes, X.shape[1]), dtype=np.int64)
    for c in range(n_classes):
        for r0 in range(0, X.shape[0], CHUNK_ROWS):
            xs = X[r0:r0 + CHUNK_ROWS][y[r0:r0 + CHUNK_ROWS] == c].astype(np.int64)
            out[c] += (xs * xs).sum(axis=0)
    return out


def gaussian_moments(T, Q, Nc, var_smoothing: float = VAR_SMOOTHING):
    """Per class and feature: mean = T / N_c and variance = (N_c Q - T^2) / N_c^2
    (population variance; numerators in exact integers, one rounding each),
    plus epsilon = var_smoothing * the largest variance of a feature over
    all training files.  Returns (mean, variance + epsilon, epsilon)."""
    T, Q, Nc = np.asarray(T), np.asarray(Q), np.asarray(Nc)
    C, F = T.shape
    mean = np.empty((C, F), dtype=np.float64)
    var = np.empty((C, F), dtype=np.float64)
    for c in range(C):
        n = int(Nc[c])
        for f in range(F):
            t, q = int(T[c, f]), int(Q[c, f])
            mean[c, f] = t / n
            var[c, f] = (n * q - t * t) / (n * n)
    N = int(Nc.sum())
    top = 0.0
    for f in range(F):
        t = sum(int(T[c, f]) for c in range(C))
        q = sum(int(Q[c, f]) for c in range(C))
        top = max(top, (N * q - t * t) / (N * N))
    eps = var_smoothing * top
    return mean, var + eps, eps


def log_prior(Nc) -> np.ndarray:
    """log P(C = c) = log N_c - log N, the empirical (unsmoothed) prior."""
    Nc = np.asarray(Nc, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return np.log(Nc) - np.log(Nc.sum())


def multinomial_log_theta(T, alpha: float) -> np.ndarray:
    """log theta[c, f] = log((T[c,f] + alpha) / (sum_f T[c,f] + alpha * F))."""
    T = np.asarray(T, dtype=np.float64)
    F = T.shape[1]
    S = T.sum(axis=1, keepdims=True)
    return np.log(T + alpha) - np.log(S + alpha * F)


def bernoulli_log_theta(D, Nc, alpha: float):
    """Presence probability theta[c, f] = (D[c,f] + alpha) / (N_c + 2 alpha).

    Returns (log theta, log(1 - theta)); the complement is taken from the
    counts, (N_c - D + alpha) / (N_c + 2 alpha), so nothing cancels."""
    D = np.asarray(D, dtype=np.float64)
    N = np.asarray(Nc, dtype=np.float64)[:, None]
    den = np.log(N + 2.0 * alpha)
    return np.log(D + alpha) - den, np.log(N - D + alpha) - den


@dataclass
class Model:
    kind: str
    alpha: float
    Nc: np.ndarray            # int64[C]
    counts: np.ndarray        # int64[C, F]: T (multinomial) or D (Bernoulli)
    log_prior: np.ndarray     # float64[C]
    log_theta: np.ndarray | None     # float64[C, F] (multinomial, Bernoulli)
    log_1m_theta: np.ndarray | None  # float64[C, F] (Bernoulli only)
    sq: np.ndarray | None = None     # int64[C, F] sums of squares (Gaussian)
    mean: np.ndarray | None = None   # float64[C, F] (Gaussian)
    var: np.ndarray | None = None    # float64[C, F] variance + epsilon (Gaussian)
    eps: float = 0.0                 # the variance floor added (Gaussian)

    @property
    def n_classes(self):
        return self.Nc.size

    @property
    def n_features(self):
        return self.counts.shape[1]


def train(X, y, n_classes: int, kind: str = MULTINOMIAL, alpha: float = 1.0) -> Model:
    """Fit one Naive Bayes model on labelled training files (section 4)."""
    if not alpha > 0:
        raise ValueError("alpha must be > 0")
    if kind not in (MULTINOMIAL, BERNOULLI, GAUSSIAN):
        raise ValueError(kind)
    Nc = class_totals(y, n_classes)
    if kind == GAUSSIAN:
        T = feature_counts(X, y, n_classes, MULTINOMIAL)
        Q = square_sums(X, y, n_classes)
        mean, var, eps = gaussian_moments(T, Q, Nc)
        return Model(kind, alpha, Nc, T, log_prior(Nc), None, None, Q, mean, var, eps)
    counts = feature_counts(X, y, n_classes, kind)
    if kind == MULTINOMIAL:
        return Model(kind, alpha, Nc, counts, log_prior(Nc),
                     multinomial_log_theta(counts, alpha), None)
    lt, l1m = bernoulli_log_theta(counts, Nc, alpha)
    return Model(kind, alpha, Nc, counts, log_prior(Nc), lt, l1m)


def weight_form(m: Model):
    """Linear form of the scorer: s = bias + g(x) @ W.T with g(x) = x
    (multinomial), 1[x > 0] (Bernoulli) or [x, x^2] (Gaussian, W = [A | B]).

    multinomial: W = log theta, bias = log prior
    bernoulli:   W = log theta - log(1 - theta),
                 bias = log prior + sum_f log(1 - theta)
    gaussian:    A = mean / var, B = -1 / (2 var),
                 bias = log prior - (1/2) sum_f (log(2 pi var) + mean^2 / var)"""
    if m.kind == GAUSSIAN:
        A = m.mean / m.var
        B = -0.5 / m.var
        bias = m.log_prior - 0.5 * (np.log(2.0 * np.pi * m.var) + m.mean * m.mean / m.var).sum(axis=1)
        return np.concatenate([A, B], axis=1), bias
    if m.kind == MULTINOMIAL:
        return m.log_theta.copy(), m.log_prior.copy()
    return m.log_theta - m.log_1m_theta, m.log_prior + m.log_1m_theta.sum(axis=1)


def gaussian_score_form(m: Model):
    """The Gaussian scorer as s_c = bias_c + sum_f h_cf (x_f - mean_cf)^2 with
    h = -1 / (2 var) and bias = log prior - (1/2) sum_f log(2 pi var): the
    density's own form, which keeps each term's relative error small when a
    variance is tiny (the expanded form A x + B x^2 cancels large terms).
    Returns (mean, h, bias)."""
    if m.kind != GAUSSIAN:
        raise ValueError("a Gaussian model")
    h = -0.5 / m.var
    bias = m.log_prior - 0.5 * np.log(2.0 * np.pi * m.var).sum(axis=1)
    return m.mean.copy(), h, bias


def joint_log_likelihood(m: Model, X) -> np.ndarray:
    """s[j, c] = log P(c) + log P(x_j | c) in float64 (float64[n, C]).

    multinomial: log P(x | c) = sum_f x_f log theta[c, f]
    bernoulli:   log P(x | c) = sum_f b_f log theta + (1 - b_f) log(1 - theta),
                 b = 1[x > 0]   (the textbook form, not the weight form)
    gaussian:    log P(x | c) = -(1/2) sum_f (log(2 pi var) + (x_f - mean)^2 / var)"""
    X = _as_np(X)
    n = X.shape[0]
    if X.shape[1] != m.n_features:
        raise ValueError("feature count mismatch")
    out = np.empty((n, m.n_classes), dtype=np.float64)
    for r0 in range(0, n, CHUNK_ROWS):
        xs = X[r0:r0 + CHUNK_ROWS].astype(np.float64)
        if xs.size and xs.min() < 0:
            raise ValueError("occurrence counts must be non-negative")
        if m.kind == MULTINOMIAL:
            s = xs @ m.log_theta.T
        elif m.kind == GAUSSIAN:
            s = np.empty((xs.shape[0], m.n_classes))
            for c in range(m.n_classes):
                d = xs - m.mean[c][None, :]
                s[:, c] = -0.5 * (np.log(2.0 * np.pi * m.var[c]).sum() + (d * d / m.var[c][None, :]).sum(axis=1))
        else:
            b = (xs > 0).astype(np.float64)
            s = b @ m.log_theta.T + (1.0 - b) @ m.log_1m_theta.T
        out[r0:r0 + xs.shape[0]] = s + m.log_prior[None, :]
    return out


@dataclass
class Decision:
    labels: np.ndarray    # int64[n]: smallest class index attaining the max score
    log_post: np.ndarray  # float64[n, C]: log P(c | x)
    margin: np.ndarray    # float64[n]: top-1 minus top-2 score (inf when C == 1)


def decide(s) -> Decision:
    """Decision rule and posteriors from joint log-likelihoods.

    The label is the class with the highest posterior; an exact tie goes to
    the lowest index (benign = 0 for the two-class detector).  The posterior
    normaliser is the log-sum-exp over classes, taken about the maximum."""
    s = np.asarray(s, dtype=np.float64)
    labels = np.argmax(s, axis=1)          # numpy returns the first maximum
    mx = s.max(axis=1, keepdims=True)
    lse = mx + np.log(np.exp(s - mx).sum(axis=1, keepdims=True))
    srt = np.sort(s, axis=1)
    margin = srt[:, -1] - srt[:, -2] if s.shape[1] > 1 else np.full(s.shape[0], np.inf)
    return Decision(labels, s - lse, margin)


def classify(m: Model, X) -> Decision:
    return decide(joint_log_likelihood(m, X))
