"""Per-group top-k feature selection and feature gather (test infrastructure).

Paper, section 3: the features are opcode occurrence counts; the opcodes that
separate malware from benign programs are found, for each size group on its
own, from the difference between the two classes' normalised opcode
occurrences, and each group keeps its top k opcodes.  Section 4: each group's
model is trained on, and classifies with, that group's top-k features
(k = 20, 40, 80, 100, 160, 200 in the experiments).

The normalisation is only cited, not given.  Reading used here: within one
group, opcode f's normalised occurrence in class c is its share of the
class's counted occurrences, phi_cf = T_cf / S_c with S_c = sum_f T_cf (for a
presence model, T = D and S_c = N_c: the share of the class's files that
contain f); a class with S_c = 0 has phi = 0.  The selection score is
d_f = |phi_1f - phi_0f|; the top k are the k largest d_f, an exact tie going
to the lower feature index; the selected list is returned in ascending
feature order, so a gathered row keeps the original feature order.

Because the comparison decides an integer result (which features), it is
made exactly: d_f * S_0 * S_1 = |T_1f S_0 - T_0f S_1| is an integer and
S_0 S_1 is the same for every f, so ranking the integers ranks d_f.  Python
integers keep every product exact.

A k-feature model is the model trained on the gathered columns: its counts
are the selected columns of the full counts (occurrence and presence sums
are per column) and its tables follow from those counts exactly as in
training (so S_c becomes the sum over the selected columns only).
"""
from __future__ import annotations

import numpy as np

from . import nb


def _two_class(counts):
    counts = np.asarray(counts)
    if counts.ndim != 2 or counts.shape[0] != 2:
        raise ValueError("selection needs the counts of exactly two classes")
    if counts.size and counts.min() < 0:
        raise ValueError("counts must be non-negative")
    return counts


def class_sums(counts, Nc=None, kind: str = nb.MULTINOMIAL):
    """S_c: the normaliser of class c (sum_f T_cf, or N_c for presence)."""
    counts = _two_class(counts)
    if kind == nb.BERNOULLI:
        if Nc is None:
            raise ValueError("presence counts are normalised by N_c")
        return [int(v) for v in np.asarray(Nc).reshape(-1)]
    return [int(sum(int(v) for v in counts[c])) for c in range(2)]


def selection_keys(counts, sums) -> list:
    """Integer numerators |T_1f S_0 - T_0f S_1| (one Python int per feature).

    When a class has S_c = 0 its phi is 0 and d_f is the other class's share
    T_f / S_other, which ranks like the other class's count T_f; the
    cross-product would be 0 for every f there, so that case keys on T_f."""
    counts = _two_class(counts)
    S0, S1 = int(sums[0]), int(sums[1])
    keys = []
    for f in range(counts.shape[1]):
        t0, t1 = int(counts[0, f]), int(counts[1, f])
        if S0 == 0 or S1 == 0:
            # phi of an empty class is 0; d_f is then the other class's
            # share, which ranks like the other class's count
            keys.append(t1 if S0 == 0 else t0)
        else:
            keys.append(abs(t1 * S0 - t0 * S1))
    return keys


def top_k(counts, sums, k: int) -> np.ndarray:
    """The k features with the largest selection score, ties to the lower
    index, returned in ascending feature order (int32[k])."""
    counts = _two_class(counts)
    F = counts.shape[1]
    if not 1 <= k <= F:
        raise ValueError("k must be in [1, F]")
    keys = selection_keys(counts, sums)
    order = sorted(range(F), key=lambda f: (-keys[f], f))
    return np.array(sorted(order[:k]), dtype=np.int32)


def select_model_features(m: nb.Model, k: int) -> np.ndarray:
    """Top-k features of a trained two-class model (its own counts)."""
    return top_k(m.counts, class_sums(m.counts, m.Nc, m.kind), k)


def gather(X, idx) -> np.ndarray:
    """out[i, j] = X[i, idx[j]] (the k selected opcode counts of each file)."""
    X = nb._as_np(X)
    idx = np.asarray(idx, dtype=np.int64).reshape(-1)
    if idx.size and (idx.min() < 0 or idx.max() >= X.shape[1]):
        raise ValueError("feature index outside [0, F)")
    return X[:, idx]


def model_on_features(m: nb.Model, idx) -> nb.Model:
    """The model trained on the gathered columns idx of m's training files,
    built from m's counts: counts[:, idx], same class totals, tables
    recomputed from the selected counts alone."""
    idx = np.asarray(idx, dtype=np.int64).reshape(-1)
    if idx.size == 0 or idx.min() < 0 or idx.max() >= m.n_features:
        raise ValueError("feature index outside [0, F)")
    counts = m.counts[:, idx].copy()
    if m.kind == nb.MULTINOMIAL:
        return nb.Model(m.kind, m.alpha, m.Nc.copy(), counts, m.log_prior.copy(),
                        nb.multinomial_log_theta(counts, m.alpha), None)
    lt, l1m = nb.bernoulli_log_theta(counts, m.Nc, m.alpha)
    return nb.Model(m.kind, m.alpha, m.Nc.copy(), counts, m.log_prior.copy(), lt, l1m)


def expanded_model(mk: nb.Model, idx, n_features: int) -> nb.Model:
    """The k-feature model mk (on the ascending feature list idx) written
    over all n_features: its counts and log tables at the selected features
    and zero elsewhere, class totals and priors unchanged.  A zero log table
    entry contributes nothing to a file's joint log likelihood, so on a full
    row it scores exactly what mk scores on the row's selected features."""
    idx = np.asarray(idx, dtype=np.int64).reshape(-1)
    if idx.size != mk.n_features or np.any(np.diff(idx) <= 0) or idx[0] < 0 or idx[-1] >= n_features:
        raise ValueError("idx must list mk's features in ascending order within [0, n_features)")
    C = mk.n_classes

    def spread(a, dtype):
        if a is None:
            return None
        out = np.zeros((C, n_features), dtype=dtype)
        out[:, idx] = a
        return out

    return nb.Model(mk.kind, mk.alpha, mk.Nc.copy(), spread(mk.counts, np.int64), mk.log_prior.copy(),
                    spread(mk.log_theta, np.float64), spread(mk.log_1m_theta, np.float64))

