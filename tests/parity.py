"""Comparison helpers for GPU-vs-oracle parity tests.

Tolerances (derived in the design notes):
  * counts and class totals: bit-exact;
  * FP64 tables: |gpu - oracle| <= 1e-6 |oracle| + 1e-12 (the relative bound,
    with an absolute floor at FP64 rounding noise of the log terms);
  * FP32 / BF16 scoring rows: equal to the oracle's own round-to-nearest-even
    of its FP64 rows, or one unit in the last place away (counted);
  * raw scores, per file and class: |ds| <= 1e-4 + 1e-6 * (sum_f |g(x_f) W_cf| + |b_c|),
    the 1e-6 table tolerance carried through the sum; log posteriors: the
    sum of that bound over the classes; posteriors: 1e-4 absolute;
  * labels: identical wherever the oracle's top-1 minus top-2 score margin
    exceeds 1e-3 (reduced precision: exceeds max(1e-3, certified band)).
"""
import numpy as np

from oracle import nb, precision as P


def to_np(t):
    return t.detach().cpu().numpy()


def assert_tables(model, om, kind):
    """Device model buffer vs oracle model."""
    C, F = model.n_classes, model.n_features
    assert (to_np(model.class_totals()) == om.Nc).all(), "class totals"
    assert (to_np(model.counts()).astype(np.int64) == om.counts).all(), "counts"
    if kind == nb.MULTINOMIAL:
        assert (to_np(model.class_sums()) == om.counts.sum(axis=1)).all(), "class sums"
    W, b = nb.weight_form(om)
    for name, got, want in (("log_theta", model.log_theta(), om.log_theta),
                            ("weight", model.weight(), W), ("bias", model.bias(), b)):
        g = to_np(got)
        assert (np.abs(g - want) <= 1e-6 * np.abs(want) + 1e-12).all(), name
    if kind == nb.BERNOULLI:
        g = to_np(model.log_1m_theta())
        assert (np.abs(g - om.log_1m_theta) <= 1e-6 * np.abs(om.log_1m_theta) + 1e-12).all()
    rows, rb = P.scoring_form(W, b)
    Fp = model.layout.padded_features
    f32 = to_np(model.form_f32())
    want32 = P.rne_f32(rows).astype(np.float32)
    assert (f32[:, F:] == 0).all()
    ulps = np.abs(f32[:, :F].view(np.int32).astype(np.int64) - want32.view(np.int32).astype(np.int64))
    assert ulps.max() <= 1, f"fp32 rows off by {ulps.max()} ulp"
    bf = to_np(model.form_bf16()).view(np.uint16)
    want16 = P.bf16_bits(P.rne_bf16(rows))
    u16 = np.abs(bf[:, :F].astype(np.int64) - want16.astype(np.int64))
    assert u16.max() <= 1, f"bf16 rows off by {u16.max()} ulp"
    fb = to_np(model.form_bias())
    assert np.abs(fb.astype(np.float64) - rb).max() <= 1e-6 * np.abs(rb).max() + 1e-6
    assert Fp % 1024 == 0
    return int((ulps > 0).sum()), int((u16 > 0).sum())


def score_bound(om, X):
    W, b = nb.weight_form(om)
    g = np.asarray(X, dtype=np.float64)
    if om.kind == nb.BERNOULLI:
        g = (g > 0).astype(np.float64)
    return 1e-4 + 1e-6 * (g @ np.abs(W).T + np.abs(b)[None, :])


def assert_scores(om, X, labels, log_post, scores, rows=None, label_gate=1e-3, lp_bound=None):
    """GPU outputs (numpy) for the files X (numpy, oracle's view) vs the oracle.
    Returns a dict of error statistics."""
    s = nb.joint_log_likelihood(om, X)
    d = nb.decide(s)
    bound = score_bound(om, X)
    stats = {"n": int(X.shape[0])}
    if scores is not None:
        err = np.abs(scores.astype(np.float64) - s)
        assert (err <= bound).all(), f"score error {err.max()} vs bound {bound[err > bound].min()}"
        stats["score_max_err"] = float(err.max())
        stats["score_literal_1e-4_rate"] = float((err <= 1e-4).mean())
    if log_post is not None:
        err = np.abs(log_post.astype(np.float64) - d.log_post)
        lb = bound.sum(axis=1, keepdims=True) if lp_bound is None else lp_bound[:, None]
        assert (err <= lb).all(), f"log-posterior error {err.max()}"
        perr = np.abs(np.exp(log_post.astype(np.float64)) - np.exp(d.log_post))
        assert perr.max() <= 1e-4, f"posterior error {perr.max()}"
        stats["log_post_max_err"] = float(err.max())
        stats["post_max_err"] = float(perr.max())
    if labels is not None:
        gate = d.margin > label_gate
        agree = labels.astype(np.int64) == d.labels
        assert agree[gate].all(), f"{int((~agree[gate]).sum())} labels differ above the margin gate"
        stats["label_agreement_all"] = float(agree.mean())
        stats["files_below_gate"] = int((~gate).sum())
    return stats
