"""Error of every scoring path against the FP64 oracle, stated per result.

Runs the library (through its C ABI) and the oracle on the same seeded
inputs at the benchmark's full sizes and writes, for each path, the error of
each result it returns:
  * raw scores s_c: the largest |error|, the share of (file, class) values
    within 1e-4 + 1e-6 (sum_f |g W_cf| + |b_c|) (the method's score
    tolerance read for FP32) and within the literal 1e-4;
  * log posteriors: the largest |error| and the share within that tolerance
    carried through the log-sum-exp;
  * posteriors: the largest |error| and the share of files within 1e-4;
  * labels: agreement with the oracle over all files, the number of files
    whose oracle margin lies inside the path's certified band (where a
    different label is allowed), and agreement above that band (which must
    be 100%).
Paths: two classes at F = 1000 (1,000,000 files; FP32 table, and the BF16
table; on the headline workload and on near-tied classes, whose small
margins populate the label band), sixteen classes at F = 4096 (4,000,000 files; the FP32 vector path,
the BF16 matrix cores on uint8 and on FP8-e4m3 features).  FP8 features are
compared two ways: against the oracle on the FP8 values the kernel was given
(arithmetic error) and against the oracle on the original counts (total
error), and the quantisation alone is stated as the oracle on q(x) against
the oracle on x.

Test infrastructure: only the test suite may call the oracle.  Usage (GPU):
    python -m tests.precision_report [--out profiles/precision_errors]
writes <out>.json and <out>.md.  --quick runs a tenth of the files.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

import paper_1905_13746_amd as nbg
from oracle import nb, precision as P
from synth import workloads as W
from tests.parity import kernel_depth, row_bounds

CHUNK = 32768
# the oracle's decoding of every FP8 byte, applied by table lookup
E4M3_LUT = P.e4m3_value(np.arange(256))


def log(msg):
    print(f"[precision] {msg}", flush=True)


class Acc:
    """Running error statistics of one path's results over file chunks."""

    def __init__(self, name, what):
        self.name, self.what = name, what
        self.n = 0
        self.score_max = 0.0
        self.score_c9 = 0
        self.score_lit = 0
        self.score_vals = 0
        self.score_c9_worst = 0.0
        self.lp_max = 0.0
        self.lp_c9 = 0
        self.lp_vals = 0
        self.post_max = 0.0
        self.post_1e4 = 0
        self.agree = 0
        self.in_band = 0
        self.agree_gated = 0
        self.gated = 0

    def add(self, s_or, lp_or, margin, lab_or, c9, band, labels=None, log_post=None, scores=None):
        n = s_or.shape[0]
        self.n += n
        if scores is not None:
            e = np.abs(scores.astype(np.float64) - s_or)
            self.score_max = max(self.score_max, float(e.max()))
            self.score_c9 += int((e <= c9).sum())
            self.score_lit += int((e <= 1e-4).sum())
            self.score_vals += e.size
            self.score_c9_worst = max(self.score_c9_worst, float((e / c9).max()))
        if log_post is not None:
            e = np.abs(log_post.astype(np.float64) - lp_or)
            self.lp_max = max(self.lp_max, float(e.max()))
            self.lp_c9 += int((e <= c9 + c9.max(axis=1, keepdims=True)).sum())
            self.lp_vals += e.size
            pe = np.abs(np.exp(log_post.astype(np.float64)) - np.exp(lp_or)).max(axis=1)
            self.post_max = max(self.post_max, float(pe.max()))
            self.post_1e4 += int((pe <= 1e-4).sum())
        if labels is not None:
            ok = labels.astype(np.int64) == lab_or
            gate = margin > np.maximum(1e-3, band)
            self.agree += int(ok.sum())
            self.in_band += int((~gate).sum())
            self.agree_gated += int(ok[gate].sum())
            self.gated += int(gate.sum())

    def result(self):
        r = {"path": self.name, "compared_with": self.what, "files": self.n}
        if self.score_vals:
            r.update({"score_max_abs_err": self.score_max, "score_c9_rate": self.score_c9 / self.score_vals,
                      "score_c9_worst_ratio": self.score_c9_worst,
                      "score_literal_1e-4_rate": self.score_lit / self.score_vals})
        if self.lp_vals:
            r.update({"log_post_max_abs_err": self.lp_max, "log_post_c9_rate": self.lp_c9 / self.lp_vals,
                      "post_max_abs_err": self.post_max, "post_1e-4_rate": self.post_1e4 / self.n})
        if self.gated or self.in_band:
            r.update(label_agreement_all_files=self.agree / self.n, files_in_certified_band=self.in_band,
                     label_agreement_above_band=(self.agree_gated / self.gated) if self.gated else None)
        return r


def bands(om, G, wtype, xtype, Gq=None):
    """Per-file label band of a path (as the parity tests gate it): the
    derived accumulation bound of the kernel's posterior rows (two classes:
    the log-odds row; otherwise twice the largest centred row), plus, for
    FP8 features compared with the original counts, the quantisation term."""
    Wt, b = nb.weight_form(om)
    rows, rb = P.scoring_form(Wt, b)
    rows_hat = P.rne_bf16(rows) if wtype == nbg.W_BF16 else P.rne_f32(rows)
    ulp = np.spacing(np.abs(rows_hat).astype(np.float32)).astype(np.float64)
    if wtype == nbg.W_BF16:
        ulp *= 2.0 ** 16
    depth, rf = kernel_depth(om.n_classes, om.n_features, wtype, xtype)
    Gk = G if Gq is None else Gq
    eb = row_bounds(rows, rb, rows_hat, P.rne_f32(rb), Gk, depth, rf, ulp)[:, :-1]
    if Gq is not None:   # the features' own rounding: sum_f |x - q(x)| |R^|
        eb = eb + np.abs(G - Gq) @ np.abs(rows_hat[:-1]).T
    return eb[:, 0] if om.n_classes == 2 else 2.0 * eb.max(axis=1)


def c9_bound(om, G):
    Wt, b = nb.weight_form(om)
    return 1e-4 + 1e-6 * (G @ np.abs(Wt).T + np.abs(b)[None, :])


def run_paths(om, Xt, paths, n_files):
    """paths: [(Acc, xtype, wtype, fp8, outs)] with outs the GPU results
    (labels, log_post, scores) over every file (device tensors or None)."""
    kind_bin = om.kind == nb.BERNOULLI
    quant = None
    for r0 in range(0, n_files, CHUNK):
        r1 = min(n_files, r0 + CHUNK)
        x = Xt[r0:r1]
        xn = x.cpu().numpy()
        s = nb.joint_log_likelihood(om, xn)
        d = nb.decide(s)
        G = (xn > 0).astype(np.float64) if kind_bin else xn.astype(np.float64)
        c9 = c9_bound(om, G)
        need_q = any(p[3] for p in paths)
        if need_q:
            qv = E4M3_LUT[W.to_fp8_e4m3(x).cpu().numpy()]
            sq = nb.joint_log_likelihood(om, qv)
            dq = nb.decide(sq)
            Gq = (qv > 0).astype(np.float64) if kind_bin else qv
            c9q = c9_bound(om, Gq)
            if quant is None:
                quant = Acc("oracle on q(x)", "oracle on x (quantisation alone)")
            # the quantisation's own effect, the oracle on both sides
            quant.add(s, d.log_post, d.margin, d.labels, c9, _quant_band(om, G, Gq), labels=dq.labels,
                      log_post=dq.log_post, scores=sq)
        for acc, xtype, wtype, fp8, outs, vs_counts in paths:
            lab, lp, sc = (None if t is None else t[r0:r1].cpu().numpy() for t in outs)
            if fp8 and not vs_counts:
                acc.add(sq, dq.log_post, dq.margin, dq.labels, c9q, bands(om, Gq, wtype, xtype),
                        labels=lab, log_post=lp, scores=sc)
            elif fp8:
                acc.add(s, d.log_post, d.margin, d.labels, c9, bands(om, G, wtype, xtype, Gq),
                        labels=lab, log_post=lp, scores=sc)
            else:
                acc.add(s, d.log_post, d.margin, d.labels, c9, bands(om, G, wtype, xtype),
                        labels=lab, log_post=lp, scores=sc)
        if (r0 // CHUNK) % 16 == 0:
            log(f"  files {r1} / {n_files}")
    return quant


def _quant_band(om, G, Gq):
    """Label band of the quantisation alone: sum_f |g(x) - g(q)| |W_c1 - W_c2|
    bounded by twice the largest per-class |W| contraction."""
    Wt, _ = nb.weight_form(om)
    e = np.abs(G - Gq) @ np.abs(Wt).T
    return 2.0 * e.max(axis=1)


def two_class(n_test, n_train, near_tie=False):
    wl = W.near_tie_u8(1000) if near_tie else W.binary_u8(1000)
    tag0 = "near-tied classes, " if near_tie else ""
    log(f"two classes F=1000 {tag0}: train {n_train}, test {n_test}")
    X, y = wl.train_set(n_train, device="cuda")
    m = nbg.Model(2, 1000, "multinomial")
    nbg.train(m, X, y)
    om = nb.train(X.cpu().numpy(), y.cpu().numpy(), 2, nb.MULTINOMIAL)
    del X, y
    Xt, _ = wl.test_set(n_test, device="cuda")
    paths = []
    for wtype, tag in ((nbg.W_F32, "FP32 table"), (nbg.W_BF16, "BF16 table")):
        lab, lp, _ = nbg.score(m, Xt, wtype=wtype)            # the timed launch: labels + log posteriors
        _, _, sc = nbg.score(m, Xt, wtype=wtype, labels=False, log_post=False, scores=True)
        torch.cuda.synchronize()
        paths.append((Acc(f"two classes, {tag0}uint8, {tag}", "oracle on x"), 0, wtype, False, (lab, lp, sc),
                      True))
    run_paths(om, Xt, paths, n_test)
    return [p[0].result() for p in paths]


def sixteen_class(n_test, n_train):
    wl = W.family16()
    F, C = wl.n_features, wl.n_classes
    log(f"sixteen classes F={F}: train {n_train}, test {n_test}")
    X, y = wl.train_set(n_train, device="cuda")
    m = nbg.Model(C, F, "multinomial")
    nbg.train(m, X, y)
    t0 = time.time()
    om = nb.train(X.cpu().numpy(), y.cpu().numpy(), C, nb.MULTINOMIAL)
    log(f"  oracle trained in {time.time() - t0:.1f} s")
    del X, y
    torch.cuda.empty_cache()
    Xt, _ = wl.test_set(n_test, device="cuda")
    q8 = nbg.quantize_fp8(Xt)
    paths = []
    specs = (("FP32 table, vector ALUs, uint8", Xt, nbg.W_F32, False, False),
             ("BF16 table, matrix cores, uint8", Xt, nbg.W_BF16, False, False),
             ("BF16 table, matrix cores, FP8-e4m3", q8, nbg.W_BF16, True, False),
             ("BF16 table, matrix cores, FP8-e4m3", q8, nbg.W_BF16, True, True))
    for name, x, wtype, fp8, vs_counts in specs:
        lab, lp, _ = nbg.score(m, x, wtype=wtype, fp8=fp8)     # the timed launch
        _, _, sc = nbg.score(m, x, wtype=wtype, fp8=fp8, labels=False, log_post=False, scores=True)
        torch.cuda.synchronize()
        what = "oracle on x" if not fp8 else ("oracle on x (total error)" if vs_counts
                                               else "oracle on q(x) (arithmetic error)")
        paths.append((Acc(f"sixteen classes, {name}", what), 2 if fp8 else 0, wtype, fp8, (lab, lp, sc),
                      vs_counts))
    quant = run_paths(om, Xt, paths, n_test)
    return [p[0].result() for p in paths] + [quant.result()]


def markdown(res, cmd):
    lines = ["# Error against the FP64 oracle, per result", "",
             f"Command: `{cmd}` (on the MI355X; writes this file and its JSON).", "",
             "Tolerance columns: C9 = |ds| <= 1e-4 + 1e-6 (sum_f |g W_cf| + |b_c|) on raw scores and "
             "that bound carried through the log-sum-exp on log posteriors; 1e-4 = the literal absolute "
             "bound (raw scores: per value; posteriors: per file, largest class).  Band = the path's "
             "certified label band (files whose oracle margin is below max(1e-3, band) may take another "
             "label).  FP8 rows: arithmetic = against the oracle on the FP8 values the kernel read; total = "
             "against the oracle on the original counts; the quantisation row is the oracle on q(x) "
             "against the oracle on x.", "",
             "| path | compared with | files | max abs score err | score C9 rate | score 1e-4 rate | "
             "max abs log-post err | log-post C9 rate | max abs posterior err | posterior 1e-4 rate | "
             "labels agree (all files) | files in band | labels agree above band |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|---|"]

    def f(r, k, fmt):
        v = r.get(k)
        return "n/a" if v is None else format(v, fmt)

    for r in res:
        lines.append(f"| {r['path']} | {r['compared_with']} | {r['files']:,} | {f(r, 'score_max_abs_err', '.3g')} | "
                     f"{f(r, 'score_c9_rate', '.6f')} | {f(r, 'score_literal_1e-4_rate', '.4f')} | "
                     f"{f(r, 'log_post_max_abs_err', '.3g')} | {f(r, 'log_post_c9_rate', '.6f')} | "
                     f"{f(r, 'post_max_abs_err', '.3g')} | {f(r, 'post_1e-4_rate', '.6f')} | "
                     f"{f(r, 'label_agreement_all_files', '.7f')} | {r.get('files_in_certified_band', 'n/a')} | "
                     f"{f(r, 'label_agreement_above_band', '.6f')} |")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="profiles/precision_errors")
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    k = 10 if args.quick else 1
    res = two_class(W.BINARY_TEST // k, W.BINARY_TRAIN // k)
    res += two_class(W.BINARY_TEST // k, W.BINARY_TRAIN // k, near_tie=True)
    res += sixteen_class(W.FAMILY_TEST // k, W.FAMILY_TRAIN // k)
    cmd = "python -m tests.precision_report" + (" --quick" if args.quick else "")
    with open(args.out + ".json", "w") as fh:
        json.dump({"command": cmd, "results": res}, fh, indent=1)
    with open(args.out + ".md", "w") as fh:
        fh.write(markdown(res, cmd))
    log("done")
    for r in res:
        log(json.dumps(r))
    return 0


if __name__ == "__main__":
    sys.exit(main())
