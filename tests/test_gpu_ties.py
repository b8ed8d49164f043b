"""GPU tests of the decision rule at exact ties (section 4: a file is malware
only if the malware posterior is the higher one, otherwise benign; read for C
classes as: the lowest class index among those with the highest posterior).

The margin-gated label checks elsewhere exclude ties by construction, so the
rule is exercised here on inputs that make the tie exact:
  * symmetric training data (every class trained on the same files, so N_c
    and every count agree): each class's table row is the same, every file's
    class scores are equal, every label must be 0 and every log posterior
    -log C;
  * sixteen classes where classes 3 and 7 are trained on the same files:
    for files of class 3's distribution the top two scores are an exact tie
    between 3 and 7, and the label must be 3.
Every scoring path is covered: two classes (streaming kernel, uint8 / int32 /
FP8, grouped launch), the FP32 vector path (3 and 16 classes), the BF16
vector path, and the BF16 matrix cores (with and without raw scores, uint8
and FP8)."""
import math

import numpy as np
import pytest
import torch

import paper_1905_13746_amd as nbg
from oracle import nb, precision as P
from synth import workloads as W
from tests.parity import to_np

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _symmetric_model(C, F, kind, clip=True, n_per_class=700):
    """A model of C classes, each trained on the same n_per_class files."""
    wl = W.Workload(wid=7, n_classes=2, n_features=F, p_zero=0.8 if clip else 0.7, clip255=clip, group=F)
    X, _ = wl.train_set(n_per_class, device=DEV)
    Xs = X.repeat(C, 1)
    y = torch.arange(C, dtype=torch.int32, device=DEV).repeat_interleave(n_per_class)
    m = nbg.Model(C, F, kind)
    nbg.train(m, Xs, y)
    om = nb.train(to_np(Xs), to_np(y), C, kind)
    # the oracle's own rows agree bit for bit, so its scores tie exactly
    Wt, b = nb.weight_form(om)
    assert (Wt == Wt[0]).all() and (b == b[0]).all()
    return wl, m


def _check_all_ties(lab, lp, sc, C):
    lab = to_np(lab)
    assert (lab == 0).all(), f"{int((lab != 0).sum())} tied files not given class 0"
    if lp is not None:
        lp = to_np(lp).astype(np.float64)
        assert np.abs(lp + math.log(C)).max() <= 1e-5
    if sc is not None:
        sc = to_np(sc)
        assert (sc == sc[:, :1]).all(), "tied class scores differ"


TWO_CLASS = [("u8_F1000", 1000, True, False), ("u8_F5000", 5000, True, False), ("i32_F1000", 1000, False, False),
             ("i32_F64", 64, False, False), ("fp8_F1000", 1000, True, True), ("u8_F100", 100, True, False)]


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
@pytest.mark.parametrize("name,F,clip,fp8", TWO_CLASS, ids=[t[0] for t in TWO_CLASS])
def test_two_class_ties_go_to_benign(name, F, clip, fp8, kind):
    _case(f"ties two classes {name} {kind}")
    wl, m = _symmetric_model(2, F, kind, clip)
    Xt, _ = wl.test_set(2053, device=DEV)
    x = W.to_fp8_e4m3(Xt) if fp8 else Xt
    for wtype in (nbg.W_F32, nbg.W_BF16):
        lab, lp, sc = nbg.score(m, x, wtype=wtype, fp8=fp8, scores=True)
        torch.cuda.synchronize()
        _check_all_ties(lab, lp, sc, 2)
        lab1, lp1, _ = nbg.score(m, x, wtype=wtype, fp8=fp8)
        torch.cuda.synchronize()
        _check_all_ties(lab1, lp1, None, 2)


def test_two_class_ties_in_grouped_launch():
    _case("ties grouped")
    F = 2000
    models, groups = [], []
    for g, n in enumerate((300, 1, 4097, 64)):
        wl, m = _symmetric_model(2, F, nb.MULTINOMIAL, n_per_class=300 + g)
        models.append(m)
        groups.append((g, wl.test_set(n, device=DEV)[0]))
    groups.insert(2, (None, groups[1][1]))                 # a group without a model of its own
    for tile in (0, 40):
        outs = nbg.score_groups(models, groups, scores=True, tile_rows=tile)
        torch.cuda.synchronize()
        for lab, lp, sc in outs:
            _check_all_ties(lab, lp, sc, 2)


MULTI = [("C3_F1000_fp32", 3, 1000, nbg.W_F32, False), ("C16_F4096_fp32", 16, 4096, nbg.W_F32, False),
         ("C5_F300_bf16_valu", 5, 300, nbg.W_BF16, False), ("C16_F4096_bf16_mfma", 16, 4096, nbg.W_BF16, False),
         ("C16_F1000_bf16_mfma_fp8", 16, 1000, nbg.W_BF16, True), ("C40_F500_bf16_mfma", 40, 500, nbg.W_BF16, False)]


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
@pytest.mark.parametrize("name,C,F,wtype,fp8", MULTI, ids=[t[0] for t in MULTI])
def test_multiclass_ties_go_to_lowest_index(name, C, F, wtype, fp8, kind):
    _case(f"ties {name} {kind}")
    wl, m = _symmetric_model(C, F, kind, n_per_class=300)
    Xt, _ = wl.test_set(1031, device=DEV)
    x = W.to_fp8_e4m3(Xt) if fp8 else Xt
    with_scores = wtype == nbg.W_BF16 or C + 1 <= 32
    lab, lp, sc = nbg.score(m, x, wtype=wtype, fp8=fp8, scores=with_scores)
    torch.cuda.synchronize()
    _check_all_ties(lab, lp, sc if with_scores else None, C)
    # labels and log posteriors only (the staged matrix-core kernel at 16 classes)
    lab1, lp1, _ = nbg.score(m, x, wtype=wtype, fp8=fp8)
    torch.cuda.synchronize()
    _check_all_ties(lab1, lp1, None, C)


@pytest.mark.parametrize("wtype,fp8", [(nbg.W_F32, False), (nbg.W_BF16, False), (nbg.W_BF16, True)],
                         ids=["fp32_valu", "bf16_mfma_u8", "bf16_mfma_fp8"])
def test_sixteen_classes_tie_between_3_and_7(wtype, fp8):
    """Classes 3 and 7 trained on the same files (the other classes on their
    own); files of class 3's distribution tie exactly between 3 and 7 at the
    top, and get label 3 wherever both are ahead of every other class by
    more than the path's certified rounding band (the label gate used by
    every other parity test)."""
    _case(f"tie 3 vs 7 wtype={wtype} fp8={fp8}")
    C, F = 16, 1000
    wl = W.Workload(wid=7, n_classes=C, n_features=F, p_zero=0.8, clip255=True, group=16 * F)
    X, y = wl.train_set(16 * 400, device=DEV)
    keep = y != 7
    X3 = X[y == 3]
    X = torch.cat([X[keep], X3])
    y = torch.cat([y[keep], torch.full((X3.shape[0],), 7, dtype=torch.int32, device=DEV)])
    m = nbg.Model(C, F, "multinomial")
    nbg.train(m, X, y)
    om = nb.train(to_np(X), to_np(y), C, nb.MULTINOMIAL)
    Wt, b = nb.weight_form(om)
    assert (Wt[3] == Wt[7]).all() and b[3] == b[7]
    Xt, yt = wl.test_set(3000, device=DEV)
    Xt = Xt[yt == 3]
    x = W.to_fp8_e4m3(Xt) if fp8 else Xt
    xo = P.e4m3_value(to_np(x)) if fp8 else to_np(Xt)
    s = nb.joint_log_likelihood(om, xo)
    others = np.delete(s, [3, 7], axis=1).max(axis=1)
    lead = s[:, 3] - others
    rows, rb = P.scoring_form(Wt, b)
    rh = P.rne_bf16(rows) if wtype == nbg.W_BF16 else P.rne_f32(rows)
    band = P.certified_band(rows, rb, rh, P.rne_f32(rb), xo, xo, False, n_terms=F + 1)
    ahead = lead > np.maximum(1e-3, band)
    assert ahead.sum() > 0.5 * len(lead)
    lab, lp, _ = nbg.score(m, x, wtype=wtype, fp8=fp8)
    torch.cuda.synchronize()
    lab, lp = to_np(lab), to_np(lp)
    assert (lab[ahead] == 3).all(), f"{int((lab[ahead] != 3).sum())} of {int(ahead.sum())} ties not given class 3"
    assert (lp[:, 3] == lp[:, 7]).all()
    if wtype == nbg.W_F32:
        _, _, sc = nbg.score(m, x, wtype=wtype, fp8=fp8, scores=True)
        torch.cuda.synchronize()
        sc = to_np(sc)
        assert (sc[:, 3] == sc[:, 7]).all()
