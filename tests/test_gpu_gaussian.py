"""GPU parity of the Gaussian Naive Bayes variant (the paper leaves the
variant open, section 4): exact per-class sums and sums of squares, the FP64
moments with the variance floor, the x and x^2 scoring rows, and two-class
scoring, against the FP64 oracle; plus its error paths."""
import numpy as np
import pytest
import torch

import paper_1905_13746_amd as nbg
from oracle import nb
from synth import workloads as W
from tests.parity import X_I32, X_U8, assert_scores, assert_tables, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _fit(X, y):
    m = nbg.Model(2, X.shape[1], "gaussian")
    nbg.train(m, X, y)
    return m, nb.train(to_np(X), to_np(y), 2, nb.GAUSSIAN)


@pytest.mark.parametrize("F,n_train,n_test", [(1000, 20_000, 20_001), (64, 3000, 777), (100, 5000, 4096),
                                              (5000, 4000, 1500), (7, 500, 301)])
def test_train_and_score_bytes(F, n_train, n_test):
    _case(f"gaussian u8 F={F}")
    wl = W.binary_u8(F)
    X, y = wl.train_set(n_train, device=DEV)
    if F % 4:                               # training takes rows of whole dwords
        Xp = torch.zeros((n_train, (F + 3) // 4 * 4), dtype=torch.uint8, device=DEV)
        Xp[:, :F] = X
        X = Xp[:, :F]
    m, om = _fit(X, y)
    assert m.trained
    assert_tables(m, om, nb.GAUSSIAN)
    Xt, _ = wl.test_set(n_test, device=DEV)
    if F % 4:
        Xq = torch.zeros((n_test, (F + 3) // 4 * 4), dtype=torch.uint8, device=DEV)
        Xq[:, :F] = Xt
        Xt = Xq[:, :F]
    for wtype in (nbg.W_F32, nbg.W_BF16):
        lab, lp, sc = nbg.score(m, Xt, wtype=wtype, scores=True)
        torch.cuda.synchronize()
        assert_scores(om, to_np(Xt), to_np(lab), to_np(lp), to_np(sc), wtype=wtype)
        lab1, lp1, _ = nbg.score(m, Xt, wtype=wtype)
        assert torch.equal(lab1, lab) and torch.equal(lp1, lp)


def test_int32_features():
    _case("gaussian int32")
    wl = W.tiny_int32()
    X, y = wl.train_set(W.TINY_TRAIN, device=DEV)
    X = X.clamp(max=60_000)
    m, om = _fit(X, y)
    assert_tables(m, om, nb.GAUSSIAN)
    Xt, _ = wl.test_set(W.TINY_TEST, device=DEV)
    lab, lp, sc = nbg.score(m, Xt, scores=True)
    torch.cuda.synchronize()
    assert_scores(om, to_np(Xt), to_np(lab), to_np(lp), to_np(sc), xtype=X_I32)


def test_zero_variance_features_and_floor():
    """Features constant within a class (variance = the floor only) and a
    feature constant over every file."""
    _case("gaussian zero-variance features")
    rng = np.random.default_rng(3)
    X = rng.poisson(2.0, size=(2000, 64)).astype(np.uint8)
    y = (np.arange(2000) % 2).astype(np.int32)
    X[y == 0, 5] = 0
    X[y == 1, 9] = 4
    X[:, 11] = 7
    m, om = _fit(torch.from_numpy(X).to(DEV), torch.from_numpy(y).to(DEV))
    assert_tables(m, om, nb.GAUSSIAN)
    Xt = rng.poisson(2.0, size=(3000, 64)).astype(np.uint8)
    lab, lp, sc = nbg.score(m, torch.from_numpy(Xt).to(DEV), scores=True)
    torch.cuda.synchronize()
    assert_scores(om, Xt, to_np(lab), to_np(lp), to_np(sc), xtype=X_U8)


def test_gaussian_errors():
    _case("gaussian errors")
    X = torch.full((100, 16), 3, dtype=torch.uint8, device=DEV)
    y = (torch.arange(100, device=DEV) % 2).to(torch.int32)
    m = nbg.Model(2, 16, "gaussian")
    with pytest.raises(nbg.NBError) as e:          # identical files: every variance zero
        nbg.train(m, X, y)
    assert e.value.code == -5
    Xi = torch.randint(0, 10, (100, 16), dtype=torch.int32, device=DEV)
    Xi[7, 3] = 70_000
    with pytest.raises(nbg.NBError) as e:          # squares could overflow the exact sums
        nbg.train(m, Xi, y)
    assert e.value.code == -2
    Xg = torch.randint(0, 5, (100, 16), dtype=torch.uint8, device=DEV)
    nbg.train(m, Xg, y)
    with pytest.raises(nbg.NBError):               # FP8 features
        nbg.score(m, nbg.quantize_fp8(Xg), fp8=True)
    m3 = nbg.Model(3, 16, "gaussian")
    y3 = (torch.arange(100, device=DEV) % 3).to(torch.int32)
    nbg.train(m3, Xg, y3)
    with pytest.raises(nbg.NBError):               # more than two classes
        nbg.score(m3, Xg)
    with pytest.raises(nbg.NBError):               # grouped scoring
        nbg.score_groups([m], [(0, Xg)])


def test_multiclass_tables():
    """Training and tables for more than two classes (scoring takes two)."""
    _case("gaussian 5 classes tables")
    wl = W.Workload(wid=9, n_classes=5, n_features=300, p_zero=0.6, clip255=True)
    X, y = wl.train_set(8000, device=DEV)
    m = nbg.Model(5, 300, "gaussian")
    nbg.train(m, X, y)
    om = nb.train(to_np(X), to_np(y), 5, nb.GAUSSIAN)
    assert_tables(m, om, nb.GAUSSIAN)


@pytest.mark.slow
def test_full_size_sampled():
    """The headline shape (F = 1000 byte features, 200,000 training and
    1,000,000 test files), checked on sampled files."""
    _case("gaussian full size")
    wl = W.binary_u8(1000)
    X, y = wl.train_set(200_000, device=DEV)
    m, om = _fit(X, y)
    assert_tables(m, om, nb.GAUSSIAN)
    Xt, _ = wl.test_set(1_000_000, device=DEV)
    lab, lp, sc = nbg.score(m, Xt, scores=True)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(5).choice(1_000_000, 20_000, replace=False))
    ii = torch.from_numpy(idx).to(DEV)
    assert_scores(om, to_np(Xt[ii]), to_np(lab[ii]), to_np(lp[ii]), to_np(sc[ii]))
