"""GPU parity: libnbgpu (through its C ABI) vs the FP64 oracle on the same
seeded inputs.  Sizes span several tiles and ragged tails; the full-size
two-class workload is checked on sampled files in the benchmark's launch
configuration."""
import numpy as np
import pytest
import torch

import paper_1905_13746_amd as nbg
from oracle import nb, precision as P
from synth import workloads as W
from tests.parity import X_I32, assert_scores, assert_tables, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _train_pair(wl, n_train, kind, device=DEV):
    X, y = wl.train_set(n_train, device=device)
    m = nbg.Model(wl.n_classes, wl.n_features, kind, device=device)
    nbg.train(m, X, y, alpha=1.0, min_files=1)
    om = nb.train(to_np(X), to_np(y), wl.n_classes, kind, alpha=1.0)
    return m, om


def test_generator_gpu_equals_cpu():
    wl = W.binary_u8(500)
    Xg, yg = wl.test_set(3000, device=DEV)
    Xc, yc = wl.test_set(3000, device="cpu")
    assert (to_np(yg) == to_np(yc)).all() and (to_np(Xg) == to_np(Xc)).all()
    t = W.tiny_int32()
    assert (to_np(t.train_set(500, device=DEV)[0]) == to_np(t.train_set(500)[0])).all()


CASES = [("tiny_int32", W.tiny_int32, W.TINY_TRAIN, W.TINY_TEST)] + [
    (f"binary_u8_F{F}", (lambda F=F: W.binary_u8(F)), 20_000 + 37, 6_000 + 5) for F in (100, 500, 1000, 5000)] + [
    ("near_tie_u8_F1000", W.near_tie_u8, 20_000 + 37, 30_000 + 5)]


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
@pytest.mark.parametrize("name,make,n_train,n_test", CASES, ids=[c[0] for c in CASES])
def test_train_and_score(name, make, n_train, n_test, kind):
    _case(f"train+score {name} {kind}")
    wl = make()
    m, om = _train_pair(wl, n_train, kind)
    assert m.trained
    assert_tables(m, om, kind)
    Xt, _ = wl.test_set(n_test, device=DEV)
    lab, lp, sc = nbg.score(m, Xt, scores=True)
    torch.cuda.synchronize()
    assert_scores(om, to_np(Xt), to_np(lab), to_np(lp), to_np(sc))
    # labels/log-posteriors alone take the one-row path; identical files give
    # identical outputs within the same bounds
    lab1, lp1, _ = nbg.score(m, Xt)
    assert_scores(om, to_np(Xt), to_np(lab1), to_np(lp1), None)


@pytest.mark.parametrize("F,ld", [(100, 128), (1000, 1004), (64, 68), (500, 2048)])
@pytest.mark.parametrize("n", [1, 7, 63, 64, 65, 127, 1001])
def test_ragged_rows_and_strides(F, ld, n):
    _case(f"ragged F={F} ld={ld} n={n}")
    wl = W.binary_u8(F)
    m, om = _train_pair(wl, 4000, nb.MULTINOMIAL)
    X, _ = wl.test_set(n + 3, device=DEV)
    buf = torch.zeros((n + 3) * ld, dtype=torch.uint8, device=DEV)
    wide = buf[: (n + 2) * ld + F].as_strided((n + 3, F), (ld, 1))
    wide.copy_(X)
    # a view that starts one row in and ends exactly at the last feature
    view = buf[ld: ld + (n - 1) * ld + F].as_strided((n, F), (ld, 1))
    lab, lp, sc = nbg.score(m, view, scores=True)
    torch.cuda.synchronize()
    assert_scores(om, to_np(X[1:n + 1]), to_np(lab), to_np(lp), to_np(sc))


def test_int32_strided():
    wl = W.tiny_int32()
    m, om = _train_pair(wl, 2000, nb.MULTINOMIAL)
    X, _ = wl.test_set(777, device=DEV)
    big = torch.zeros((777, 80), dtype=torch.int32, device=DEV)
    big[:, :64] = X
    lab, lp, sc = nbg.score(m, big[:, :64], scores=True)
    torch.cuda.synchronize()
    assert_scores(om, to_np(X), to_np(lab), to_np(lp), to_np(sc))


# int32 features at widths where a file spans 64 lanes (F = 1000, 1001: the
# last loads of a lane only partly live), several chunks (F = 1500, 5000),
# contiguous and padded rows; test files carry counts well above 255 (every
# other file scaled by 37) and a ragged last block.
INT32_WIDE = [(1000, 1000, 3001), (1001, 1001, 2999), (1500, 1536, 1777), (5000, 5000, 1203)]


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
@pytest.mark.parametrize("F,ld,n", INT32_WIDE, ids=[f"F{f}_ld{ld}_n{n}" for f, ld, n in INT32_WIDE])
def test_int32_two_class_wide(F, ld, n, kind):
    _case(f"int32 two classes F={F} ld={ld} n={n} {kind}")
    wl = W.Workload(wid=8, n_classes=2, n_features=F, p_zero=0.8, clip255=False, group=F)
    m, om = _train_pair(wl, 6000 + 13, kind)
    assert_tables(m, om, kind)
    X, _ = wl.test_set(n, device=DEV)
    X[::2] *= 37
    buf = torch.zeros((n, ld), dtype=torch.int32, device=DEV)
    buf[:, :F] = X
    x = buf[:, :F]
    lab, lp, sc = nbg.score(m, x, scores=True)
    torch.cuda.synchronize()
    assert_scores(om, to_np(X), to_np(lab), to_np(lp), to_np(sc), xtype=X_I32)
    lab1, lp1, _ = nbg.score(m, x)
    torch.cuda.synchronize()
    assert_scores(om, to_np(X), to_np(lab1), to_np(lp1), None, xtype=X_I32)
    # a view that ends exactly at the last feature of the last file
    tight = buf.view(-1)[: (n - 1) * ld + F].as_strided((n, F), (ld, 1))
    lab2, lp2, sc2 = nbg.score(m, tight, scores=True)
    torch.cuda.synchronize()
    assert torch.equal(lab2, lab) and torch.equal(lp2, lp) and torch.equal(sc2, sc)


@pytest.mark.slow
def test_full_size_int32_two_class_sampled():
    """The int32-feature variant of the headline workload as the benchmark
    runs it: 100,000 training files and 1,000,000 test files of F = 1000
    int32 counts, one launch over every file; sampled files against the
    oracle."""
    _case("full size int32 F=1000")
    wl = W.binary_u8(1000)
    X, y = wl.train_set(100_000, device=DEV)
    X = X.to(torch.int32)
    m = nbg.Model(2, 1000, "multinomial")
    nbg.train(m, X, y)
    om = nb.train(to_np(X), to_np(y), 2, nb.MULTINOMIAL)
    assert_tables(m, om, nb.MULTINOMIAL)
    del X
    Xt = wl.test_set(W.BINARY_TEST, device=DEV)[0].to(torch.int32)
    lab, lp, _ = nbg.score(m, Xt)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([rng.choice(W.BINARY_TEST, 20_000, replace=False),
                                    [0, 1, W.BINARY_TEST - 2, W.BINARY_TEST - 1]]))
    it = torch.from_numpy(idx).to(DEV)
    assert_scores(om, to_np(Xt[it]), to_np(lab[it]), to_np(lp[it]), None, xtype=X_I32)


def test_train_on_strided_rows_matches():
    wl = W.binary_u8(100)
    X, y = wl.train_set(5000, device=DEV)
    big = torch.zeros((5000, 132), dtype=torch.uint8, device=DEV)
    big[:, :100] = X
    m = nbg.Model(2, 100, "multinomial")
    nbg.train(m, big[:, :100], y)
    om = nb.train(to_np(X), to_np(y), 2, nb.MULTINOMIAL)
    assert (to_np(m.counts()) == om.counts).all()


def test_batch_composition_is_bitwise_invariant():
    _case("batch invariance")
    wl = W.binary_u8(1000)
    m, _ = _train_pair(wl, 10_000, nb.MULTINOMIAL)
    X, _ = wl.test_set(4096, device=DEV)
    full = nbg.score(m, X, scores=True)
    for a, b in ((0, 1), (5, 6), (100, 1000), (4000, 4096), (17, 2093)):
        part = nbg.score(m, X[a:b], scores=True)
        for u, v in zip(full, part):
            assert torch.equal(u[a:b], v)


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_fp8_features_arithmetic_parity(kind):
    _case(f"fp8 {kind}")
    wl = W.binary_u8(1000)
    m, om = _train_pair(wl, 20_000, kind)
    X, _ = wl.test_set(3000, device=DEV)
    q8 = W.to_fp8_e4m3(X)                      # input encoding (torch cast)
    qv = P.e4m3_value(to_np(q8))               # oracle reads the FP8 values it was given
    lab, lp, sc = nbg.score(m, q8, fp8=True, scores=True)
    torch.cuda.synchronize()
    assert_scores(om, qv, to_np(lab), to_np(lp), to_np(sc))


def test_quantize_kernel_bit_exact():
    x = torch.arange(0, 256, dtype=torch.int32).to(torch.uint8).repeat(37, 1).to(DEV)
    got = to_np(nbg.quantize_fp8(x))
    want, _ = P.quantize_fp8(to_np(x))
    assert (got == want).all()
    X, _ = W.binary_u8(500).test_set(999, device=DEV)
    assert (to_np(nbg.quantize_fp8(X)) == P.quantize_fp8(to_np(X))[0]).all()
    # ragged row ends, unaligned rows (byte path) and strided outputs
    for F, off in ((1001, 0), (37, 0), (100, 1), (16, 3)):
        base = torch.randint(0, 256, (300 * 1040 + 8,), dtype=torch.uint8, device=DEV)
        xv = base[off: off + 299 * 1040 + F].as_strided((300, F), (1040, 1))
        out = torch.full((300, 1048), 7, dtype=torch.uint8, device=DEV)
        nbg.quantize_fp8(xv, out=out[:, :F])
        assert (to_np(out[:, :F]) == P.quantize_fp8(to_np(xv))[0]).all()
        assert (to_np(out[:, F:]) == 7).all()            # nothing written past F


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
@pytest.mark.parametrize("near_tie", [False, True], ids=["binary_u8", "near_tie_u8"])
def test_bf16_table_within_certified_band(kind, near_tie):
    _case(f"bf16 {kind} near_tie={near_tie}")
    wl = W.near_tie_u8(1000) if near_tie else W.binary_u8(1000)
    m, om = _train_pair(wl, 20_000, kind)
    X, _ = wl.test_set(30_000 if near_tie else 5000, device=DEV)
    lab, lp, sc = nbg.score(m, X, wtype=nbg.W_BF16, scores=True)
    torch.cuda.synchronize()
    Xn = to_np(X)
    Wt, b = nb.weight_form(om)
    rows, rb = P.scoring_form(Wt, b)
    rh = P.rne_bf16(rows)
    bh = P.rne_f32(rb)
    band = P.certified_band(rows, rb, rh, bh, Xn, Xn, kind == nb.BERNOULLI, n_terms=om.n_features + 1)
    s = nb.joint_log_likelihood(om, Xn)
    d = nb.decide(s)
    gate = d.margin > np.maximum(1e-3, band)
    assert (to_np(lab)[gate] == d.labels[gate]).all()
    if near_tie:   # the case exists to put files inside the band
        assert (~gate).sum() > 0
    # arithmetic parity against the rounded table itself
    g = (Xn > 0).astype(np.float64) if kind == nb.BERNOULLI else Xn.astype(np.float64)
    exact_h = P.posterior_rows(rh, bh, Xn, kind == nb.BERNOULLI)[:, 0]
    delta = to_np(lp)[:, 1].astype(np.float64) - to_np(lp)[:, 0]
    tol = 1e-4 + 1e-6 * (g @ np.abs(rh[0]) + abs(bh[0])) + 2e-7 * np.abs(exact_h)
    assert (np.abs(delta - exact_h) <= tol).all()


def test_training_errors_detected_on_device():
    wl = W.binary_u8(100)
    X, y = wl.train_set(3000, device=DEV)
    m = nbg.Model(2, 100, "multinomial")
    bad = y.clone()
    bad[1234] = 5
    with pytest.raises(nbg.NBError) as e:
        nbg.train(m, X, bad)
    assert e.value.code == -5 and not m.trained
    few = y.clone()
    few[few == 1] = 0
    few[:3] = 1
    with pytest.raises(nbg.NBError) as e:
        nbg.train(m, X, few, min_files=6)
    assert e.value.code == -3
    nbg.train(m, X, few, min_files=3)
    assert m.trained
    t = W.tiny_int32()
    Xi, yi = t.train_set(500, device=DEV)
    Xi[77, 5] = -1
    mi = nbg.Model(2, 64, "multinomial")
    with pytest.raises(nbg.NBError) as e:
        nbg.train(mi, Xi, yi)
    assert e.value.code == -5
    # asynchronous training reports through nb_model_status
    nbg.train(m, X, bad, asynchronous=True)
    assert nbg.model_status(m) == -5
    # a count above INT32_MAX (int32 features), then a clean run clears the flags
    Xo = Xi.clone()
    Xo[Xo < 0] = 0
    Xo[0, 3] = 1 << 30
    Xo[2, 3] = 1 << 30                     # rows 0 and 2 share class 0
    with pytest.raises(nbg.NBError) as e:
        nbg.train(mi, Xo, yi)
    assert e.value.code == -2 and not mi.trained
    Xo[2, 3] = 7
    nbg.train(mi, Xo, yi)
    assert mi.trained and nbg.model_status(mi) == 0


@pytest.mark.slow
def test_full_size_two_class_sampled():
    """200,000 train / 1,000,000 test files, F = 1000 bytes; every test file is
    scored by the GPU exactly as the benchmark does, the oracle checks a
    sample of 20,000 files plus the first and last rows."""
    _case("full size binary_u8 F=1000")
    wl = W.binary_u8(1000)
    X, y = wl.train_set(W.BINARY_TRAIN, device=DEV)
    m = nbg.Model(2, 1000, "multinomial")
    nbg.train(m, X, y)
    om = nb.train(to_np(X), to_np(y), 2, nb.MULTINOMIAL)
    assert_tables(m, om, nb.MULTINOMIAL)
    del X
    Xt, _ = wl.test_set(W.BINARY_TEST, device=DEV)
    lab, lp, _ = nbg.score(m, Xt)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    idx = np.unique(np.concatenate([rng.choice(W.BINARY_TEST, 20_000, replace=False),
                                    [0, 1, W.BINARY_TEST - 2, W.BINARY_TEST - 1]]))
    it = torch.from_numpy(idx).to(DEV)
    assert_scores(om, to_np(Xt[it]), to_np(lab[it]), to_np(lp[it]), None)
