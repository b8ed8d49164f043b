"""GPU parity of per-group feature selection, the k-feature model and the
feature gather (section 3: top-k opcodes per size group by the normalised
malware-benign occurrence difference; section 4: each group trained and
classified on its k features), against the FP64 oracle.

Bars: selected index lists, gathered bytes and counts are integers, so
bit-exact; the k-feature model's tables and scores follow the training and
scoring bars of tests/parity.py."""
import numpy as np
import pytest
import torch

import paper_1905_13746_amd as nbg
from oracle import nb, select
from synth import workloads as W
from tests.parity import assert_scores, assert_tables, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _trained(g, F, n, kind=nb.MULTINOMIAL, int32=False):
    wl = W.Workload(wid=4, n_classes=2, n_features=F, p_zero=0.7, clip255=False, group=g) if int32 \
        else W.group_workload(g, F)
    X, y = wl.train_set(n, device=DEV)
    if (F * X.element_size()) % 4:          # training takes rows of whole dwords: pad the stride
        Xp = torch.zeros((n, (F + 3) // 4 * 4), dtype=X.dtype, device=DEV)
        Xp[:, :F] = X
        X = Xp[:, :F]
    m = nbg.Model(2, F, kind)
    nbg.train(m, X, y)
    return m, nb.train(to_np(X), to_np(y), 2, kind), X, y, wl


# ------------------------------------------------------------------ select

@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
@pytest.mark.parametrize("F,ks", [(1, [1]), (7, [1, 3, 7]), (300, [1, 20, 200, 299, 300]),
                                  (2000, [20, 40, 80, 100, 160, 200, 1999]), (5000, [200, 4096])])
def test_select_matches_oracle(kind, F, ks):
    _case(f"select F={F} {kind}")
    models, oms = [], []
    for g in range(3):
        m, om, *_ = _trained(g, F, 600, kind)
        models.append(m)
        oms.append(om)
    for k in ks:
        idx = to_np(nbg.select_features(models, k))
        for m_i, om in enumerate(oms):
            want = select.select_model_features(om, k)
            assert idx[m_i].tolist() == want.tolist(), (k, m_i)


def test_select_more_models_than_one_launch_and_strided_output():
    """70 models (two launches of up to 64 workgroups), rows written with a
    stride larger than k; the padding is left untouched."""
    _case("select 70 models")
    models, oms = [], []
    for g in range(70):
        m, om, *_ = _trained(g, 64, 120)
        models.append(m)
        oms.append(om)
    out = torch.full((70, 40), -7, dtype=torch.int32, device=DEV)
    nbg.select_features(models, 33, out=out)
    got = to_np(out)
    for i, om in enumerate(oms):
        assert got[i, :33].tolist() == select.select_model_features(om, 33).tolist()
    assert (got[:, 33:] == -7).all()


def test_select_ties_empty_class_and_wide_keys():
    """Exact ties (duplicated columns), a class with no occurrences at all,
    and int32 counts large enough that |T_1 S_0 - T_0 S_1| needs more than
    64 bits."""
    _case("select ties / empty class / wide keys")
    rng = np.random.default_rng(3)
    # duplicated columns: every feature appears twice
    base = rng.poisson(2.0, size=(400, 50)).astype(np.uint8)
    X = np.concatenate([base, base], axis=1)
    y = (np.arange(400) % 2).astype(np.int32)
    # class 1 has no occurrences: S_1 = 0
    Xe = rng.poisson(1.5, size=(300, 92)).astype(np.uint8)
    ye = (np.arange(300) % 2).astype(np.int32)
    Xe[ye == 1] = 0
    # large int32 counts: T up to ~1.9e9, S ~ 1e11, products ~ 2^67
    Xw = rng.integers(0, 4_000_000, size=(500, 120)).astype(np.int32)
    Xw[:, ::7] = 0
    yw = (np.arange(500) % 2).astype(np.int32)
    for name, Xn, yn in (("ties", X, y), ("empty", Xe, ye), ("wide", Xw, yw)):
        xt = torch.from_numpy(Xn).to(DEV)
        m = nbg.Model(2, Xn.shape[1])
        nbg.train(m, xt, torch.from_numpy(yn).to(DEV))
        om = nb.train(Xn, yn, 2, nb.MULTINOMIAL)
        if name == "wide":
            S = om.counts.sum(axis=1)
            assert int(om.counts.max()) * int(S.max()) > 2 ** 64
        for k in (1, 5, 49, 50, 51, Xn.shape[1]):
            if k <= Xn.shape[1]:
                got = to_np(nbg.select_features([m], k))[0]
                assert got.tolist() == select.select_model_features(om, k).tolist(), (name, k)


def test_select_argument_errors():
    m, *_ = _trained(0, 50, 100)
    with pytest.raises(nbg.NBError):
        nbg.select_features([m], 51)
    three = nbg.Model(3, 50)
    with pytest.raises(nbg.NBError):
        nbg.select_features([three], 5)


# ------------------------------------------------------------------ k-feature model

@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
@pytest.mark.parametrize("F,k", [(2000, 200), (1000, 20), (300, 300), (64, 1)])
def test_model_on_features_matches_oracle_and_training(kind, F, k):
    _case(f"k-feature model F={F} k={k} {kind}")
    m, om, X, y, wl = _trained(5, F, 1500, kind)
    idx = nbg.select_features([m], k)[0].contiguous()
    mk = nbg.model_on_features(m, idx)
    assert mk.trained and mk.n_features == k
    omk = select.model_on_features(om, to_np(idx))
    assert_tables(mk, omk, kind)
    # the same model as training on the gathered files (same counts, same
    # table kernels): bit-identical buffers from the counts on
    def padded(n):   # rows of a multiple of 4 bytes, as training and scoring take them
        return torch.empty((n, (k + 3) // 4 * 4), dtype=X.dtype, device=DEV)
    Xg = nbg.gather_features(X, idx, out=padded(X.shape[0]))[:, :k]
    mt = nbg.Model(2, k, kind)
    nbg.train(mt, Xg, y)
    for part in ("counts", "class_totals", "class_sums", "log_theta", "weight", "bias", "form_f32", "form_bf16",
                 "form_bias"):
        assert torch.equal(getattr(mk, part)(), getattr(mt, part)()), part
    # scoring the gathered test files with the k-feature model
    Xt, _ = wl.test_set(3001, device=DEV)
    Xtg = nbg.gather_features(Xt, idx, out=padded(Xt.shape[0]))[:, :k]
    lab, lp, sc = nbg.score(mk, Xtg, scores=True)
    assert_scores(omk, select.gather(to_np(Xt), to_np(idx)), to_np(lab), to_np(lp), to_np(sc))


def test_model_on_features_rejects_bad_index():
    _case("k-feature model bad index")
    m, *_ = _trained(1, 100, 200)
    bad = torch.tensor([3, 100, 7], dtype=torch.int32, device=DEV)
    with pytest.raises(nbg.NBError) as e:
        nbg.model_on_features(m, bad)
    assert e.value.code == -5
    neg = torch.tensor([-1], dtype=torch.int32, device=DEV)
    with pytest.raises(nbg.NBError):
        nbg.model_on_features(m, neg)
    # repeats and any order are allowed
    rep = torch.tensor([9, 2, 9, 0], dtype=torch.int32, device=DEV)
    mk = nbg.model_on_features(m, rep)
    assert torch.equal(mk.counts(), m.counts()[:, rep.long()])


# ------------------------------------------------------------------ expand

def _padded_rows(X, F):
    """X [n, F] on rows of whole dwords (the stride training and scoring take)."""
    if (F * X.element_size()) % 4 == 0:
        return X
    Xp = torch.zeros((X.shape[0], (F + 3) // 4 * 4), dtype=X.dtype, device=DEV)
    Xp[:, :F] = X
    return Xp[:, :F]


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
@pytest.mark.parametrize("F,k", [(2000, 200), (1000, 20), (300, 300), (7, 3), (1025, 1)])
def test_expanded_model_scores_full_rows(kind, F, k):
    _case(f"expanded model F={F} k={k} {kind}")
    m, om, X, y, wl = _trained(6, F, 1500, kind)
    idx = nbg.select_features([m], k)[0].contiguous()
    mk = nbg.model_on_features(m, idx)
    me = nbg.expand_model(mk, idx, F)
    assert me.trained and me.n_features == F
    ii = idx.long()
    rest = torch.ones(F, dtype=torch.bool, device=DEV)
    rest[ii] = False
    # tables and rows: the k-feature model's at the selected features, zero elsewhere
    for part in ("counts", "log_theta", "weight") + (("log_1m_theta",) if kind == nb.BERNOULLI else ()):
        full, small = getattr(me, part)(), getattr(mk, part)()
        assert torch.equal(full[:, ii], small), part
        assert not full[:, rest].any(), part
    for part in ("form_f32", "form_bf16"):
        full, small = getattr(me, part)(), getattr(mk, part)()
        assert torch.equal(full[:, ii], small[:, :k]), part
        assert not full[:, :F][:, rest].any() and not full[:, F:].any(), part
    for part in ("class_totals", "class_sums", "bias", "form_bias"):
        assert torch.equal(getattr(me, part)(), getattr(mk, part)()), part
    ome = select.expanded_model(select.model_on_features(om, to_np(idx)), to_np(idx), F)
    Xt, _ = wl.test_set(3001, device=DEV)
    Xt = _padded_rows(Xt, F)
    for wtype in (nbg.W_F32, nbg.W_BF16):
        lab, lp, sc = nbg.score(me, Xt, wtype=wtype, scores=True)
        torch.cuda.synchronize()
        assert_scores(ome, to_np(Xt), to_np(lab), to_np(lp), to_np(sc), wtype=wtype)


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_expanded_models_in_one_grouped_launch(kind):
    """Size groups scored on their full rows with expanded k-feature models,
    one launch, against the oracle; a group without a model takes the next."""
    _case(f"expanded models grouped {kind}")
    F, k = 1000, 80
    ms, oms, wls = [], [], []
    for g in range(3):
        m, om, _, _, wl = _trained(10 + g, F, 1200, kind)
        idx = nbg.select_features([m], k)[0].contiguous()
        ms.append(nbg.expand_model(nbg.model_on_features(m, idx), idx, F))
        oms.append(select.expanded_model(select.model_on_features(om, to_np(idx)), to_np(idx), F))
        wls.append(wl)
    xs = [wls[g].test_set(n, device=DEV)[0] for g, n in enumerate((777, 2048, 5))]
    x3 = wls[2].test_set(300, device=DEV)[0]
    outs = nbg.score_groups(ms, [(0, xs[0]), (1, xs[1]), (None, x3), (2, xs[2])], scores=True)
    torch.cuda.synchronize()
    for (lab, lp, sc), x, om in zip(outs, (xs[0], xs[1], x3, xs[2]), (oms[0], oms[1], oms[2], oms[2])):
        assert_scores(om, to_np(x), to_np(lab), to_np(lp), to_np(sc))


def test_expand_rejects_bad_index_lists():
    _case("expand bad index")
    m, *_ = _trained(1, 100, 300)
    idx = torch.tensor([3, 7, 50], dtype=torch.int32, device=DEV)
    mk = nbg.model_on_features(m, idx)
    for bad in ([3, 50, 7], [3, 7, 7], [3, 7, 100], [-1, 7, 50]):
        with pytest.raises(nbg.NBError) as e:
            nbg.expand_model(mk, torch.tensor(bad, dtype=torch.int32, device=DEV), 100)
        assert e.value.code == -5, bad
    with pytest.raises(nbg.NBError):                 # fewer features than the k-feature model
        nbg.expand_model(mk, idx, 2)
    me = nbg.expand_model(mk, idx, 60)               # any width that holds the indices
    assert me.trained and torch.equal(me.counts()[:, idx.long()], mk.counts())


# ------------------------------------------------------------------ gather

def _x(dtype, n, F, ld, seed):
    g = torch.Generator().manual_seed(seed)
    if dtype == torch.int32:
        full = torch.randint(0, 1 << 30, (n, ld), generator=g, dtype=torch.int32)
    else:
        full = torch.randint(0, 256, (n, ld), generator=g, dtype=torch.uint8)
    return full.to(DEV)[:, :F]


GATHER_CASES = [
    # (dtype, n, F, ld, k, order)  order: "sorted", "random", "repeats"
    (torch.uint8, 1000, 1000, 1000, 200, "sorted"),      # one 1 KB load per row, 4 rows per wave
    (torch.uint8, 3001, 2000, 2000, 200, "sorted"),      # 2 loads per row, ragged row count
    (torch.uint8, 777, 2000, 2048, 2000, "random"),      # padded stride, every feature
    (torch.uint8, 501, 5000, 5000, 2048, "repeats"),     # 8 loads per row, all register indices
    (torch.uint8, 300, 4100, 4100, 2049, "random"),      # more than 2048 indices
    (torch.uint8, 64, 9000, 9000, 300, "random"),        # row above 8 KB: global gather
    (torch.uint8, 257, 1001, 1001, 257, "random"),       # odd stride: not dword aligned
    (torch.uint8, 5, 7, 7, 3, "random"),                 # tiny, ragged tails everywhere
    (torch.uint8, 1, 1, 1, 1, "sorted"),
    (torch.uint8, 1003, 1000, 1000, 202, "random"),      # staged, last group of two outputs
    (torch.uint8, 97, 2000, 2000, 21, "sorted"),         # staged, last group of one output
    (torch.int32, 99, 300, 300, 7, "random"),            # staged int32, last group of three
    (torch.int32, 1000, 500, 500, 100, "sorted"),        # 2 KB rows
    (torch.int32, 333, 2048, 2050, 1500, "random"),      # 8 KB rows
    (torch.int32, 100, 2100, 2100, 2100, "repeats"),     # above 8 KB: global gather
    (torch.int32, 9, 3, 3, 5, "repeats"),
]


def _idx(order, F, k, seed):
    rng = np.random.default_rng(seed)
    if order == "sorted":
        v = np.sort(rng.choice(F, size=min(k, F), replace=False))
    elif order == "random":
        v = rng.permutation(F)[:k] if k <= F else rng.integers(0, F, size=k)
    else:
        v = rng.integers(0, F, size=k)
    return v.astype(np.int32)


@pytest.mark.parametrize("case", GATHER_CASES, ids=lambda c: f"{str(c[0])[6:]}-n{c[1]}-F{c[2]}-ld{c[3]}-k{c[4]}-{c[5]}")
def test_gather_matches_oracle(case):
    dtype, n, F, ld, k, order = case
    _case(f"gather {case}")
    x = _x(dtype, n, F, ld, seed=n + F + k)
    idx_np = _idx(order, F, k, seed=F * 7 + k)
    assert idx_np.size == k
    idx = torch.from_numpy(idx_np).to(DEV)
    out = nbg.gather_features(x, idx)
    torch.cuda.synchronize()
    want = select.gather(to_np(x), idx_np)
    assert np.array_equal(to_np(out), want)


def test_gather_fp8_strided_and_unaligned_output():
    _case("gather fp8 / output stride / unaligned output")
    x = _x(torch.uint8, 500, 1000, 1000, seed=1)
    q = nbg.quantize_fp8(x)
    idx_np = _idx("random", 1000, 130, seed=2)
    idx = torch.from_numpy(idx_np).to(DEV)
    out = torch.full((500, 150), 0xAB, dtype=torch.uint8, device=DEV)
    nbg.gather_features(q, idx, out=out, fp8=True)
    got = to_np(out)
    assert np.array_equal(got[:, :130], select.gather(to_np(q), idx_np))
    assert (got[:, 130:] == 0xAB).all()
    # output rows at an odd byte offset and odd stride: byte stores
    raw = torch.full((500 * 131 + 1,), 0xCD, dtype=torch.uint8, device=DEV)
    view = raw[1:].view(500, 131)
    nbg.gather_features(x, idx, out=view)
    assert np.array_equal(to_np(view)[:, :130], select.gather(to_np(x), idx_np))
    assert (to_np(view)[:, 130] == 0xCD).all() and int(to_np(raw[:1])[0]) == 0xCD


def test_gather_flags_bad_indices():
    _case("gather bad index")
    x = _x(torch.uint8, 100, 64, 64, seed=4)
    idx_np = np.array([0, 63, 64, -1, 5], dtype=np.int32)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    out = nbg.gather_features(x, torch.from_numpy(idx_np).to(DEV), status=status)
    got = to_np(out)
    xn = to_np(x)
    assert (got[:, [0, 1, 4]] == xn[:, [0, 63, 5]]).all()
    assert (got[:, 2] == 0).all() and (got[:, 3] == 0).all()
    assert int(status.item()) & 1
    ok = torch.zeros(1, dtype=torch.int32, device=DEV)
    nbg.gather_features(x, torch.tensor([1, 2], dtype=torch.int32, device=DEV), status=ok)
    assert int(ok.item()) == 0
    # no files: nothing launched, nothing written
    e = nbg.gather_features(x[:0], torch.tensor([1], dtype=torch.int32, device=DEV))
    assert e.shape == (0, 1)


@pytest.mark.slow
def test_gather_full_size_sampled():
    """A million files of 2000 byte features, top 200 (the benchmark's
    gather), checked on sampled rows; plus the last rows of the buffer."""
    _case("gather full size")
    n, F, k = 1_000_000, 2000, 200
    x = torch.randint(0, 256, (n, F), dtype=torch.uint8, device=DEV)
    idx_np = np.sort(np.random.default_rng(9).choice(F, size=k, replace=False)).astype(np.int32)
    out = nbg.gather_features(x, torch.from_numpy(idx_np).to(DEV))
    rows = np.concatenate([np.random.default_rng(10).choice(n, 2000, replace=False), np.arange(n - 5, n)])
    ri = torch.from_numpy(rows).to(DEV)
    assert np.array_equal(to_np(out[ri]), select.gather(to_np(x[ri]), idx_np))
