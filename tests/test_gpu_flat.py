"""Flat staging of two-class blocks (byte features, more than 512 features):
a block of rows is fetched as one aligned byte range into LDS and each row
read back from there.  The lane mapping and the arithmetic are those of the
direct loads, so the outputs must be bit-identical to the same files scored
through a stride that does not qualify for staging (row stride not a
multiple of 8 bytes), across feature counts, start offsets inside a cache
line, ragged row counts around the block and window boundaries, feature
types, kinds and output sets; and the FP64 oracle bounds hold."""
import numpy as np
import pytest
import torch

import paper_1905_13746_amd as nbg
from oracle import nb
from synth import workloads as W
from tests.parity import assert_scores, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _model(F, kind, n_train=3000):
    wl = W.binary_u8(F)
    X, y = wl.train_set(n_train, device=DEV)
    m = nbg.Model(2, F, kind)
    nbg.train(m, X, y)
    return wl, m, nb.train(to_np(X), to_np(y), 2, kind)


def _strided(X, ld):
    """The rows of X behind a row stride of ld bytes (a fresh buffer)."""
    n, F = X.shape
    buf = torch.zeros((n, ld), dtype=X.dtype, device=X.device)
    buf[:, :F] = X
    return buf[:, :F]


def _eq(a, b):
    for u, v in zip(a, b):
        if v is None:
            assert u is None
        else:
            assert torch.equal(u, v)


# feature counts: one chunk (16 KB and 32 KB windows), two chunks, the
# largest that still stage
FS = [520, 904, 1000, 1016, 1024, 1496, 1800, 2000, 2032]


def _direct_ld(F):
    """A row stride of 4 mod 8 bytes: never staged."""
    return F + 4 if (F + 4) % 8 else F + 8


@pytest.mark.parametrize("F", FS)
@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_flat_equals_direct_loads(F, kind):
    _case(f"flat vs direct F={F} kind={kind}")
    wl, m, om = _model(F, kind)
    # ragged counts around the 16-row block and the staging window; starts
    # at several offsets inside a 128-byte line (rows of the view begin
    # `lead` rows into the buffer)
    Xall, _ = wl.test_set(4200, device=DEV)
    for lead, n in ((0, 4096), (1, 4000 - 1), (3, 2049), (0, 17), (5, 300), (0, 33)):
        X = Xall[lead:lead + n]
        ref = _strided(X, _direct_ld(F))
        for wtype in (nbg.W_F32, nbg.W_BF16):
            for scores in (False, True):
                got = nbg.score(m, X, wtype=wtype, scores=scores)
                want = nbg.score(m, ref, wtype=wtype, scores=scores)
                torch.cuda.synchronize()
                _eq(got, want)
    lab, lp, sc = nbg.score(m, Xall[1:], scores=True)
    torch.cuda.synchronize()
    assert_scores(om, to_np(Xall[1:]), to_np(lab), to_np(lp), to_np(sc))


@pytest.mark.parametrize("F", [1000, 2000])
def test_flat_fp8_features(F):
    """FP8 bytes past a row's last feature belong to the next row (or are
    NaN encodings): the staged path masks them as the direct path does."""
    _case(f"flat fp8 F={F}")
    wl, m, _ = _model(F, nb.MULTINOMIAL)
    X, _ = wl.test_set(3001, device=DEV)
    q = nbg.quantize_fp8(X)
    ref = _strided(q, _direct_ld(F))
    for scores in (False, True):
        got = nbg.score(m, q[1:], wtype=nbg.W_BF16, fp8=True, scores=scores)
        want = nbg.score(m, ref[1:], wtype=nbg.W_BF16, fp8=True, scores=scores)
        torch.cuda.synchronize()
        _eq(got, want)


def test_flat_in_grouped_schedules():
    """The stream schedule runs as the staged sweep (blocks of the
    concatenated groups staged through LDS, groups smaller than a window
    scored as tails); static ranges and dynamic items load directly.  Each
    is bit-identical to each group scored alone, with groups starting at
    arbitrary rows of one buffer."""
    _case("flat grouped F=2000")
    F = 2000
    models, xs = [], []
    base = W.group_workload(0, F).test_set(20000, device=DEV)[0]
    cuts = [0, 7, 300, 301, 4000, 4017, 9000, 15000, 19999, 20000]
    for g in range(len(cuts) - 1):
        X, y = W.group_workload(g, F).train_set(1000, device=DEV)
        mm = nbg.Model(2, F, "multinomial")
        nbg.train(mm, X, y)
        models.append(mm)
        xs.append(base[cuts[g]:cuts[g + 1]])
    groups = list(enumerate(xs))
    # (the stream schedule holds one table row: no raw scores)
    for sched, scores in (("stream", False), ("static", True), (None, True)):
        plan = nbg.GroupPlan(models, groups, scores=scores, schedule=sched, tile_rows=0 if sched else 512)
        info = plan.info()
        assert info["schedule"] == {"stream": "stream", "static": "static", None: "dynamic"}[sched]
        assert info["staged"] == (1 if sched == "stream" else 0)
        plan.launch()
        torch.cuda.synchronize()
        for (g, x), out in zip(groups, plan.outs):
            want = nbg.score(models[g], x, scores=scores)
            torch.cuda.synchronize()
            _eq(out, want)
        plan.close()
