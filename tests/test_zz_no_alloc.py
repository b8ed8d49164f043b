"""nb_score_groups_static (grouped scoring with the work list in the
library's fixed device array, no workspace) against nb_score_groups (caller
workspace): same kernels, so every output must be bit-identical.  Two calls
in a row, the second smaller, so the array's leftover contents from the
first call must not leak into the second; a work list beyond the array's
size is refused before anything is enqueued."""
import ctypes

import pytest
import torch

import paper_1905_13746_amd as nbg
from oracle import nb
from synth import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _models(F, n_models, kind=nb.MULTINOMIAL):
    ms = []
    for g in range(n_models):
        X, y = W.group_workload(g, F).train_set(1200, device=DEV)
        m = nbg.Model(2, F, kind)
        nbg.train(m, X, y)
        ms.append(m)
    return ms


def _groups(F, sizes, models_of, seed_group=0):
    return [(mi, W.group_workload(seed_group + g, F).test_set(n, device=DEV)[0])
            for g, (n, mi) in enumerate(zip(sizes, models_of))]


def _assert_same(a, b):
    for ga, gb in zip(a, b):
        for u, v in zip(ga, gb):
            if v is None:
                assert u is None
            else:
                assert torch.equal(u, v)


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
@pytest.mark.parametrize("tile_rows", [0, 256])
@pytest.mark.parametrize("wtype", [nbg.W_F32, nbg.W_BF16])
def test_static_matches_workspace_twice(kind, tile_rows, wtype):
    F = 2000
    models = _models(F, 3, kind)
    first = _groups(F, [0, 1, 7, 300, 1001, 2500, 64, 33, 9000, 5], [0, 1, None, 2, 0, None, 1, 2, 0, None])
    second = _groups(F, [5, 120, 17], [2, None, 0], seed_group=20)
    for name, groups in (("first", first), ("second (smaller)", second)):
        _case(f"static vs workspace: {name} call, kind={kind} tile_rows={tile_rows} wtype={wtype}")
        want = nbg.score_groups(models, groups, wtype=wtype, scores=True, tile_rows=tile_rows)
        got = nbg.score_groups(models, groups, wtype=wtype, scores=True, tile_rows=tile_rows, static=True)
        torch.cuda.synchronize()
        _assert_same(got, want)
        # and each group's labels match the group scored alone
        for (mi, x), (lab, _, _) in zip(groups, got):
            if x.shape[0] == 0 or mi is None:
                continue
            lab1, _, _ = nbg.score(models[mi], x, wtype=wtype)
            torch.cuda.synchronize()
            assert torch.equal(lab, lab1)


def test_static_int32_features():
    _case("static vs workspace: int32 features F=1000")
    F = 1000
    models = []
    xs = []
    for g in range(2):
        wl = W.Workload(wid=4, n_classes=2, n_features=F, p_zero=0.7, clip255=False, group=g)
        X, y = wl.train_set(1500, device=DEV)
        m = nbg.Model(2, F, nb.MULTINOMIAL)
        nbg.train(m, X, y)
        models.append(m)
        xs.append(wl.test_set(777 + 500 * g, device=DEV)[0])
    groups = [(0, xs[0]), (1, xs[1]), (None, xs[0][:100])]
    for rep in range(2):
        want = nbg.score_groups(models, groups, scores=True)
        got = nbg.score_groups(models, groups, scores=True, static=True)
        torch.cuda.synchronize()
        _assert_same(got, want)
        groups = groups[:1]


def test_static_refuses_work_lists_beyond_the_array():
    """Tens of thousands of one-file groups need a work list larger than the
    fixed array: NB_ENOMEM, with a message, and no output is written."""
    _case("static: oversized work list refused")
    F = 64
    lib = nbg.load()
    models = _models(F, 1)
    n_groups = 40000
    X = W.group_workload(0, F).test_set(n_groups, device=DEV)[0]
    labels = torch.full((n_groups,), -7, dtype=torch.int32, device=DEV)
    outs = [(labels[i:i + 1], None, None) for i in range(n_groups)]
    groups = [(0, X[i:i + 1]) for i in range(n_groups)]
    call = nbg._GroupCall(models, groups, labels=True, log_post=False, outs=outs)
    cm, nm, cg, ng, xt = call.args()
    need = lib.nb_score_groups_workspace_bytes(cm, nm, cg, ng, xt, 0, 0)
    assert need > 4 << 20
    rc = lib.nb_score_groups_static(cm, nm, cg, ng, xt, 0, 0, None)
    assert rc == -6
    assert b"static array" in lib.nb_last_error()
    torch.cuda.synchronize()
    assert bool((labels == -7).all())
    # the same call through a workspace is fine, and a static call after the
    # refusal still works
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    assert lib.nb_score_groups(cm, nm, cg, ng, xt, 0, 0, ctypes.c_void_p(ws.data_ptr()), need, None) == 0
    torch.cuda.synchronize()
    small = [(0, X[:50])]
    want = nbg.score_groups(models, small, scores=True)
    got = nbg.score_groups(models, small, scores=True, static=True)
    torch.cuda.synchronize()
    _assert_same(got, want)
    assert torch.equal(got[0][0], labels[:50])
