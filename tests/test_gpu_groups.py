"""GPU parity of batched size-group scoring (one persistent launch over the
work items of many groups, each with its own two-class model; groups
without a model borrow the next group's).  Checked against each group scored
alone through nb_score (bit-identical: same per-file summation order), the
FP64 oracle, graph replays against the eager call, and tile invariance."""
import os

import numpy as np
import pytest
import torch

import paper_1905_13746_amd as nbg
from oracle import groups as og, nb
from synth import workloads as W
from tests.parity import X_FP8, X_I32, X_U8, assert_scores, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(msg):
    print(f"[case] {msg}", flush=True)


# group sizes: empty, single file, ragged around the 8-file block, larger
SIZES = [0, 1, 7, 8, 9, 300, 1001, 2500, 64, 33]
HAS_MODEL = [True, True, False, True, True, False, True, True, True, False]


def _build(F, kind, sizes=SIZES, has=HAS_MODEL, xdtype=torch.uint8, fp8=False, train_files=1200):
    """Train one model per group that has one; make each group's test files."""
    models, oms, gmodel, xs, xs_oracle = [], [], [], [], []
    for g, (n, h) in enumerate(zip(sizes, has)):
        wl = W.group_workload(g, F) if xdtype == torch.uint8 else W.Workload(
            wid=4, n_classes=2, n_features=F, p_zero=0.7, clip255=False, group=g)
        if h:
            X, y = wl.train_set(train_files, device=DEV)
            m = nbg.Model(2, F, kind)
            nbg.train(m, X, y)
            oms.append(nb.train(to_np(X), to_np(y), 2, kind))
            gmodel.append(len(models))
            models.append(m)
        else:
            gmodel.append(None)
        Xt, _ = wl.test_set(n, device=DEV)
        if fp8:
            q = W.to_fp8_e4m3(Xt)
            xs.append(q)
            from oracle import precision as P
            xs_oracle.append(P.e4m3_value(to_np(q)))
        else:
            xs.append(Xt)
            xs_oracle.append(to_np(Xt))
    route = og.route(np.array(has))
    return models, oms, gmodel, xs, xs_oracle, route


def _alone(models, gmodel, route, xs, g, wtype, fp8, scores=True):
    m = models[gmodel[route[g]]]
    return nbg.score(m, xs[g], wtype=wtype, fp8=fp8, scores=scores)


def _assert_equal(got, want):
    for u, v in zip(got, want):
        if v is None:
            assert u is None
        else:
            assert torch.equal(u, v)


@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
@pytest.mark.parametrize("wtype", [nbg.W_F32, nbg.W_BF16])
def test_groups_match_alone_and_oracle(kind, wtype):
    _case(f"groups F=2000 {kind} wtype={wtype}")
    F = 2000
    models, oms, gmodel, xs, xo, route = _build(F, kind)
    outs = nbg.score_groups(models, list(zip(gmodel, xs)), wtype=wtype, scores=True)
    torch.cuda.synchronize()
    for g in range(len(SIZES)):
        if SIZES[g] == 0:
            continue
        _assert_equal(outs[g], _alone(models, gmodel, route, xs, g, wtype, False))
        om = oms[gmodel[route[g]]]
        lab, lp, sc = outs[g]
        assert_scores(om, xo[g], to_np(lab), to_np(lp), to_np(sc), wtype=wtype)


def test_fallback_routing_is_the_group_rule():
    # the library's routing equals the oracle's next-then-previous rule
    r = og.route(np.array(HAS_MODEL))
    assert list(r) == [0, 1, 3, 3, 4, 6, 6, 7, 8, 8]


@pytest.mark.parametrize("F,xdtype,fp8", [(100, torch.uint8, False), (1000, torch.uint8, False),
                                          (64, torch.int32, False), (1000, torch.int32, False),
                                          (1500, torch.int32, False), (500, torch.uint8, True),
                                          (5000, torch.uint8, False)],
                         ids=["F100_u8", "F1000_u8", "F64_i32", "F1000_i32", "F1500_i32", "F500_fp8", "F5000_u8"])
def test_groups_other_shapes(F, xdtype, fp8):
    _case(f"groups F={F} {xdtype} fp8={fp8}")
    models, oms, gmodel, xs, xo, route = _build(F, nb.MULTINOMIAL, xdtype=xdtype, fp8=fp8)
    for scores in (False, True):
        outs = nbg.score_groups(models, list(zip(gmodel, xs)), fp8=fp8, scores=scores)
        torch.cuda.synchronize()
        for g in range(len(SIZES)):
            if SIZES[g] == 0:
                continue
            _assert_equal(outs[g], _alone(models, gmodel, route, xs, g, nbg.W_F32, fp8, scores))
            lab, lp, sc = outs[g]
            xt = X_FP8 if fp8 else (X_I32 if xdtype == torch.int32 else X_U8)
            assert_scores(oms[gmodel[route[g]]], xo[g], to_np(lab), to_np(lp),
                          None if sc is None else to_np(sc), xtype=xt)


def test_tile_invariance():
    _case("groups tile invariance")
    models, _, gmodel, xs, _, _ = _build(2000, nb.MULTINOMIAL)
    ref = nbg.score_groups(models, list(zip(gmodel, xs)), scores=True)      # default schedule
    for tile in (1, 8, 40, 1000, 1 << 20):                                  # dynamic items
        got = nbg.score_groups(models, list(zip(gmodel, xs)), scores=True, tile_rows=tile)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            _assert_equal(b, a)


def test_plan_graph_replays_equal_eager():
    _case("groups plan replay")
    models, _, gmodel, xs, _, _ = _build(2000, nb.MULTINOMIAL)
    eager = nbg.score_groups(models, list(zip(gmodel, xs)), scores=True)
    plan = nbg.GroupPlan(models, list(zip(gmodel, xs)), scores=True)
    info = plan.info()
    assert info["n_files"] == sum(SIZES) and info["n_items"] > 0 and info["grid"] >= 1
    assert info["schedule"] in ("stream", "static")
    for rep in range(4):
        for o in plan.outs:
            for t in o:
                if t is not None:
                    t.fill_(-7)
        # unrelated eager work on the same stream between replays
        junk = torch.randn(1 << 20, device=DEV).sum()
        plan.launch()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for g in range(len(SIZES)):
            _assert_equal(plan.outs[g], eager[g])
    plan.close()


@pytest.mark.parametrize("tile", [0, 64])
def test_plan_new_data_in_same_buffers(tile):
    _case(f"groups plan refill tile={tile}")
    models, oms, gmodel, xs, _, route = _build(1000, nb.MULTINOMIAL)
    plan = nbg.GroupPlan(models, list(zip(gmodel, xs)), tile_rows=tile)
    assert plan.info()["schedule"] == ("stream" if tile == 0 else "dynamic")
    for step in range(2):
        for g, x in enumerate(xs):
            if x.shape[0]:
                wl = W.group_workload(g, 1000)
                x.copy_(wl.test_set(x.shape[0], device=DEV, row0=1000 * (step + 1))[0])
        plan.launch()
        torch.cuda.synchronize()
        for g in range(len(SIZES)):
            if SIZES[g]:
                _assert_equal(plan.outs[g], _alone(models, gmodel, route, xs, g, nbg.W_F32, False, False))
    plan.close()


@pytest.mark.parametrize("F,scores", [(2000, False), (1000, True), (100, True), (500, False)])
def test_every_schedule_matches_alone(F, scores):
    """Each schedule a plan can pick (stream at several item sizes, static
    ranges, dynamic items) gives each group nb_score's own results."""
    _case(f"groups schedules F={F} scores={scores}")
    models, _, gmodel, xs, _, route = _build(F, nb.MULTINOMIAL)
    groups = list(zip(gmodel, xs))
    for sched, tile in (("stream", 1), ("stream", 100), ("stream", 5000), ("stream", 0), ("static", 0),
                        (None, 64), (None, 2048)):
        plan = nbg.GroupPlan(models, groups, scores=scores, schedule=sched, tile_rows=tile)
        assert plan.info()["schedule"] == (sched or "dynamic")
        plan.launch()
        torch.cuda.synchronize()
        for g in range(len(SIZES)):
            if SIZES[g]:
                _assert_equal(plan.outs[g], _alone(models, gmodel, route, xs, g, nbg.W_F32, False, scores))
        plan.close()


def test_plan_autotune_and_cache(tmp_path):
    _case("groups plan tune")
    path = str(tmp_path / "tiles.json")
    os.environ["NB_TUNE_CACHE"] = path
    try:
        models, _, gmodel, xs, _, route = _build(2000, nb.MULTINOMIAL)
        groups = list(zip(gmodel, xs))
        p1 = nbg.GroupPlan(models, groups, tune=True)
        i1 = p1.info()
        assert i1["tuned"] == 1 and i1["tile_rows"] % i1["rows_per_block"] == 0
        p1.launch()
        torch.cuda.synchronize()
        for g in range(len(SIZES)):
            if SIZES[g]:
                _assert_equal(p1.outs[g], _alone(models, gmodel, route, xs, g, nbg.W_F32, False, False))
        p2 = nbg.GroupPlan(models, groups, tune=True)
        assert p2.info()["tuned"] == 2 and p2.info()["tile_rows"] == i1["tile_rows"]
        with open(path) as f:
            text = f.read()
        assert "score2_groups/F2000" in text
        p1.close()
        p2.close()
    finally:
        del os.environ["NB_TUNE_CACHE"]


def test_groups_argument_errors():
    models, _, gmodel, xs, _, _ = _build(100, nb.MULTINOMIAL, sizes=[5, 6], has=[True, True], train_files=200)
    with pytest.raises(nbg.NBError) as e:
        nbg.score_groups(models, [(None, xs[0]), (None, xs[1])])
    assert e.value.code == -4                                  # no model anywhere
    other = nbg.Model(2, 200)
    with pytest.raises(nbg.NBError):
        nbg.score_groups([models[0], other], [(0, xs[0]), (1, xs[1])])   # F differs
    three = nbg.Model(3, 100)
    with pytest.raises(nbg.NBError):
        nbg.score_groups([three], [(0, xs[0])])                # not two classes
    with pytest.raises(nbg.NBError):
        nbg.score_groups(models, [(2, xs[0])])                 # index out of range


@pytest.mark.slow
def test_groups_full_size_sampled():
    """The 256-group lognormal workload (F = 2000) in the benchmark's plan
    configuration: whole groups against nb_score alone, sampled files of
    every group against the oracle."""
    sizes = W.group_sizes()
    F = 2000
    rng = np.random.default_rng(11)
    models, oms, xs = [], [], []
    for g, n in enumerate(sizes):
        _case(f"full-size group {g} n={n}") if g % 64 == 0 else None
        wl = W.group_workload(g, F)
        X, y = wl.train_set(min(2 * int(n), 4000), device=DEV)
        m = nbg.Model(2, F, nb.MULTINOMIAL)
        nbg.train(m, X, y)
        models.append(m)
        oms.append((wl, X, y))
        xs.append(wl.test_set(int(n), device=DEV)[0])
    plan = nbg.GroupPlan(models, [(g, x) for g, x in enumerate(xs)], scores=True)
    plan.launch()
    torch.cuda.synchronize()
    for g in range(len(sizes)):
        if g % 16 == 0:
            _assert_equal(plan.outs[g], nbg.score(models[g], xs[g], scores=True))
        wl, X, y = oms[g]
        om = nb.train(to_np(X), to_np(y), 2, nb.MULTINOMIAL)
        idx = rng.choice(int(sizes[g]), size=min(24, int(sizes[g])), replace=False)
        lab, lp, sc = plan.outs[g]
        ii = torch.from_numpy(idx).to(DEV)
        assert_scores(om, to_np(xs[g][ii]), to_np(lab[ii]), to_np(lp[ii]), to_np(sc[ii]))
    plan.close()


def _slices(base, sizes):
    cuts = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    return [base[cuts[i]:cuts[i + 1]] for i in range(len(sizes))]


@pytest.mark.parametrize("F,sched,tile", [(2000, "stream", 0), (1000, "stream", 0), (2000, "static", 0),
                                          (2000, None, 256), (1000, None, 64)],
                         ids=["sweep_F2000", "stream_F1000", "static_F2000", "dynamic_F2000", "dynamic_F1000"])
def test_plan_update_takes_new_steps(F, sched, tile):
    """A plan re-pointed at each step's groups (new sizes, fewer groups, new
    inputs and outputs, empty and untrained groups) replays its captured
    graph with the new work list: every step equals the eager grouped call,
    with two updates and launches queued before anything is awaited."""
    _case(f"plan update F={F} sched={sched} tile={tile}")
    models, _, gmodel, xs, _, _ = _build(F, nb.MULTINOMIAL)
    plan = nbg.GroupPlan(models, list(zip(gmodel, xs)), schedule=sched, tile_rows=tile)
    base = W.group_workload(31, F).test_set(30000, device=DEV)[0]
    steps = [
        ([400, 0, 9000, 17, 2500, 1, 64, 333, 12000, 5], gmodel),                       # same count, new sizes
        ([5000, 3000, 77], [1, None, 0]),                                               # fewer groups
        ([1, 2, 3, 4, 5, 6, 7, 8, 9, 10], [None, 2, None, 0, 1, 3, 5, None, 6, 4]),     # tiny groups
    ]
    queued = []
    for k, (sizes, owners) in enumerate(steps):
        groups = list(zip(owners, _slices(base[(k * 997):], sizes)))
        outs = plan.update(models, groups)
        plan.launch()
        queued.append((groups, outs))
        if len(queued) == 2:      # two steps in flight, then check both
            torch.cuda.synchronize()
            for gr, o in queued:
                want = nbg.score_groups(models, gr)
                torch.cuda.synchronize()
                for a, b in zip(o, want):
                    _assert_equal(a, b)
            queued.clear()
    torch.cuda.synchronize()
    for gr, o in queued:
        want = nbg.score_groups(models, gr)
        torch.cuda.synchronize()
        for a, b in zip(o, want):
            _assert_equal(a, b)
    plan.close()


def test_plan_update_refusals():
    _case("plan update refusals")
    F = 2000
    models, _, gmodel, xs, _, _ = _build(F, nb.MULTINOMIAL, sizes=[300, 40, 2000], has=[True, True, True])
    plan = nbg.GroupPlan(models, list(zip(gmodel, xs)), schedule="stream")
    base = W.group_workload(5, F).test_set(200000, device=DEV)[0]
    with pytest.raises(nbg.NBError) as e:                      # more groups than at creation
        plan.update(models, [(0, base[:10])] * 4)
    assert e.value.code == -1
    with pytest.raises(nbg.NBError) as e:                      # other outputs: another kernel
        plan.update(models, [(0, base[:10])], scores=True)
    assert e.value.code == -1
    other = nbg.Model(2, 1000)
    with pytest.raises(nbg.NBError) as e:                      # another feature count
        plan.update([other], [(0, base[:10, :1000])])
    assert e.value.code == -1
    # a much larger step (the sweep's work list does not grow with the files)
    big = [(0, base[:150000]), (1, base[150000:150001]), (2, base[150001:])]
    outs = plan.update(models, big)
    plan.launch()
    torch.cuda.synchronize()
    for a, b in zip(outs, nbg.score_groups(models, big)):
        _assert_equal(a, b)
    # the plan still serves a valid step after the refusals
    gr = [(0, base[:500]), (None, base[500:800]), (2, base[800:900])]
    outs = plan.update(models, gr)
    plan.launch()
    torch.cuda.synchronize()
    for a, b in zip(outs, nbg.score_groups(models, gr)):
        _assert_equal(a, b)
    plan.close()


def test_score_groups_returns_before_the_device():
    """nb_score_groups enqueues and returns (its work list staged through
    pinned memory): many calls queued back to back, each with its own
    groups and outputs, all equal to the groups scored alone."""
    _case("score_groups asynchronous")
    F = 2000
    models, _, gmodel, xs, _, route = _build(F, nb.MULTINOMIAL)
    base = W.group_workload(17, F).test_set(40000, device=DEV)[0]
    rng = np.random.default_rng(5)
    calls = []
    for k in range(24):
        sizes = rng.integers(0, 3000, size=6)
        owners = [int(v) if v >= 0 else None for v in rng.integers(-1, len(models), size=6)]
        if all(o is None for o in owners):
            owners[0] = 0
        groups = list(zip(owners, _slices(base[int(rng.integers(0, 20000)):], sizes)))
        calls.append((groups, nbg.score_groups(models, groups, scores=True)))
    torch.cuda.synchronize()
    for groups, outs in calls:
        rt = og.route(np.array([o is not None for o, _ in groups]))
        for g, (o, x) in enumerate(groups):
            if x.shape[0] == 0:
                continue
            _assert_equal(outs[g], nbg.score(models[groups[rt[g]][0]], x, scores=True))
