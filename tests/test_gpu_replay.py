"""The paper's group-wise pipeline end to end on the GPU (sections 3-4):
100 size groups, a model per group with enough files of both classes (the
seven small groups use the next group's model and its features), per-group
top-k feature selection, the k-feature models, the gather of each test
file's selected features, and one grouped classification launch; checked
against the FP64 oracle doing the same steps on the CPU."""
import numpy as np
import pytest
import torch

import paper_1905_13746_amd as nbg
from oracle import groups as og, nb, select
from synth import workloads as W
from tests.parity import assert_scores, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def trained_groups():
    F = W.PAPER_F
    benign, malware, share = W.paper_groups()
    has = np.minimum(benign, malware) >= 6
    full, oms = {}, {}
    for g in np.flatnonzero(has):
        X, y = W.paper_train_set(int(g), F, device=DEV)
        m = nbg.Model(2, F, "multinomial")
        nbg.train(m, X, y, min_files=6)
        full[int(g)] = m
        oms[int(g)] = nb.train(to_np(X), to_np(y), 2, nb.MULTINOMIAL)
    return benign, malware, share, has, full, oms


def test_routing_matches_paper_groups(trained_groups):
    benign, malware, _, has, _, _ = trained_groups
    assert sorted(np.flatnonzero(~has).tolist()) == list(W.PAPER_UNTRAINED)
    lib = nbg.route_groups(np.stack([benign, malware], axis=1), 6)
    assert lib.tolist() == og.route(og.trained_mask(np.stack([benign, malware], axis=1), 6)).tolist()


@pytest.mark.parametrize("k,files", [(20, 768), (200, 768 * 4), (80, 768 * 2)])
def test_pipeline_matches_oracle(trained_groups, k, files):
    _case(f"replay k={k} files={files}")
    benign, malware, share, has, full, oms = trained_groups
    G = len(benign)
    route = nbg.route_groups(np.stack([benign, malware], axis=1), 6)
    tg = sorted(full)
    pos = {g: i for i, g in enumerate(tg)}
    idx = nbg.select_features([full[g] for g in tg], k)
    got_idx = to_np(idx)
    okm = {}
    for g in tg:
        oi = select.select_model_features(oms[g], k)
        assert got_idx[pos[g]].tolist() == oi.tolist(), g
        okm[g] = select.model_on_features(oms[g], oi)
    kms = [nbg.model_on_features(full[g], idx[pos[g]].contiguous()) for g in tg]
    counts = W.split_files(files, share)
    assert counts.sum() == files
    xs, xs_full = [], []
    for g in range(G):
        Xt, _ = W.paper_group_workload(g).test_set(int(counts[g]), device=DEV)
        xs_full.append(Xt)
        xs.append(nbg.gather_features(Xt, idx[pos[int(route[g])]].contiguous()))
    plan = nbg.GroupPlan(kms, [(pos[g] if has[g] else None, xs[g]) for g in range(G)], scores=True)
    plan.launch()
    torch.cuda.synchronize()
    for g in range(G):
        if counts[g] == 0:
            continue
        rg = int(route[g])
        xk = select.gather(to_np(xs_full[g]), select.select_model_features(oms[rg], k))
        assert np.array_equal(to_np(xs[g]), xk), g
        lab, lp, sc = plan.outs[g]
        assert_scores(okm[rg], xk, to_np(lab), to_np(lp), to_np(sc))
    plan.close()
