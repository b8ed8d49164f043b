"""The C ABI library on the CPU: it loads, exports every symbol include/nb.h
declares, computes layouts, validates arguments before touching a device, and
its host-side size-group routing matches the oracle.  No compute call runs."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1905_13746_amd as nbg
from paper_1905_13746_amd import _lib
from oracle import groups

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nb.h")

FAKE_DEV = 0x7F0000000000   # 256-byte aligned; never dereferenced by these tests


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return nbg.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


def test_version_and_layout(lib):
    assert b"gfx950" in lib.nb_version()
    L = _lib.NbLayout()
    assert lib.nb_model_layout(2, 1000, ctypes.byref(L)) == 0
    assert L.padded_features == 1024 and L.form_rows == 1
    offs = [L.off_status, L.off_class_totals, L.off_class_sums, L.off_counts, L.off_log_theta,
            L.off_log_1m_theta, L.off_weight, L.off_bias, L.off_form_f32, L.off_form_bf16, L.off_form_bias]
    assert offs == sorted(offs) and all(o % 256 == 0 for o in offs)
    assert L.off_counts - L.off_class_sums >= 16 and L.off_log_theta - L.off_counts >= 4 * 2000
    assert L.total_bytes == lib.nb_model_bytes(2, 1000)
    assert lib.nb_model_layout(16, 4096, ctypes.byref(L)) == 0 and L.form_rows == 16
    assert lib.nb_model_bytes(1, 10) == 0 and lib.nb_model_bytes(257, 10) == 0
    assert lib.nb_model_bytes(2, 0) == 0
    assert lib.nb_model_layout(1, 10, ctypes.byref(L)) == -1


def _model(C=2, F=100, kind=0):
    return _lib.NbModel(kind, C, F, 0, FAKE_DEV)


def _train(lib, m, **kw):
    a = dict(x=FAKE_DEV, xtype=0, n=10, ld=m.n_features, y=FAKE_DEV, alpha=1.0, minf=1,
             ws=FAKE_DEV, wsb=1 << 30, flags=0)
    a.update(kw)
    return lib.nb_train(ctypes.byref(m), a["x"], a["xtype"], a["n"], a["ld"], a["y"], a["alpha"], a["minf"],
                        a["ws"], a["wsb"], a["flags"], None)


@pytest.mark.parametrize("kw,code", [
    (dict(alpha=0.0), -1), (dict(alpha=float("nan")), -1), (dict(n=0), -1),
    (dict(ld=50), -1), (dict(xtype=2), -1), (dict(xtype=9), -1), (dict(x=None), -1),
    (dict(y=None), -1), (dict(minf=0), -1), (dict(wsb=16), -6), (dict(ws=None), -6),
    (dict(x=FAKE_DEV + 2), -1), (dict(n=9_000_000), -2),
])
def test_train_argument_errors(lib, kw, code):
    assert _train(lib, _model(), **kw) == code
    assert lib.nb_last_error()


def test_train_rejects_bad_models(lib):
    assert _train(lib, _model(C=1)) == -1
    assert _train(lib, _model(kind=5)) == -1
    bad = _lib.NbModel(0, 2, 100, 0, FAKE_DEV + 8)
    assert _train(lib, bad) == -1
    assert lib.nb_train(None, FAKE_DEV, 0, 10, 100, FAKE_DEV, 1.0, 1, FAKE_DEV, 1 << 30, 0, None) == -1


def _score(lib, m, **kw):
    a = dict(x=FAKE_DEV, xtype=0, n=10, ld=m.n_features, wt=0, lab=FAKE_DEV, lp=FAKE_DEV, sc=None)
    a.update(kw)
    return lib.nb_score(ctypes.byref(m), a["x"], a["xtype"], a["n"], a["ld"], a["wt"], a["lab"], a["lp"],
                        a["sc"], None)


@pytest.mark.parametrize("kw,code", [
    (dict(xtype=7), -1), (dict(wt=3), -1), (dict(n=-1), -1), (dict(lab=None, lp=None), -1),
    (dict(x=None), -1), (dict(ld=99), -1), (dict(ld=101), -1), (dict(lp=FAKE_DEV + 4), -1),
])
def test_score_argument_errors(lib, kw, code):
    assert _score(lib, _model(), **kw) == code


def test_odd_byte_width_needs_a_padded_stride(lib):
    """A contiguous byte matrix with F = 513 has rows at every byte offset;
    the rule (include/nb.h) is a stride that is a multiple of 4 bytes, so it
    is refused before anything is enqueued (the padded case is a GPU test)."""
    for C in (2, 7, 16):
        m = _model(C=C, F=513)
        for wt in (0, 1):
            assert _score(lib, m, ld=513, wt=wt) == -1
            assert b"multiple of 4" in lib.nb_last_error()
        assert _train(lib, m, ld=513) == -1
        assert b"multiple of 4" in lib.nb_last_error()
    assert _score(lib, _model(F=513), ld=513, xtype=2) == -1      # FP8 bytes too


def test_score_rejects_strides_beyond_the_staging_range(lib):
    """Every scoring path stages a group of rows through one buffer resource
    with 32-bit offsets: strides whose group spans 2 GiB are refused before
    anything is launched."""
    for C, wt, xtype in ((3, 0, 0), (2, 0, 0), (16, 1, 0), (3, 0, 1)):
        eb = 4 if xtype == 1 else 1
        ld = (1 << 25) // eb
        assert _score(lib, _model(C=C), ld=ld, wt=wt, xtype=xtype) == -1, (C, wt, xtype)
        assert b"stride" in lib.nb_last_error(), (C, wt, xtype)


def test_score_empty_batch_is_noop(lib):
    assert _score(lib, _model(), n=0, x=None) == 0


def test_workspace_size_is_deterministic(lib):
    a = lib.nb_train_workspace_bytes(2, 1000, 200_000, 0)
    assert a > 0 and a == lib.nb_train_workspace_bytes(2, 1000, 200_000, 0)
    assert lib.nb_train_workspace_bytes(1, 1000, 10, 0) == 0


def test_route_groups_matches_oracle(lib):
    rng = np.random.default_rng(0)
    for _ in range(200):
        G, C = int(rng.integers(1, 30)), int(rng.integers(2, 4))
        cc = rng.integers(0, 12, size=(G, C))
        trained = groups.trained_mask(cc, 6)
        if not trained.any():
            with pytest.raises(nbg.NBError):
                nbg.route_groups(cc, 6)
            continue
        assert (nbg.route_groups(cc, 6) == groups.route(trained)).all()


def test_route_groups_paper_fixture():
    import json
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "size_groups.json")))
    cc = np.full((g["n_groups"], 2), 40)
    for k, grp in enumerate(g["untrained_1based"]):
        cc[grp - 1, k % 2] = 3
    r = nbg.route_groups(cc, g["min_files"])
    for grp_s, tgt in g["fallback_1based"].items():
        assert r[int(grp_s) - 1] + 1 == tgt


def _groups_call(lib, models, groups, xtype=0, wtype=0, tile=0):
    cm = (_lib.NbModel * len(models))(*models)
    cg = (_lib.NbGroup * len(groups))(*groups)
    return lib.nb_score_groups(cm, len(models), cg, len(groups), xtype, wtype, tile, FAKE_DEV, 1 << 20, None)


def _group(model, n=10, F=100, **kw):
    g = _lib.NbGroup(model, 0, FAKE_DEV, n, F, FAKE_DEV, FAKE_DEV, None)
    for k, v in kw.items():
        setattr(g, k, v)
    return g


@pytest.mark.parametrize("case,code", [
    ("no_model_anywhere", -4), ("index_out_of_range", -1), ("index_below_minus_one", -1),
    ("three_classes", -1), ("features_differ", -1), ("kinds_differ", -1), ("reserved_set", -1),
    ("bad_xtype", -1), ("bad_wtype", -1), ("negative_n", -1), ("no_outputs", -1), ("ld_too_small", -1),
    ("misaligned_log_post", -1),
])
def test_score_groups_argument_errors(lib, case, code):
    """Every argument error is found on the host before any device work."""
    m2 = [_model(), _model()]
    groups, models, xt, wt = [_group(0), _group(1)], m2, 0, 0
    if case == "no_model_anywhere":
        groups = [_group(-1), _group(-1)]
    elif case == "index_out_of_range":
        groups = [_group(0), _group(2)]
    elif case == "index_below_minus_one":
        groups = [_group(-2)]
    elif case == "three_classes":
        models = [_model(C=3), _model()]
    elif case == "features_differ":
        models = [_model(), _model(F=200)]
    elif case == "kinds_differ":
        models = [_model(), _model(kind=1)]
    elif case == "reserved_set":
        groups = [_group(0, reserved=1)]
    elif case == "bad_xtype":
        xt = 5
    elif case == "bad_wtype":
        wt = 4
    elif case == "negative_n":
        groups = [_group(0, n=-1)]
    elif case == "no_outputs":
        groups = [_group(0, labels=None, log_post=None)]
    elif case == "ld_too_small":
        groups = [_group(0, ld=99)]
    elif case == "misaligned_log_post":
        groups = [_group(0, log_post=FAKE_DEV + 4)]
    assert _groups_call(lib, models, groups, xt, wt) == code
    assert lib.nb_last_error()


def test_group_plan_rejects_before_allocating(lib):
    cm = (_lib.NbModel * 1)(_model())
    cg = (_lib.NbGroup * 1)(_group(-1))
    out = ctypes.c_void_p(1)
    assert lib.nb_group_plan_create(cm, 1, cg, 1, 0, 0, 0, 0, None, ctypes.byref(out)) == -4
    assert not out.value
    cg = (_lib.NbGroup * 1)(_group(0))
    assert lib.nb_group_plan_create(cm, 1, cg, 1, 0, 0, -5, 0, None, ctypes.byref(out)) == -1
    assert lib.nb_group_plan_create(cm, 1, cg, 1, 0, 0, 0, 8, None, ctypes.byref(out)) == -1    # unknown flag
    assert lib.nb_group_plan_create(cm, 1, cg, 1, 0, 0, 0, 2 | 4, None, ctypes.byref(out)) == -1  # two schedules
    assert lib.nb_group_plan_destroy(None) == 0
    assert lib.nb_group_plan_launch(None, None) == -1


def test_selection_argument_errors(lib):
    """Feature selection, k-feature models and the gather validate their
    arguments before touching a device."""
    trained = _model(2, 100)
    trained.trained = 1
    arr = (_lib.NbModel * 1)(trained)
    idx = ctypes.c_void_p(FAKE_DEV)
    assert lib.nb_select_features(arr, 0, 5, idx, 5, None) == -1          # no models
    assert lib.nb_select_features(arr, 1, 5, None, 5, None) == -1         # idx NULL
    assert lib.nb_select_features(arr, 1, 0, idx, 5, None) == -1          # k < 1
    assert lib.nb_select_features(arr, 1, 5, idx, 4, None) == -1          # ld_idx < k
    assert lib.nb_select_features(arr, 1, 101, idx, 101, None) == -1      # k > F
    untrained = (_lib.NbModel * 1)(_model(2, 100))
    assert lib.nb_select_features(untrained, 1, 5, idx, 5, None) == -1
    three = _model(3, 100)
    three.trained = 1
    assert lib.nb_select_features((_lib.NbModel * 1)(three), 1, 5, idx, 5, None) == -1

    assert lib.nb_model_select_workspace_bytes(2, 200) > 0
    assert lib.nb_model_select_workspace_bytes(1, 200) == 0
    assert lib.nb_model_select_workspace_bytes(2, 0) == 0
    ws = ctypes.c_void_p(FAKE_DEV)
    big = 1 << 30
    out = _lib.NbModel(0, 2, 7, 0, FAKE_DEV + (1 << 20))
    assert lib.nb_model_select(ctypes.byref(_model(2, 100)), idx, 7, 1.0, ctypes.byref(out), ws, big, 0,
                               None) == -1                                # full not trained
    assert lib.nb_model_select(ctypes.byref(trained), idx, 8, 1.0, ctypes.byref(out), ws, big, 0, None) == -1
    other_kind = _lib.NbModel(1, 2, 7, 0, FAKE_DEV + (1 << 20))
    assert lib.nb_model_select(ctypes.byref(trained), idx, 7, 1.0, ctypes.byref(other_kind), ws, big, 0,
                               None) == -1
    same_buf = _lib.NbModel(0, 2, 7, 0, FAKE_DEV)
    assert lib.nb_model_select(ctypes.byref(trained), idx, 7, 1.0, ctypes.byref(same_buf), ws, big, 0,
                               None) == -1
    assert lib.nb_model_select(ctypes.byref(trained), None, 7, 1.0, ctypes.byref(out), ws, big, 0, None) == -1
    assert lib.nb_model_select(ctypes.byref(trained), idx, 7, 0.0, ctypes.byref(out), ws, big, 0, None) == -1
    assert lib.nb_model_select(ctypes.byref(trained), idx, 7, 1.0, ctypes.byref(out), ws, 16, 0, None) == -6

    x = ctypes.c_void_p(FAKE_DEV)
    o = ctypes.c_void_p(FAKE_DEV + (1 << 24))
    g = lib.nb_gather_features
    assert g(x, 7, 10, 100, 100, idx, 5, o, 5, None, None) == -1          # unknown type
    assert g(x, 0, 10, 0, 100, idx, 5, o, 5, None, None) == -1            # F < 1
    assert g(x, 0, 10, 100, 100, idx, 0, o, 5, None, None) == -1          # k < 1
    assert g(x, 0, -1, 100, 100, idx, 5, o, 5, None, None) == -1          # n < 0
    assert g(x, 0, 10, 100, 99, idx, 5, o, 5, None, None) == -1           # ld < F
    assert g(x, 0, 10, 100, 100, idx, 5, o, 4, None, None) == -1          # ld_out < k
    assert g(None, 0, 0, 100, 100, None, 5, None, 5, None, None) == 0     # n == 0: no-op
    assert g(None, 0, 10, 100, 100, idx, 5, o, 5, None, None) == -1       # x NULL
    assert g(x, 0, 10, 100, 100, None, 5, o, 5, None, None) == -1         # idx NULL
    assert g(ctypes.c_void_p(FAKE_DEV + 2), 1, 10, 100, 100, idx, 5, o, 5, None, None) == -1  # int32 misaligned
    assert g(x, 0, 10, 100, 100, ctypes.c_void_p(FAKE_DEV + 2), 5, o, 5, None, None) == -1    # idx misaligned


def test_expand_argument_errors(lib):
    km = _model(2, 10)
    km.trained = 1
    idx = ctypes.c_void_p(FAKE_DEV)
    out = _lib.NbModel(0, 2, 100, 0, FAKE_DEV + (1 << 20))
    assert lib.nb_model_expand(ctypes.byref(_model(2, 10)), idx, ctypes.byref(out), 0, None) == -1  # untrained
    assert lib.nb_model_expand(ctypes.byref(km), None, ctypes.byref(out), 0, None) == -1
    assert lib.nb_model_expand(ctypes.byref(km), idx, None, 0, None) == -1
    small = _lib.NbModel(0, 2, 5, 0, FAKE_DEV + (1 << 20))
    assert lib.nb_model_expand(ctypes.byref(km), idx, ctypes.byref(small), 0, None) == -1      # fewer features
    other = _lib.NbModel(1, 2, 100, 0, FAKE_DEV + (1 << 20))
    assert lib.nb_model_expand(ctypes.byref(km), idx, ctypes.byref(other), 0, None) == -1      # kind differs
    same = _lib.NbModel(0, 2, 100, 0, FAKE_DEV)
    assert lib.nb_model_expand(ctypes.byref(km), idx, ctypes.byref(same), 0, None) == -1       # same buffer
    g = _lib.NbModel(2, 2, 10, 1, FAKE_DEV)
    gout = _lib.NbModel(2, 2, 100, 0, FAKE_DEV + (1 << 20))
    assert lib.nb_model_expand(ctypes.byref(g), idx, ctypes.byref(gout), 0, None) == -1        # Gaussian
