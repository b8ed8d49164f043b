"""Group-wise Naive Bayes malware detection on MI355X (gfx950).

Thin Python binding of libnbgpu (include/nb.h): argument marshalling only.
torch supplies device memory and streams; every step of training and scoring
runs in the library's HIP kernels.  There is no CPU fallback: if the library
is not built, importing the binding's functions raises.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (BERNOULLI, GAUSSIAN, MULTINOMIAL, NBError, TRAIN_ASYNC, W_BF16, W_F32, X_FP8, X_I32,  # noqa: F401
                   X_U8, check, load)

KIND = {"multinomial": MULTINOMIAL, "bernoulli": BERNOULLI, "gaussian": GAUSSIAN}
_XTYPE = {torch.uint8: X_U8, torch.int32: X_I32, torch.float8_e4m3fn: X_FP8}


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def xtype_of(x: torch.Tensor, fp8: bool = False) -> int:
    if fp8:
        if x.dtype not in (torch.uint8, torch.float8_e4m3fn):
            raise TypeError("FP8 features must be uint8 or float8_e4m3fn storage")
        return X_FP8
    if x.dtype not in _XTYPE:
        raise TypeError(f"unsupported feature dtype {x.dtype}")
    return _XTYPE[x.dtype]


def _rows(x: torch.Tensor):
    if x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("features must be a 2-D row-major tensor with unit column stride")
    return x.shape[0], x.shape[1], x.stride(0)


class Model:
    """A Naive Bayes model held in one device buffer owned by torch."""

    def __init__(self, n_classes: int, n_features: int, kind="multinomial", device="cuda"):
        lib = load()
        self.kind = KIND[kind] if isinstance(kind, str) else int(kind)
        nbytes = lib.nb_model_bytes(n_classes, n_features)
        if nbytes == 0:
            raise ValueError("n_classes must be in [2, 256] and n_features in [1, 2**20]")
        self.buf = torch.zeros(nbytes, dtype=torch.uint8, device=device)
        self.c = _lib.NbModel(self.kind, n_classes, n_features, 0, self.buf.data_ptr())
        self.layout = _lib.NbLayout()
        check(lib.nb_model_layout(n_classes, n_features, ctypes.byref(self.layout)), "nb_model_layout")

    n_classes = property(lambda self: self.c.n_classes)
    n_features = property(lambda self: self.c.n_features)
    trained = property(lambda self: bool(self.c.trained))

    def _view(self, off, dtype, count):
        esz = torch.empty((), dtype=dtype).element_size()
        return self.buf[off:off + esz * count].view(dtype)

    # views into the model buffer (no copies)
    def class_totals(self):
        return self._view(self.layout.off_class_totals, torch.int64, self.n_classes)

    def class_sums(self):
        return self._view(self.layout.off_class_sums, torch.int64, self.n_classes)

    def counts(self):
        C, F = self.n_classes, self.n_features
        return self._view(self.layout.off_counts, torch.int32, C * F).view(C, F)

    def log_theta(self):
        C, F = self.n_classes, self.n_features
        return self._view(self.layout.off_log_theta, torch.float64, C * F).view(C, F)

    def log_1m_theta(self):
        C, F = self.n_classes, self.n_features
        return self._view(self.layout.off_log_1m_theta, torch.float64, C * F).view(C, F)

    def weight(self):
        C, F = self.n_classes, self.n_features
        return self._view(self.layout.off_weight, torch.float64, C * F).view(C, F)

    def bias(self):
        return self._view(self.layout.off_bias, torch.float64, self.n_classes)

    def form_f32(self):
        P, Fp = self.layout.form_rows, self.layout.padded_features
        return self._view(self.layout.off_form_f32, torch.float32, (P + 1) * Fp).view(P + 1, Fp)

    def form_bf16(self):
        P, Fp = self.layout.form_rows, self.layout.padded_features
        return self._view(self.layout.off_form_bf16, torch.int16, (P + 1) * Fp).view(P + 1, Fp)

    def form_bias(self):
        return self._view(self.layout.off_form_bias, torch.float32, self.layout.form_rows + 1)

    # Gaussian models
    def sumsq(self):
        C, F = self.n_classes, self.n_features
        return self._view(self.layout.off_sumsq, torch.int64, C * F).view(C, F)

    def mean(self):
        C, F = self.n_classes, self.n_features
        return self._view(self.layout.off_mean, torch.float64, C * F).view(C, F)

    def var(self):
        C, F = self.n_classes, self.n_features
        return self._view(self.layout.off_var, torch.float64, C * F).view(C, F)

    def form2_f32(self):
        P, Fp = self.layout.form_rows, self.layout.padded_features
        return self._view(self.layout.off_form2_f32, torch.float32, (P + 1) * Fp).view(P + 1, Fp)

    def form2_bf16(self):
        P, Fp = self.layout.form_rows, self.layout.padded_features
        return self._view(self.layout.off_form2_bf16, torch.int16, (P + 1) * Fp).view(P + 1, Fp)

    def epsilon(self):
        return self._view(self.layout.off_epsilon, torch.float64, 1)


def train_workspace(model: Model, n: int, xtype: int = X_U8, device="cuda"):
    nbytes = load().nb_train_workspace_bytes(model.n_classes, model.n_features, n, xtype)
    return torch.empty(max(nbytes, 8), dtype=torch.uint8, device=device)


def train(model: Model, x: torch.Tensor, y: torch.Tensor, alpha: float = 1.0, min_files: int = 1,
          workspace: torch.Tensor | None = None, asynchronous: bool = False, stream=None):
    """Fit `model` on features x [n, F] (uint8 or int32) and int32 labels y."""
    n, F, ld = _rows(x)
    if y.dtype != torch.int32 or y.numel() != n:
        raise ValueError("y must be int32 with one label per row")
    xt = xtype_of(x)
    if workspace is None:
        workspace = train_workspace(model, n, xt, x.device)
    rc = load().nb_train(ctypes.byref(model.c), _ptr(x), xt, n, ld, _ptr(y), float(alpha), int(min_files),
                         _ptr(workspace), workspace.numel(), TRAIN_ASYNC if asynchronous else 0, _stream(stream))
    check(rc, "nb_train")
    return model


def model_status(model: Model, stream=None) -> int:
    return load().nb_model_status(ctypes.byref(model.c), _stream(stream))


def score(model: Model, x: torch.Tensor, wtype: int = W_F32, fp8: bool = False, labels=True, log_post=True,
          scores=False, out=None, stream=None):
    """Score files x [n, F]; returns (labels int32[n], log_post f32[n,C], scores f32[n,C]),
    with None for outputs not requested.  `out` may pass preallocated outputs."""
    n, F, ld = _rows(x)
    C = model.n_classes
    dev = x.device
    if out is not None:
        lab, lp, sc = out
    else:
        lab = torch.empty(n, dtype=torch.int32, device=dev) if labels else None
        lp = torch.empty((n, C), dtype=torch.float32, device=dev) if log_post else None
        sc = torch.empty((n, C), dtype=torch.float32, device=dev) if scores else None
    rc = load().nb_score(ctypes.byref(model.c), _ptr(x), xtype_of(x, fp8), n, ld, int(wtype),
                         _ptr(lab), _ptr(lp), _ptr(sc), _stream(stream))
    check(rc, "nb_score")
    return lab, lp, sc


def quantize_fp8(x: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """FP8-e4m3 bytes of uint8 counts: RNE(min(x, 240))."""
    n, F, ld = _rows(x)
    if x.dtype != torch.uint8:
        raise TypeError("quantize_fp8 takes uint8 counts")
    if out is None:
        out = torch.empty((n, F), dtype=torch.uint8, device=x.device)
    check(load().nb_quantize_fp8(_ptr(x), n, F, ld, _ptr(out), out.stride(0), _stream(stream)),
          "nb_quantize_fp8")
    return out


def select_features(models, k: int, out: torch.Tensor | None = None, stream=None):
    """Top-k features of each trained two-class model by the normalised
    class occurrence difference: int32 [len(models), k], rows ascending."""
    models = list(models)
    arr = (_lib.NbModel * len(models))(*[m.c for m in models])
    if out is None:
        out = torch.empty((len(models), int(k)), dtype=torch.int32, device=models[0].buf.device)
    if out.dtype != torch.int32 or out.dim() != 2 or out.stride(1) != 1:
        raise ValueError("out must be a row-major int32 [n_models, >= k] tensor")
    check(load().nb_select_features(arr, len(models), int(k), _ptr(out), out.stride(0), _stream(stream)),
          "nb_select_features")
    return out


def model_on_features(full: Model, idx: torch.Tensor, alpha: float = 1.0, workspace: torch.Tensor | None = None,
                      asynchronous: bool = False, out: Model | None = None, stream=None) -> Model:
    """The model trained on the features idx (int32, device), built from
    full's counts without its training files (into `out` when given)."""
    if idx.dtype != torch.int32 or idx.dim() != 1 or not idx.is_contiguous():
        raise ValueError("idx must be a contiguous 1-D int32 tensor")
    k = idx.numel()
    m = out if out is not None else Model(full.n_classes, k, full.kind, device=full.buf.device)
    if workspace is None:
        nbytes = load().nb_model_select_workspace_bytes(full.n_classes, k)
        workspace = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=full.buf.device)
    rc = load().nb_model_select(ctypes.byref(full.c), _ptr(idx), k, float(alpha), ctypes.byref(m.c),
                                _ptr(workspace), workspace.numel(), TRAIN_ASYNC if asynchronous else 0,
                                _stream(stream))
    check(rc, "nb_model_select")
    return m


def expand_model(km: Model, idx: torch.Tensor, n_features: int, out: Model | None = None,
                 asynchronous: bool = False, stream=None) -> Model:
    """The k-feature model km widened to n_features: scores full rows as km
    scores their selected features idx (int32, ascending, device)."""
    if idx.dtype != torch.int32 or idx.dim() != 1 or not idx.is_contiguous():
        raise ValueError("idx must be a contiguous 1-D int32 tensor")
    m = out if out is not None else Model(km.n_classes, n_features, km.kind, device=km.buf.device)
    rc = load().nb_model_expand(ctypes.byref(km.c), _ptr(idx), ctypes.byref(m.c),
                                TRAIN_ASYNC if asynchronous else 0, _stream(stream))
    check(rc, "nb_model_expand")
    return m


def gather_features(x: torch.Tensor, idx: torch.Tensor, out: torch.Tensor | None = None, fp8: bool = False,
                    status: torch.Tensor | None = None, stream=None):
    """out[i, j] = x[i, idx[j]] for features x [n, F] and int32 indices idx [k]."""
    n, F, ld = _rows(x)
    if idx.dtype != torch.int32 or idx.dim() != 1 or not idx.is_contiguous():
        raise ValueError("idx must be a contiguous 1-D int32 tensor")
    k = idx.numel()
    if out is None:
        out = torch.empty((n, k), dtype=x.dtype, device=x.device)
    if out.dim() != 2 or out.stride(1) != 1 or out.shape[0] != n or out.shape[1] < k:
        raise ValueError("out must be a row-major [n, >= k] tensor")
    if out.dtype != x.dtype:
        raise TypeError("out must have the dtype of x")
    rc = load().nb_gather_features(_ptr(x), xtype_of(x, fp8), n, F, ld, _ptr(idx), k, _ptr(out), out.stride(0),
                                   _ptr(status), _stream(stream))
    check(rc, "nb_gather_features")
    return out


def route_groups(class_counts, min_files: int = 6):
    """Model index for each size group (host logic; see include/nb.h)."""
    import numpy as np
    cc = np.ascontiguousarray(np.asarray(class_counts, dtype=np.int64))
    G, C = cc.shape
    route = np.empty(G, dtype=np.int32)
    check(load().nb_route_groups(cc.ctypes.data_as(ctypes.c_void_p), G, C, int(min_files),
                                 route.ctypes.data_as(ctypes.c_void_p)), "nb_route_groups")
    return route


def probe_read(buf: torch.Tensor, sink: torch.Tensor | None = None, stream=None):
    """Launch the read-bandwidth probe over buf (contiguous, bytes % 16 == 0)."""
    lib = load()
    if sink is None:
        sink = torch.empty(lib.nb_probe_sink_words(), dtype=torch.int32, device=buf.device)
    check(lib.nb_probe_read(_ptr(buf), buf.numel() * buf.element_size(), _ptr(sink), _stream(stream)),
          "nb_probe_read")
    return sink


class _GroupCall:
    """Marshalling of a grouped call: the models array, one nb_group per group
    and its output tensors (allocated here unless given)."""

    def __init__(self, models, groups, fp8=False, labels=True, log_post=True, scores=False, outs=None):
        if not models or not groups:
            raise ValueError("need at least one model and one group")
        self.models = list(models)
        self.cmodels = (_lib.NbModel * len(self.models))(*[m.c for m in self.models])
        self.xs, self.outs = [], []
        self.cgroups = (_lib.NbGroup * len(groups))()
        self.xtype = None
        for i, (mi, x) in enumerate(groups):
            n, F, ld = _rows(x)
            xt = xtype_of(x, fp8)
            if self.xtype is None:
                self.xtype = xt
            elif xt != self.xtype:
                raise TypeError("all groups must share one feature type")
            if outs is not None:
                lab, lp, sc = outs[i]
            else:
                dev = x.device
                lab = torch.empty(n, dtype=torch.int32, device=dev) if labels else None
                lp = torch.empty((n, 2), dtype=torch.float32, device=dev) if log_post else None
                sc = torch.empty((n, 2), dtype=torch.float32, device=dev) if scores else None
            self.xs.append(x)
            self.outs.append((lab, lp, sc))
            g = self.cgroups[i]
            g.model = -1 if mi is None else int(mi)
            g.reserved = 0
            g.x = x.data_ptr() if n > 0 else None
            g.n, g.ld = n, ld
            g.labels = None if lab is None else lab.data_ptr()
            g.log_post = None if lp is None else lp.data_ptr()
            g.scores = None if sc is None else sc.data_ptr()

    def args(self):
        return self.cmodels, len(self.models), self.cgroups, len(self.cgroups), self.xtype


def score_groups(models, groups, wtype: int = W_F32, fp8: bool = False, labels=True, log_post=True, scores=False,
                 tile_rows: int = 0, outs=None, stream=None, static: bool = False):
    """Score size groups in one launch.  groups: [(model index or None, x [n, F])]
    (None: no model of its own; the next group's model is used).  Returns the
    per-group (labels, log_post, scores) outputs.  static=True calls
    nb_score_groups_static (work list in the library's fixed device array, no
    workspace allocated)."""
    lib = load()
    call = _GroupCall(models, groups, fp8, labels, log_post, scores, outs)
    cm, nm, cg, ng, xt = call.args()
    if static:
        check(lib.nb_score_groups_static(cm, nm, cg, ng, xt, int(wtype), int(tile_rows), _stream(stream)),
              "nb_score_groups_static")
        return call.outs
    ws_bytes = lib.nb_score_groups_workspace_bytes(cm, nm, cg, ng, xt, int(wtype), int(tile_rows))
    if ws_bytes == 0:   # invalid arguments: the call itself reports which
        check(lib.nb_score_groups(cm, nm, cg, ng, xt, int(wtype), int(tile_rows), None, 0, _stream(stream)),
              "nb_score_groups")
        return call.outs    # nothing to score
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=call.xs[0].device)
    check(lib.nb_score_groups(cm, nm, cg, ng, xt, int(wtype), int(tile_rows), _ptr(ws), ws_bytes, _stream(stream)),
          "nb_score_groups")
    return call.outs


class GroupPlan:
    """A fixed grouped call captured once (work list on the device, HIP graph
    of the one persistent launch); launch() replays it."""

    def __init__(self, models, groups, wtype: int = W_F32, fp8: bool = False, labels=True, log_post=True,
                 scores=False, tile_rows: int = 0, tune: bool = False, schedule: str | None = None, outs=None,
                 stream=None):
        """schedule: None (tile_rows > 0: dynamic items; else tuned or the
        default), "static" or "stream" (items of tile_rows files)."""
        lib = load()
        self._lib = lib
        self.call = _GroupCall(models, groups, fp8, labels, log_post, scores, outs)
        cm, nm, cg, ng, xt = self.call.args()
        flags = (_lib.PLAN_TUNE if tune else 0) | {None: 0, "static": _lib.PLAN_STATIC,
                                                   "stream": _lib.PLAN_STREAM}[schedule]
        h = ctypes.c_void_p()
        check(lib.nb_group_plan_create(cm, nm, cg, ng, xt, int(wtype), int(tile_rows), flags, _stream(stream),
                                       ctypes.byref(h)),
              "nb_group_plan_create")
        self.handle = h

    @property
    def outs(self):
        return self.call.outs

    def update(self, models, groups, fp8: bool = False, labels=True, log_post=True, scores=False, outs=None,
               stream=None):
        """A new step: re-point the plan at these groups (same models' kind
        and feature count, same outputs, at most the creation's number of
        groups); the next launch() on the same stream scores them.  Returns
        the new per-group outputs."""
        call = _GroupCall(models, groups, fp8, labels, log_post, scores, outs)
        cm, nm, cg, ng, _ = call.args()
        check(self._lib.nb_group_plan_update(self.handle, cm, nm, cg, ng, _stream(stream)), "nb_group_plan_update")
        # the plan's copies of the old step may still be in flight: keep both
        self._prev, self.call = self.call, call
        return call.outs

    def launch(self, stream=None):
        check(self._lib.nb_group_plan_launch(self.handle, _stream(stream)), "nb_group_plan_launch")

    def info(self) -> dict:
        inf = _lib.NbGroupPlanInfo()
        check(self._lib.nb_group_plan_query(self.handle, ctypes.byref(inf)), "nb_group_plan_query")
        d = {k: getattr(inf, k) for k, _ in inf._fields_}
        d["schedule"] = ("static", "dynamic", "stream")[d["schedule"]]
        return d

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            check(self._lib.nb_group_plan_destroy(self.handle), "nb_group_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve(models, requests, arena: torch.Tensor | None = None, arena_bytes: int = 0, max_batch_requests: int = 64,
          n_streams: int = 4, xtype: int = X_U8, wtype: int = W_F32, device_inputs: bool = False,
          simulate: tuple | None = None):
    """Replay a request trace through the continuous-batching server.

    requests: list of dicts {model, x (tensor [n, F]; host, ideally pinned,
    or device with device_inputs), arrival_s, labels (int32[n] host tensor or
    None), log_post (float32[n, 2] host tensor or None)}.  The arena is a
    device uint8 tensor (or arena_bytes with simulate=(batch_s, bytes_per_s),
    which runs the scheduler with modelled batch times and no device work).
    Returns (stats dict, [(status, done_s)] per request)."""
    lib = load()
    creq = (_lib.NbRequest * len(requests))()
    keep = []
    for i, r in enumerate(requests):
        q = creq[i]
        q.model = int(r["model"])
        x = r.get("x")
        q.x = None if x is None else x.data_ptr()
        q.n = int(r["n"]) if x is None else x.shape[0]
        q.arrival_s = float(r["arrival_s"])
        lab, lp = r.get("labels"), r.get("log_post")
        q.labels_host = None if lab is None else lab.data_ptr()
        q.log_post_host = None if lp is None else lp.data_ptr()
        keep.append((x, lab, lp))
    cfg = _lib.NbServeCfg()
    if simulate is not None:
        cfg.arena, cfg.arena_bytes = None, int(arena_bytes)
        cfg.sim_batch_s, cfg.sim_bytes_per_s = float(simulate[0]), float(simulate[1])
    else:
        cfg.arena, cfg.arena_bytes = arena.data_ptr(), arena.numel() * arena.element_size()
    cfg.max_batch_requests, cfg.n_streams = int(max_batch_requests), int(n_streams)
    cfg.xtype, cfg.wtype = int(xtype), int(wtype)
    cfg.flags = (_lib.SERVE_DEVICE_INPUTS if device_inputs else 0) | (_lib.SERVE_SIMULATE if simulate else 0)
    cmodels = (_lib.NbModel * len(models))(*[m.c if hasattr(m, "c") else m for m in models])
    st = _lib.NbServeStats()
    check(lib.nb_serve(cmodels, len(models), creq, len(requests), ctypes.byref(cfg), ctypes.byref(st)), "nb_serve")
    stats = {k: getattr(st, k) for k, _ in st._fields_ if k != "reserved"}
    return stats, [(creq[i].status, creq[i].done_s) for i in range(len(requests))]
