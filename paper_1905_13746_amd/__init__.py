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
from ._lib import (BERNOULLI, MULTINOMIAL, NBError, TRAIN_ASYNC, W_BF16, W_F32, X_FP8, X_I32,  # noqa: F401
                   X_U8, check, load)

KIND = {"multinomial": MULTINOMIAL, "bernoulli": BERNOULLI}
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
