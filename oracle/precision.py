"""Reduced-precision mirrors for the oracle (test infrastructure).

The GPU library scores in FP32 accumulation with its table rounded either to
FP32 (the plain path) or to BF16 (reduced precision), and it may take features
as FP8-e4m3 bytes.  These functions state, from the number formats' own
definitions, what those roundings produce, so tests can separate arithmetic
error (GPU vs oracle on the same rounded operands) from rounding error
(oracle on rounded operands vs oracle on exact ones).

Scoring forms.  Posteriors depend on score differences only, so the scorer may
contract against an equivalent table:
  two classes:  row 0 = W_1 - W_0 (bias b_1 - b_0), giving the log-odds
                Delta = s_1 - s_0; aux row = W_0 (bias b_0) recovers s_0.
  C > 2:        row c = W_c - m with m_f = mean_c W_{c,f} (bias b_c - mean b),
                the class-centred scores; aux row = m (bias mean b) restores
                the raw scores, s_c = centred_c + aux.
Both are exact identities of the FP64 weight form s = bias + g(x) @ W.T.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24          # unit roundoff of FP32


def rne_to_bits(a, mant_bits: int, min_exp: int):
    """Round float64 values to a binary format with `mant_bits` stored
    significand bits, round-to-nearest-even, without double rounding.
    `min_exp` is the exponent of the smallest normal number.  Values returned
    as float64 (exactly representable in the target format).  No overflow
    handling: callers keep values inside the format's range."""
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    nz = a != 0
    m, e = np.frexp(a[nz])              # a = m * 2**e, 0.5 <= |m| < 1
    lead = np.maximum(e - 1, min_exp)   # exponent of the leading bit (subnormals clamp)
    quantum = np.ldexp(1.0, lead - mant_bits)
    out[nz] = np.rint(a[nz] / quantum) * quantum   # rint: ties to even
    return out


def rne_bf16(a):
    """BF16 (8 exponent, 7 stored significand bits) RNE directly from FP64."""
    return rne_to_bits(a, 7, -126)


def rne_f32(a):
    """FP32 RNE from FP64 (24-bit significand)."""
    return rne_to_bits(a, 23, -126)


def bf16_bits(v) -> np.ndarray:
    """uint16 bit patterns of values already representable in BF16."""
    f = np.asarray(v, dtype=np.float64).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


# OCP FP8 E4M3 ("e4m3fn"): bias 7, 3 stored significand bits, no infinities,
# largest finite 448, smallest normal 2**-6.
E4M3_BIAS = 7
E4M3_MANT = 3


def e4m3_value(byte) -> np.ndarray:
    """Decode e4m3fn bytes to float64 (NaN for the two NaN encodings)."""
    b = np.asarray(byte, dtype=np.int64)
    s = np.where(b & 0x80, -1.0, 1.0)
    e = (b >> 3) & 0xF
    m = b & 0x7
    val = np.where(e == 0, m / 8.0 * 2.0 ** (1 - E4M3_BIAS),
                   (1.0 + m / 8.0) * np.exp2(e.astype(np.float64) - E4M3_BIAS))
    val = np.where((e == 0xF) & (m == 0x7), np.nan, val)
    return s * val


def quantize_fp8(x, saturate: float = 240.0):
    """Counts -> FP8-e4m3 bytes: min(x, saturate), then RNE onto the e4m3fn
    grid.  Returns (bytes uint8, values float64)."""
    v = np.minimum(np.asarray(x, dtype=np.float64), saturate)
    if v.size and v.min() < 0:
        raise ValueError("counts must be non-negative")
    q = rne_to_bits(v, E4M3_MANT, 1 - E4M3_BIAS)
    byte = np.zeros(q.shape, dtype=np.uint8)
    nz = q > 0
    m, e = np.frexp(q[nz])
    lead = e - 1
    normal = lead >= 1 - E4M3_BIAS
    ebits = np.where(normal, lead + E4M3_BIAS, 0)
    frac = np.where(normal, q[nz] / np.exp2(lead.astype(np.float64)) - 1.0,
                    q[nz] / 2.0 ** (1 - E4M3_BIAS))
    mbits = np.rint(frac * 8.0).astype(np.int64)
    byte[nz] = ((ebits << 3) | mbits).astype(np.uint8)
    return byte, q


def scoring_form(W, bias):
    """FP64 rows of the equivalent scoring table (see module docstring).

    Returns (rows [P+1, F], row_bias [P+1]) with P = 1 for two classes and
    P = C otherwise; the last row is the aux row."""
    W = np.asarray(W, dtype=np.float64)
    bias = np.asarray(bias, dtype=np.float64)
    if W.shape[0] == 2:
        return np.stack([W[1] - W[0], W[0]]), np.array([bias[1] - bias[0], bias[0]])
    m = W.mean(axis=0)
    mb = bias.mean()
    return np.vstack([W - m[None, :], m[None, :]]), np.concatenate([bias - mb, [mb]])


def posterior_rows(rows, row_bias, X, binarize: bool):
    """FP64 scores of the posterior rows only: g(X) @ rows[:-1].T + bias."""
    g = np.asarray(X, dtype=np.float64)
    if binarize:
        g = (g > 0).astype(np.float64)
    return g @ rows[:-1].T + row_bias[None, :-1]


def certified_band(rows64, bias64, rows_hat, bias_hat, X, Xq, binarize: bool,
                   n_terms: int, round_factor: float = 2.0):
    """Per-file bound B_j on the score-difference error of a scorer that uses
    the rounded table (rows_hat, bias_hat) on the rounded features Xq with FP32
    accumulation, relative to the exact FP64 scores on X.

    |error of each posterior row| <= sum_f g(x)|W^ - W| + sum_f |g(x) - g(q)| |W^|
                                     + |b^ - b| + gamma * (sum_f |g(q) W^| + |b^|)
    with gamma = k n u / (1 - k n u) for n accumulated terms in any order and a
    per-addition rounding of at most k units (k = round_factor).  A label can
    differ from the oracle's only where the oracle's margin is below B_j:
    for two classes B_j is the bound of the single log-odds row, otherwise
    twice the largest row bound."""
    g = np.asarray(X, dtype=np.float64)
    gq = np.asarray(Xq, dtype=np.float64)
    if binarize:
        g, gq = (g > 0).astype(np.float64), (gq > 0).astype(np.float64)
    P = rows64.shape[0] - 1
    R, Rh = rows64[:P], rows_hat[:P]
    nu = round_factor * n_terms * U32
    gamma = nu / (1.0 - nu)
    err = (g @ np.abs(Rh - R).T + np.abs(g - gq) @ np.abs(Rh).T
           + np.abs(bias_hat[:P] - bias64[:P])[None, :]
           + gamma * (gq @ np.abs(Rh).T + np.abs(bias_hat[:P])[None, :]))
    if P == 1:
        return err[:, 0]
    return 2.0 * err.max(axis=1)
