"""Philox-4x32-10 counter-based generator, written from its published definition
(Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11).

Implemented with torch integer ops only, so the same code yields bit-identical
words on the CPU and on a GPU device: a test-side row sample regenerated on the
host equals the row the device generated.  Every 32-bit quantity is held in an
int64 tensor and every product is split so that no intermediate exceeds 2**63
(no reliance on wrap-around).

This module draws input data only; it holds none of the classifier's arithmetic.
"""
import torch

MASK32 = 0xFFFFFFFF
# Multipliers and Weyl key increments of Philox-4x32 (SC'11, section 5).
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
ROUNDS = 10


def _mulhilo(a: int, b: torch.Tensor):
    """(hi, lo) 32-bit words of the 64-bit product a*b, a < 2**32 a constant."""
    a_hi, a_lo = a >> 16, a & 0xFFFF
    t = b * a_lo                      # < 2**48
    u = b * a_hi                      # < 2**48
    mid = t + ((u & 0xFFFF) << 16)    # < 2**48 + 2**32
    return (u >> 16) + (mid >> 32), mid & MASK32


def philox4x32(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox rounds on counter words c0..c3 (int64 tensors holding u32),
    key (k0, k1).  Returns the four output words as int64 tensors."""
    for r in range(ROUNDS):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        hi0, lo0 = _mulhilo(PHILOX_M0, c0)
        hi1, lo1 = _mulhilo(PHILOX_M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def element_words(key0: int, key1: int, row0: int, n_rows: int, n_cols: int,
                  device="cpu"):
    """Two independent u32 words per element (i, j) of an n_rows x n_cols
    block whose first row has global index row0.

    Counter of element (i, j) is (j // 2, i mod 2**32, i // 2**32, 0); words
    0,1 of the block go to even j and words 2,3 to odd j.  Returns
    (w_a, w_b), int64 tensors of shape [n_rows, n_cols].
    """
    n_pairs = (n_cols + 1) // 2
    rows = torch.arange(row0, row0 + n_rows, dtype=torch.int64, device=device)
    pairs = torch.arange(n_pairs, dtype=torch.int64, device=device)
    c0 = pairs.unsqueeze(0).expand(n_rows, n_pairs)
    c1 = (rows & MASK32).unsqueeze(1).expand(n_rows, n_pairs)
    c2 = (rows >> 32).unsqueeze(1).expand(n_rows, n_pairs)
    c3 = torch.zeros((), dtype=torch.int64, device=device).expand(n_rows, n_pairs)
    o0, o1, o2, o3 = philox4x32(c0, c1, c2, c3, key0 & MASK32, key1 & MASK32)
    w_a = torch.stack((o0, o2), dim=2).reshape(n_rows, 2 * n_pairs)[:, :n_cols]
    w_b = torch.stack((o1, o3), dim=2).reshape(n_rows, 2 * n_pairs)[:, :n_cols]
    return w_a, w_b
