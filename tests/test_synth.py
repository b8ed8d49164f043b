"""The seeded input generators: Philox known answers, chunk independence and
the stated distributions (CPU only)."""
import math

import numpy as np
import pytest
import torch

from synth import philox, workloads as W


@pytest.mark.parametrize("ctr,key,want", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff, 0xffffffff), (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_known_answers(ctr, key, want):
    """Known-answer vectors published with the Random123 library."""
    out = philox.philox4x32(*[torch.tensor([c], dtype=torch.int64) for c in ctr], *key)
    assert tuple(int(o) for o in out) == want


def test_rows_do_not_depend_on_chunking():
    w = W.binary_u8(100)
    X, y = w.train_set(300)
    y2 = w.labels(W.ROLE_TRAIN_Y, 120, 50)
    assert (y2 == y[120:170]).all()
    X2 = w.features(W.ROLE_TRAIN_X, 120, y2)
    assert (X2 == X[120:170]).all()
    X3 = w.features(W.ROLE_TRAIN_X, 0, y, chunk_elems=1000)
    assert (X3 == X).all()


def test_feature_distribution():
    w = W.binary_u8(200)
    X, y = w.train_set(6000)
    assert X.dtype == torch.uint8
    Xn = X.double().numpy()
    for c in range(2):
        mean = Xn[y.numpy() == c].mean(axis=0)
        lam = np.minimum(w.lam[c], 255)
        want = (1 - w.p_zero) * lam
        z = np.abs(mean - want) / np.sqrt((1 - w.p_zero) * lam * (1 + w.p_zero * lam) / 3000 + 1e-12)
        assert np.mean(z < 4.5) > 0.99
    zero = (1 - w.p_zero) * np.exp(-w.lam).mean() + w.p_zero
    assert abs((Xn == 0).mean() - zero) < 0.01


def test_int32_workload_and_priors():
    w = W.tiny_int32()
    X, y = w.train_set(W.TINY_TRAIN)
    assert X.dtype == torch.int32 and X.shape == (2000, 64)
    assert (y.numpy() == np.arange(2000) % 2).all()
    f = W.family16()
    yy = f.labels(W.ROLE_TRAIN_Y, 0, 50000).numpy()
    freq = np.bincount(yy, minlength=16) / yy.size
    assert np.abs(freq - f.prior).max() < 0.01
    assert math.isclose(f.prior.sum(), 1.0)


def test_group_sizes_and_requests():
    n = W.group_sizes()
    assert n.size == 256 and n.min() >= 100 and n.max() <= 100_000
    sizes, models, t = W.serve_requests(5000, 1000.0)
    assert sizes.min() >= 1 and sizes.max() <= 4096 and set(models.tolist()) <= set(range(8))
    assert (np.diff(t) >= 0).all()
