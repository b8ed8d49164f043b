"""Pins for the oracle's reduced-precision mirrors (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import nb, precision as P


def _bf16_val(bits):
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def test_bf16_rne_brute_force_nearest():
    rng = np.random.default_rng(0)
    v = rng.normal(0, 8, 20000) * np.exp2(rng.integers(-20, 20, 20000))
    got = P.rne_bf16(v)
    t = (v.astype(np.float32).view(np.uint32) >> 16).astype(np.int64)
    for i in range(v.size):
        cands = [b & 0xFFFF for b in (t[i] - 1, t[i], t[i] + 1)]
        vals = _bf16_val(cands)
        err = np.abs(vals - v[i])
        best = err.min()
        ok = [b for b, e in zip(cands, err) if e == best]
        want = vals[cands.index(min(ok, key=lambda b: (b & 1, b)))] if len(ok) > 1 else vals[list(err).index(best)]
        assert got[i] == want, (v[i], got[i], want)


def test_bf16_ties_to_even_and_no_double_rounding():
    rng = np.random.default_rng(1)
    bits = rng.integers(0x3C00, 0x4400, 2000)      # values around 2**-7 .. 2**8
    a, b = _bf16_val(bits), _bf16_val(bits + 1)
    mid = (a + b) / 2.0
    even = np.where(bits % 2 == 0, a, b)
    assert (P.rne_bf16(mid) == even).all()
    # just above the midpoint must round up; a route through FP32 would land on
    # the midpoint and then go to even
    up = mid + (b - a) * 2.0 ** -30
    assert (P.rne_bf16(up) == b).all()
    via_f32 = torch.from_numpy(up.astype(np.float32)).to(torch.bfloat16).double().numpy()
    assert (via_f32 != b).any()


def test_f32_rne_matches_numpy_cast():
    rng = np.random.default_rng(2)
    v = rng.normal(0, 100, 100000)
    assert (P.rne_f32(v) == v.astype(np.float32).astype(np.float64)).all()


def test_e4m3_decode_matches_torch():
    allb = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(allb).view(torch.float8_e4m3fn).double().numpy()
    got = P.e4m3_value(allb)
    assert np.array_equal(np.isnan(ref), np.isnan(got))
    ok = ~np.isnan(ref)
    assert (ref[ok] == got[ok]).all()
    assert np.nanmax(got) == 448.0


def test_fp8_quantiser_brute_force():
    x = np.arange(0, 400)
    byte, q = P.quantize_fp8(x, 240.0)
    grid_b = np.arange(0, 0x7F, dtype=np.int64)            # positive finite encodings
    grid_v = P.e4m3_value(grid_b)
    for xi, bi, qi in zip(x, byte, q):
        v = min(float(xi), 240.0)
        err = np.abs(grid_v - v)
        best = np.flatnonzero(err == err.min())
        pick = best[0] if best.size == 1 else [k for k in best if grid_b[k] % 2 == 0][0]
        assert qi == grid_v[pick] and bi == grid_b[pick], (xi, qi, bi)
    # integers are exact through 16; 17 rounds to 16; saturation at 240
    assert (q[:17] == x[:17]).all() and q[17] == 16 and (q[240:] == 240).all()
    assert P.e4m3_value(byte).tolist() == q.tolist()


def test_fp8_quantiser_matches_torch_cast():
    from synth.workloads import to_fp8_e4m3
    x = torch.arange(0, 256, dtype=torch.int32)
    byte, _ = P.quantize_fp8(x.numpy())
    assert (to_fp8_e4m3(x).numpy() == byte).all()


@pytest.mark.parametrize("C", [2, 5])
@pytest.mark.parametrize("kind", [nb.MULTINOMIAL, nb.BERNOULLI])
def test_scoring_form_is_exact_identity(C, kind):
    rng = np.random.default_rng(4)
    F = 30
    y = np.arange(300) % C
    X = rng.poisson(rng.gamma(0.5, 2, (C, F))[y])
    Xt = rng.poisson(1.0, (40, F))
    m = nb.train(X, y, C, kind)
    s = nb.joint_log_likelihood(m, Xt)
    rows, rb = P.scoring_form(*nb.weight_form(m))
    g = Xt if kind == nb.MULTINOMIAL else (Xt > 0)
    post = P.posterior_rows(rows, rb, Xt, kind == nb.BERNOULLI)
    aux = g @ rows[-1] + rb[-1]
    if C == 2:
        np.testing.assert_allclose(post[:, 0], s[:, 1] - s[:, 0], rtol=1e-11, atol=1e-9)
        np.testing.assert_allclose(aux, s[:, 0], rtol=1e-12)
    else:
        np.testing.assert_allclose(post + aux[:, None], s, rtol=1e-12)
        np.testing.assert_allclose(nb.decide(post).log_post, nb.decide(s).log_post, atol=1e-9)


@pytest.mark.parametrize("C", [2, 16])
def test_certified_band_covers_bf16_fp32_scoring(C):
    rng = np.random.default_rng(6)
    F = 256
    y = np.arange(4000) % C
    lam = rng.gamma(0.5, 2, (C, F))
    X = np.minimum(rng.poisson(lam[y]), 255)
    Xt = np.minimum(rng.poisson(lam[np.arange(3000) % C]), 255)
    m = nb.train(X, y, C, nb.MULTINOMIAL)
    rows, rb = P.scoring_form(*nb.weight_form(m))
    rh, bh = P.rne_bf16(rows), P.rne_f32(rb)
    # an FP32 scorer on the rounded table (torch CPU float32 matmul)
    sh = (torch.from_numpy(Xt.astype(np.float32)) @ torch.from_numpy(rh[:-1].T.astype(np.float32))
          + torch.from_numpy(bh[:-1].astype(np.float32))).double().numpy()
    exact = P.posterior_rows(rows, rb, Xt, False)
    band = P.certified_band(rows, rb, rh, bh, Xt, Xt, False, n_terms=F + 1)
    err = np.abs(sh - exact)
    if C == 2:
        assert (err[:, 0] <= band).all()
        lab_h, lab = (sh[:, 0] > 0), (exact[:, 0] > 0)
        margin = np.abs(exact[:, 0])
    else:
        assert (2 * err.max(axis=1) <= band).all()
        lab_h, lab = sh.argmax(1), exact.argmax(1)
        srt = np.sort(exact, 1)
        margin = srt[:, -1] - srt[:, -2]
    assert (lab_h[margin > band] == lab[margin > band]).all()
