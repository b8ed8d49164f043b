"""The serving scheduler on the CPU (simulation mode: the same admission,
batching and arena logic as on the device, with modelled batch times and no
device calls).  Checks the invariants of continuous batching: every request
is served or rejected, rejection exactly when a request cannot fit an empty
arena, the arena is never over-committed, no more batches in flight than
streams, arrival order without overtaking, exact modelled latencies and the
reported percentiles."""
import numpy as np
import pytest

import paper_1905_13746_amd as nbg
from paper_1905_13746_amd import _lib
from synth import workloads as W

FAKE = 0x7F0000000000
A = 256


def _up(v):
    return (v + A - 1) // A * A


def footprint(n, F, lab=True, lp=True, device_inputs=False):
    """Device bytes a request needs alone: inputs, outputs, work-list bound."""
    x = 0 if device_inputs else _up(n * F)
    wl = _up(256 + 16 * (n // 32 + 2) + 4 * A)
    return x + (_up(4 * n) if lab else 0) + (_up(8 * n) if lp else 0) + wl


def models(fs):
    return [_lib.NbModel(0, 2, f, 0, FAKE) for f in fs]


def reqs(sizes, mids, arrivals, lab=True, lp=True):
    return [{"model": int(m), "x": None, "n": int(n), "arrival_s": float(t),
             "labels": _Fake() if lab else None, "log_post": _Fake() if lp else None}
            for n, m, t in zip(sizes, mids, arrivals)]


class _Fake:
    """Stands in for a host tensor: the simulation never touches outputs."""

    def data_ptr(self):
        return FAKE


def run(ms, rs, arena_bytes, batch_s=1e-4, rate=1e10, **kw):
    return nbg.serve(ms, rs, arena_bytes=arena_bytes, simulate=(batch_s, rate), **kw)


def test_single_request_latency_is_the_model():
    ms = models([1000])
    st, out = run(ms, reqs([100], [0], [0.5]), 1 << 30, batch_s=2e-3, rate=1e9)
    status, done = out[0]
    assert status == 0
    assert done == pytest.approx(0.5 + 2e-3 + 100 * 1000 / 1e9, rel=1e-12)
    assert st["served"] == 1 and st["batches"] == 1 and st["p50_s"] == pytest.approx(done - 0.5)


def test_cfg5_trace_invariants():
    sizes, mids, arr = W.serve_requests(3000, qps=20_000.0)
    ms = models(W.SERVE_F)
    arena = 64 << 20
    st, out = run(ms, reqs(sizes, mids, arr), arena, n_streams=4, max_batch_requests=32)
    status = np.array([s for s, _ in out])
    done = np.array([d for _, d in out])
    need = np.array([footprint(n, W.SERVE_F[m]) for n, m in zip(sizes, mids)])
    assert ((status == -8) == (need > arena)).all()                 # rejected iff it can never fit
    assert st["served"] + st["rejected"] == len(sizes)
    assert st["peak_arena_bytes"] <= arena
    assert 1 <= st["max_in_flight"] <= 4
    ok = status == 0
    lat = done[ok] - arr[ok]
    assert (lat > 0).all()
    assert st["p50_s"] == pytest.approx(np.percentile(lat, 50), rel=1e-9)
    assert st["p99_s"] == pytest.approx(np.percentile(lat, 99), rel=1e-9)
    assert st["max_s"] == pytest.approx(lat.max(), rel=1e-12)
    assert st["files_per_s"] == pytest.approx(sizes[ok].sum() / (done[ok].max() - arr.min()), rel=1e-9)


def test_one_stream_keeps_arrival_order():
    rng = np.random.default_rng(3)
    sizes = rng.integers(1, 4097, size=500)
    arr = np.sort(rng.uniform(0, 0.05, size=500))
    st, out = run(models([500, 5000]), reqs(sizes, rng.integers(0, 2, 500), arr), 256 << 20, n_streams=1,
                  max_batch_requests=8)
    done = np.array([d for _, d in out])
    assert (np.diff(done) >= 0).all()              # no overtaking with one stream
    assert st["max_in_flight"] == 1 and st["rejected"] == 0


def test_tight_arena_serialises_and_rejects_only_oversized():
    F = 1000
    sizes = [1000, 5000, 1000, 40, 1000]
    # room for one 1000-file request at a time, never for the 5000-file one
    arena = footprint(1000, F) + footprint(40, F)
    st, out = run(models([F]), reqs(sizes, [0] * 5, [0, 0, 0, 0, 0]), arena, n_streams=4)
    assert [s for s, _ in out] == [0, -8, 0, 0, 0]
    assert st["peak_arena_bytes"] <= arena
    d = [x for _, x in out]
    assert d[0] <= d[2] <= d[4]


def test_batch_size_limit_and_concurrency():
    n = 64
    st, out = run(models([500]), reqs([10] * n, [0] * n, [0.0] * n), 1 << 30, n_streams=2, max_batch_requests=4)
    assert st["batches"] == n // 4 and st["max_in_flight"] == 2


def test_device_inputs_need_no_input_space():
    sizes = [2000] * 3
    arena = footprint(2000, 5000, device_inputs=True) * 3
    st_dev, _ = run(models([5000]), reqs(sizes, [0] * 3, [0] * 3), arena, device_inputs=True)
    assert st_dev["rejected"] == 0
    st_host, out = run(models([5000]), reqs(sizes, [0] * 3, [0] * 3), arena)
    assert all(s == -8 for s, _ in out)


@pytest.mark.parametrize("bad", ["model", "n", "outputs", "arrival", "streams", "batch", "flags", "rate"])
def test_serve_argument_errors(bad):
    ms = models([1000])
    r = reqs([10], [0], [0.0])
    kw = {}
    if bad == "model":
        r[0]["model"] = 3
    elif bad == "n":
        r[0]["n"] = 0
    elif bad == "outputs":
        r[0]["labels"] = r[0]["log_post"] = None
    elif bad == "arrival":
        r[0]["arrival_s"] = -1.0
    elif bad == "streams":
        kw["n_streams"] = 0
    elif bad == "batch":
        kw["max_batch_requests"] = 0
    with pytest.raises(nbg.NBError) as e:
        if bad == "rate":
            nbg.serve(ms, r, arena_bytes=1 << 20, simulate=(0.0, 0.0))
        elif bad == "flags":
            lib = nbg.load()
            cfg = _lib.NbServeCfg(None, 1 << 20, 4, 1, 0, 0, 2 | 8, 0, 0.0, 1e9)
            st = _lib.NbServeStats()
            creq = (_lib.NbRequest * 1)(_lib.NbRequest(0, 0, None, 10, 0.0, FAKE, FAKE, 0.0))
            cm = (_lib.NbModel * 1)(*ms)
            nbg.check(lib.nb_serve(cm, 1, creq, 1, cfg, st), "nb_serve")
        else:
            run(ms, r, 1 << 20, **kw)
    assert e.value.code == -1
