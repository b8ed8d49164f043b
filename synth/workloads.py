"""Seeded synthetic stand-ins for the paper's opcode-occurrence data.

The paper's inputs (per-file counts of the top-k opcodes of Malicia malware and
benign Windows executables, section 3) are not available, so every workload here
is synthetic, with the structure the paper describes: per-file non-negative
integer occurrence counts, two classes (benign = 0, malware = 1), size groups
with their own models, and a 2:1 train:test split.

Recipe (all draws reproducible from (SEED, workload id, role, group)):
  * class rates   lam[c, f] ~ Gamma(shape 0.5, scale 2)       (numpy PCG64)
  * class priors  balanced (y_i = i mod C) or Dirichlet(1)     (numpy PCG64)
  * feature x_if  ~ Poisson(lam[y_i, f]), then zero with probability p_zero,
                  then clipped at 255 for byte features.
  * Poisson and zero-mask uniforms come from Philox-4x32-10 (synth.philox):
    element (i, f) of a stream uses words (a, b); u = (2w + 1) / 2**33.
    x = #{k : u_b >= CDF_lam(k)}, computed exactly in integers against
    thresholds ceil(CDF(k) * 2**33); zero iff u_a < p_zero.
The same code runs on CPU and GPU tensors and gives identical bytes.

This module holds no classifier arithmetic: it only draws inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from .philox import element_words

SEED = 190513746
TWO33 = 1 << 33

ROLE_LAMBDA = 0
ROLE_PRIOR = 1
ROLE_TRAIN_Y = 2
ROLE_TRAIN_X = 3
ROLE_TEST_Y = 4
ROLE_TEST_X = 5
ROLE_SIZES = 7
ROLE_REQUESTS = 8


def _np_rng(*spawn_key):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED, spawn_key=spawn_key)))


def _philox_key1(wid: int, group: int, role: int) -> int:
    return ((wid & 0xFF) << 24) | ((group & 0xFFFF) << 8) | (role & 0xFF)


def poisson_search_table(lam: np.ndarray, kmax: int | None):
    """Sorted int64 search keys for inverse-CDF Poisson draws per (c, f).

    Segment s = c*F + f holds s * 2**34 + ceil(CDF(k) * 2**33) for
    k = 0, 1, ... while the threshold is below 2**33 (and k < kmax when the
    features are clipped).  Returns (keys, segment_start)."""
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    kcap = 256 if kmax is None else kmax
    if kmax is None:
        kcap = max(256, int(lam.max() + 12 * math.sqrt(lam.max() + 1) + 32))
    k = np.arange(kcap, dtype=np.float64)
    # pmf by recurrence p_k = p_{k-1} * lam / k in log space for stability
    logp = -lam[:, None] + k[None, :] * np.log(np.maximum(lam[:, None], 1e-300)) \
        - np.array([math.lgamma(v + 1.0) for v in k])[None, :]
    logp[lam == 0.0, 1:] = -np.inf
    logp[lam == 0.0, 0] = 0.0
    cdf = np.cumsum(np.exp(logp), axis=1)
    thr = np.ceil(cdf * TWO33)
    valid = thr < TWO33
    seg = np.arange(lam.size, dtype=np.int64)[:, None]
    keys = (seg << 34) + thr.astype(np.int64)
    counts = valid.sum(axis=1)
    start = np.concatenate(([0], np.cumsum(counts)[:-1])).astype(np.int64)
    return keys[valid].astype(np.int64), start


@dataclass
class Workload:
    """A labelled feature distribution: C classes, F features, one model."""
    wid: int                 # workload id (seed stream)
    n_classes: int
    n_features: int
    p_zero: float
    clip255: bool            # byte features (clip at 255) vs int32 (no clip)
    group: int = 0
    prior: np.ndarray | None = None   # None: balanced y_i = i mod C
    near_tie: float = 0.0    # > 0: every class c > 0 gets lam[0, f] exp(near_tie z_cf)
    lam: np.ndarray = field(init=False)

    def __post_init__(self):
        rng = _np_rng(self.wid, ROLE_LAMBDA, self.group)
        self.lam = rng.gamma(0.5, 2.0, size=(self.n_classes, self.n_features))
        if self.near_tie > 0.0:
            # classes that differ only slightly: many files score close to a
            # tie, which populates the label band of reduced-precision paths
            z = _np_rng(self.wid, ROLE_LAMBDA, self.group, 1).standard_normal(
                (self.n_classes - 1, self.n_features))
            self.lam[1:] = self.lam[0][None, :] * np.exp(self.near_tie * z)
        self._tab = {}

    @property
    def xdtype(self):
        return torch.uint8 if self.clip255 else torch.int32

    def _table(self, device):
        key = str(device)
        if key not in self._tab:
            keys, start = poisson_search_table(self.lam, 255 if self.clip255 else None)
            self._tab[key] = (torch.from_numpy(keys).to(device),
                              torch.from_numpy(start).to(device))
        return self._tab[key]

    def labels(self, role: int, row0: int, n: int, device="cpu") -> torch.Tensor:
        """int32 class labels of rows row0 .. row0+n-1 of a stream."""
        C = self.n_classes
        if self.prior is None:
            return (torch.arange(row0, row0 + n, dtype=torch.int64, device=device) % C).to(torch.int32)
        cum = np.cumsum(np.asarray(self.prior, dtype=np.float64))[:-1]
        thr = torch.from_numpy(np.ceil(cum * TWO33).astype(np.int64)).to(device)
        wa, _ = element_words(SEED, _philox_key1(self.wid, self.group, role), row0, n, 1, device)
        return torch.searchsorted(thr, 2 * wa[:, 0] + 1, right=True).to(torch.int32)

    def features(self, role: int, row0: int, y: torch.Tensor, device="cpu",
                 chunk_elems: int = 1 << 24) -> torch.Tensor:
        """[n, F] features of rows row0 .. row0+n-1 for the given labels y."""
        n, F = int(y.numel()), self.n_features
        out = torch.empty((n, F), dtype=self.xdtype, device=device)
        keys, start = self._table(device)
        zthr = math.ceil(self.p_zero * TWO33)
        fidx = torch.arange(F, dtype=torch.int64, device=device)
        rows_per = max(1, chunk_elems // max(F, 1))
        key1 = _philox_key1(self.wid, self.group, role)
        for r in range(0, n, rows_per):
            m = min(rows_per, n - r)
            yy = y[r:r + m].to(device=device, dtype=torch.int64)
            wa, wb = element_words(SEED, key1, row0 + r, m, F, device)
            seg = yy[:, None] * F + fidx[None, :]
            x = torch.searchsorted(keys, (seg << 34) + (2 * wb + 1), right=True) - start[seg]
            x = torch.where(2 * wa + 1 < zthr, torch.zeros_like(x), x)
            out[r:r + m] = x.to(self.xdtype)
        return out

    def train_set(self, n: int, device="cpu", row0: int = 0):
        y = self.labels(ROLE_TRAIN_Y, row0, n, device)
        return self.features(ROLE_TRAIN_X, row0, y, device), y

    def test_set(self, n: int, device="cpu", row0: int = 0):
        y = self.labels(ROLE_TEST_Y, row0, n, device)
        return self.features(ROLE_TEST_X, row0, y, device), y


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the experiment shapes the method is run at.
# ---------------------------------------------------------------------------

def tiny_int32() -> Workload:
    """2 classes, 64 int32 occurrence features, 70% zeros, no clip;
    2,000 train + 2,000 test files."""
    return Workload(wid=1, n_classes=2, n_features=64, p_zero=0.7, clip255=False)


TINY_TRAIN, TINY_TEST = 2_000, 2_000


def binary_u8(n_features: int = 1000) -> Workload:
    """2 classes, byte features (Poisson clipped at 255, 80% zeros);
    200,000 train / 1,000,000 test files; F in {100, 500, 1000, 5000}."""
    return Workload(wid=2, n_classes=2, n_features=n_features, p_zero=0.8, clip255=True,
                    group=n_features)


BINARY_TRAIN, BINARY_TEST = 200_000, 1_000_000


def near_tie_u8(n_features: int = 1000, spread: float = 0.05) -> Workload:
    """The byte two-class workload with near-tied classes: lam[1, f] =
    lam[0, f] exp(spread z_f), z ~ N(0, 1) (not an experiment shape of the
    paper: a stress case for the label decision)."""
    return Workload(wid=7, n_classes=2, n_features=n_features, p_zero=0.8, clip255=True,
                    near_tie=spread)


def family16() -> Workload:
    """16 classes with Dirichlet(1) priors, F = 4096 byte features, 80% zeros;
    800,000 train / 4,000,000 test files."""
    prior = _np_rng(3, ROLE_PRIOR).dirichlet(np.ones(16))
    return Workload(wid=3, n_classes=16, n_features=4096, p_zero=0.8, clip255=True,
                    prior=prior)


FAMILY_TRAIN, FAMILY_TEST = 800_000, 4_000_000


def group_sizes(n_groups: int = 256, mu: float = 7.0, sigma: float = 1.5,
                lo: int = 100, hi: int = 100_000, step: int = 0) -> np.ndarray:
    """Test-file counts of size groups: lognormal(mu, sigma) clipped to [lo, hi];
    step > 0 draws the counts of a later step of the same workload."""
    rng = _np_rng(4, ROLE_SIZES) if step == 0 else _np_rng(4, ROLE_SIZES, step)
    return np.clip(np.rint(rng.lognormal(mu, sigma, size=n_groups)), lo, hi).astype(np.int64)


def group_workload(g: int, n_features: int = 2000) -> Workload:
    """Size group g: its own class rates, 2 classes, byte features, 80% zeros."""
    return Workload(wid=4, n_classes=2, n_features=n_features, p_zero=0.8, clip255=True, group=g)


# The experiment shape of the paper (sections 3-4): 13,665 executables
# (11,305 malware, 2,360 benign) in 100 size groups of 5 KB, split 2:1 into
# training and test files; groups 5, 8, 61, 65, 97, 98 and 100 have fewer
# than six training files of one class.  Not given, so read here: per-group
# file counts are lognormal(0, 1) shares of the total (at least 30 files),
# benign files are 2,360 / 13,665 of each group's training files (at least
# 6, and 3 in the seven groups above), and the full opcode histogram has
# 1024 features.
PAPER_N_GROUPS = 100
PAPER_FILES = 13_665
PAPER_MALWARE = 11_305
PAPER_UNTRAINED = (4, 7, 60, 64, 96, 97, 99)     # 0-based indices of groups 5, 8, 61, 65, 97, 98, 100
PAPER_F = 1024
PAPER_KS = (20, 40, 80, 100, 160, 200)


def paper_groups():
    """(benign training files, malware training files, test-file share) per group."""
    rng = _np_rng(6, ROLE_SIZES)
    w = rng.lognormal(0.0, 1.0, size=PAPER_N_GROUPS)
    sizes = np.maximum(np.rint(PAPER_FILES * w / w.sum()), 30).astype(np.int64)
    train = np.rint(sizes * 2.0 / 3.0).astype(np.int64)
    benign = np.maximum(np.rint(train * (1.0 - PAPER_MALWARE / PAPER_FILES)), 6).astype(np.int64)
    malware = np.maximum(train - benign, 6).astype(np.int64)
    benign[list(PAPER_UNTRAINED)] = 3
    return benign, malware, sizes / sizes.sum()


def split_files(n_total: int, share) -> np.ndarray:
    """n_total files over groups in proportion to share (largest remainders)."""
    share = np.asarray(share, dtype=np.float64)
    raw = n_total * share / share.sum()
    out = np.floor(raw).astype(np.int64)
    rest = int(n_total - out.sum())
    if rest > 0:
        out[np.argsort(-(raw - out), kind="stable")[:rest]] += 1
    return out


def paper_group_workload(g: int, n_features: int = PAPER_F) -> Workload:
    """Size group g of the paper-shaped experiment: its own class rates, byte
    opcode counts with 80% zeros, test labels at the dataset's class ratio."""
    prior = np.array([1.0 - PAPER_MALWARE / PAPER_FILES, PAPER_MALWARE / PAPER_FILES])
    return Workload(wid=6, n_classes=2, n_features=n_features, p_zero=0.8, clip255=True, group=g, prior=prior)


def paper_train_set(g: int, n_features: int = PAPER_F, device="cpu"):
    """Group g's training files: its benign then its malware files."""
    benign, malware, _ = paper_groups()
    y = torch.cat([torch.zeros(int(benign[g]), dtype=torch.int32),
                   torch.ones(int(malware[g]), dtype=torch.int32)]).to(device)
    return paper_group_workload(g, n_features).features(ROLE_TRAIN_X, 0, y, device), y


SERVE_F = (500, 1000, 5000, 500, 1000, 5000, 500, 1000)


def serve_model_workload(m: int) -> Workload:
    """Resident model m of the serving mix: 2 classes, F from SERVE_F."""
    return Workload(wid=5, n_classes=2, n_features=SERVE_F[m], p_zero=0.8, clip255=True, group=m)


def serve_requests(n_requests: int, qps: float, n_models: int = 8, max_files: int = 4096):
    """Scan requests: size floor(exp(U(0, ln(max_files + 1)))), model uniform,
    Poisson arrivals at rate qps.  Returns (sizes, models, arrival_s)."""
    rng = _np_rng(5, ROLE_REQUESTS)
    sizes = np.floor(np.exp(rng.uniform(0.0, math.log(max_files + 1), size=n_requests))).astype(np.int64)
    sizes = np.clip(sizes, 1, max_files)
    models = rng.integers(0, n_models, size=n_requests).astype(np.int32)
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    return sizes, models, np.cumsum(gaps)


def to_fp8_e4m3(x: torch.Tensor, sat: float = 240.0) -> torch.Tensor:
    """Encode non-negative counts as FP8-e4m3 (OCP e4m3fn) bytes: saturate at
    `sat`, round to nearest even (torch's cast).  Returns a uint8 view."""
    return x.to(torch.float32).clamp_(max=sat).to(torch.float8_e4m3fn).view(torch.uint8)
