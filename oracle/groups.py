"""Size-group model validity and fallback routing (test infrastructure).

Paper, section 3: files are partitioned into size groups of 5 KB each (100
groups up to 500 KB), and each group keeps its own top-k features.
Paper, section 4: a model is trained per group, except for groups with fewer
than six files in either class (malware or benign); the files of such a group
are classified with the next group's trained model.

Readings: the threshold counts training files per class; "next" is the first
trained group with a higher index, and where none exists (the last group is
itself untrained in the paper's data) the nearest trained group below.
"""
from __future__ import annotations

import numpy as np


def trained_mask(class_counts, min_files: int = 6) -> np.ndarray:
    """bool[G]: group g gets a model iff every class has >= min_files files."""
    cc = np.asarray(class_counts, dtype=np.int64)
    return cc.min(axis=1) >= min_files


def route(trained) -> np.ndarray:
    """int64[G]: index of the group whose model scores group g's files."""
    trained = np.asarray(trained, dtype=bool)
    G = trained.size
    if not trained.any():
        raise ValueError("no group has a trained model")
    out = np.empty(G, dtype=np.int64)
    for g in range(G):
        if trained[g]:
            out[g] = g
            continue
        nxt = [h for h in range(g + 1, G) if trained[h]]
        if nxt:
            out[g] = nxt[0]
        else:
            out[g] = [h for h in range(g - 1, -1, -1) if trained[h]][0]
    return out
