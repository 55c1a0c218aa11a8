"""Exact k-NN ground truth (FP64) and Recall@k, for reporting search quality.

Recall@k is the fraction of the true k nearest neighbours (exhaustive search)
found among the k returned ids, averaged over queries (section 5.4). The true
neighbours are ordered by (distance, id); for inner product "distance" means
descending inner product.
"""

from __future__ import annotations

import numpy as np


def exact_knn(X: np.ndarray, Q: np.ndarray, k: int, metric: str,
              chunk: int = 65536, log=None):
    """Return (ids [nq,k] int64, dist [nq,k] float64) by FP64 exhaustive search.

    For L2 the distance is the squared Euclidean distance; for IP it is the
    inner product (larger is better). Ties are broken by the smaller id.
    """
    nq = len(Q)
    Q64 = Q.astype(np.float64)
    qn = (Q64 ** 2).sum(axis=1)
    best_d = np.full((nq, 0), 0.0)
    best_i = np.zeros((nq, 0), dtype=np.int64)
    for s in range(0, len(X), chunk):
        if log and s and s % (chunk * 32) == 0:
            log(f"ground truth: {s} of {len(X)} rows")
        Xc = X[s:s + chunk].astype(np.float64)
        g = Q64 @ Xc.T
        if metric == "l2":
            key = qn[:, None] + (Xc ** 2).sum(axis=1)[None, :] - 2.0 * g
        else:
            key = -g
        ids = np.arange(s, s + len(Xc), dtype=np.int64)[None, :].repeat(nq, 0)
        kk = min(k, key.shape[1])
        part = np.argpartition(key, kk - 1, axis=1)[:, :kk] if kk < key.shape[1] \
            else np.argsort(key, axis=1)
        cand_d = np.concatenate([best_d, np.take_along_axis(key, part, 1)], 1)
        cand_i = np.concatenate([best_i, np.take_along_axis(ids, part, 1)], 1)
        # Candidates at the cut may tie with excluded ones; re-check exactly below.
        order = np.lexsort((cand_i, cand_d), axis=1)[:, :k]
        best_d = np.take_along_axis(cand_d, order, 1)
        best_i = np.take_along_axis(cand_i, order, 1)
    # Recompute distances directly (no expansion) so ties are resolved on exact values.
    diff_d = np.empty_like(best_d)
    for qi in range(nq):
        rows = X[best_i[qi]].astype(np.float64)
        if metric == "l2":
            diff_d[qi] = ((rows - Q64[qi]) ** 2).sum(axis=1)
        else:
            diff_d[qi] = rows @ Q64[qi]
    key = diff_d if metric == "l2" else -diff_d
    order = np.lexsort((best_i, key), axis=1)
    return np.take_along_axis(best_i, order, 1), np.take_along_axis(diff_d, order, 1)


def recall_at_k(found: np.ndarray, truth: np.ndarray, k: int) -> float:
    """Mean over queries of |found[:k] ∩ truth[:k]| / k."""
    hits = 0
    for f, t in zip(found, truth):
        hits += len(set(f[:k].tolist()) & set(t[:k].tolist()))
    return hits / (k * len(found))
