"""Host-side IVF + residual-PQ index construction (Alg. 1: KMeans, PQ
codebooks per subspace, Quantize), used to produce a trained index as input.

This is the offline construction the search path assumes (section 4.1): the
data are partitioned with k-means into L lists, residuals against each
list's arithmetic-mean centroid are product-quantised with m subspaces of
d' = d/m dimensions and K = 16 centroids (4-bit codes). For inner-product
data the lists are selected with normalised centroids while residuals use the
non-normalised mean centroids (section 4.6.1).

Choices the paper leaves open (k-means seeding, iteration counts, empty
cluster handling, sub-sampling) are fixed here; they shape the index, which
is shared data, and do not affect parity between the GPU path and the oracle.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .synth import STREAM_KMEANS, STREAM_PQ, WorkloadConfig, rng_for

KSUB = 16


def _nearest(X: np.ndarray, C: np.ndarray, ip: bool, chunk: int = 32768):
    """Index of the nearest row of C for each row of X (squared L2, or max IP)."""
    out = np.empty(len(X), dtype=np.int64)
    cn = (C.astype(np.float32) ** 2).sum(axis=1)
    Ct = np.ascontiguousarray(C.T, dtype=np.float32)
    for s in range(0, len(X), chunk):
        g = X[s:s + chunk] @ Ct
        if ip:
            out[s:s + chunk] = np.argmax(g, axis=1)
        else:
            out[s:s + chunk] = np.argmin(cn[None, :] - 2.0 * g, axis=1)
    return out


def _group_means(X: np.ndarray, a: np.ndarray, k: int):
    order = np.argsort(a, kind="stable")
    counts = np.bincount(a, minlength=k)
    sums = np.zeros((k, X.shape[1]), dtype=np.float64)
    nz = np.nonzero(counts)[0]
    starts = np.concatenate(([0], np.cumsum(counts)[:-1]))[nz]
    sums[nz] = np.add.reduceat(X[order].astype(np.float64), starts, axis=0)
    return sums, counts


def _kmeans(X: np.ndarray, k: int, iters: int, rng, ip: bool) -> np.ndarray:
    n = len(X)
    C = X[rng.choice(n, size=k, replace=n < k)].astype(np.float64)
    for _ in range(iters):
        Cs = C
        if ip:
            nrm = np.linalg.norm(C, axis=1, keepdims=True)
            nrm[nrm == 0] = 1.0
            Cs = C / nrm
        a = _nearest(X, Cs.astype(np.float32), ip)
        sums, counts = _group_means(X, a, k)
        empty = counts == 0
        C = np.where(counts[:, None] > 0, sums / np.maximum(counts, 1)[:, None], C)
        if empty.any():
            C[empty] = X[rng.choice(n, size=int(empty.sum()))]
    return C


def _spill_lists(X: np.ndarray, cm: np.ndarray, primary: np.ndarray, lam: float,
                 chunk: int = 16384) -> np.ndarray:
    """SOAR spill list of every row (float32 BLAS, chunked): the list l != p
    minimising ||x - c_l||^2 + lam * <x - c_l, r>^2 / ||r||^2, r = x - c_p."""
    out = np.empty(len(X), dtype=np.int64)
    C = np.asarray(cm, dtype=np.float32)
    Ct = np.ascontiguousarray(C.T)
    cn = (C.astype(np.float64) ** 2).sum(axis=1).astype(np.float32)
    for s in range(0, len(X), chunk):
        x = np.asarray(X[s:s + chunk], dtype=np.float32)
        p = primary[s:s + chunk]
        r = x - C[p]
        rr = (r * r).sum(axis=1)
        xc = x @ Ct
        dist = (x * x).sum(axis=1)[:, None] - 2.0 * xc + cn[None, :]
        proj = (r * x).sum(axis=1)[:, None] - r @ Ct
        loss = dist + lam * proj * proj / np.where(rr > 0, rr, 1.0)[:, None]
        loss[np.arange(len(x)), p] = np.inf
        out[s:s + chunk] = np.argmin(loss, axis=1)
    return out


def spill_index(X: np.ndarray, index: dict, lam: float, spill=None) -> dict:
    """A copy of `index` where every point also lies in its SOAR spill list
    (section 4.6.2): list_ids then holds 2 entries per point (ascending ids
    within a list), codes are per entry ([entries, m], the residual to that
    entry's list) and "copies" is 2. `spill` overrides the spill lists."""
    assert "dims" not in index, "spill the sub-index before filtration"
    off, lid = index["list_offsets"], np.asarray(index["list_ids"], dtype=np.int64)
    L = len(off) - 1
    assert L >= 2, "a spill list needs a second list"
    primary = np.full(len(X), -1, dtype=np.int64)
    primary[lid] = np.repeat(np.arange(L), np.diff(off))
    assert (primary >= 0).all(), "every row must be in a list"
    if spill is None:
        spill = _spill_lists(X, index["cm"], primary, lam)
    ent_list = np.concatenate([primary, spill])
    ent_id = np.concatenate([np.arange(len(X)), np.arange(len(X))])
    order = np.lexsort((ent_id, ent_list))
    ent_list, ent_id = ent_list[order], ent_id[order]
    codes = np.empty((len(ent_id), index["codebooks"].shape[0]), dtype=np.uint8)
    step = 262144
    for s in range(0, len(ent_id), step):
        ids, ls = ent_id[s:s + step], ent_list[s:s + step]
        codes[s:s + step] = encode(X[ids] - index["cm"][ls], index["codebooks"])
    out = dict(index)
    offsets = np.zeros(L + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(np.bincount(ent_list, minlength=L))
    out.update(codes=codes, list_offsets=offsets, list_ids=ent_id.astype(np.int32),
               copies=2, spill=spill, soar_lambda=float(lam))
    return out


def train_index(X: np.ndarray, cfg: WorkloadConfig, iters: int = 10,
                pq_iters: int = 12, train_per_list: int = 64,
                pq_train: int = 65536, dims=None):
    """Build an IVF-PQ index over X (float32 [n, d]).

    Returns a dict of numpy arrays:
      cm [L,d] f32 arithmetic-mean centroids (residual origin),
      cp [L,d] f32 probe centroids (= cm for L2, cm/|cm| for IP),
      codebooks [m,16,d'] f32, codes [n,m] u8 (0..15),
      list_offsets [L+1] i64, list_ids [n] i32 (ascending within a list).
    dims: kept dimensions of a component filtration (computed by the caller);
    the index is then built over X[:, dims] with m scaled to keep d', and
    the dict carries "dims" and "d_base" (the full row width).
    """
    if dims is not None:
        dims = np.asarray(dims, dtype=np.int64)
        d_base = X.shape[1]
        m = cfg.m * len(dims) // d_base
        sub = dataclasses.replace(cfg, d=len(dims), m=m, background=0)
        index = train_index(np.ascontiguousarray(X[:, dims]), sub, iters, pq_iters,
                            train_per_list, pq_train)
        index.update(dims=dims, d_base=d_base)
        return index
    n, d = X.shape
    L, m = cfg.L, cfg.m
    assert d % m == 0
    ip = cfg.metric == "ip"
    rng = rng_for(cfg, STREAM_KMEANS)
    nt = min(n, max(train_per_list * L, L))
    Xt = X[rng.choice(n, size=nt, replace=False)] if nt < n else X
    C = _kmeans(Xt, L, iters, rng, ip)
    if ip:
        nrm = np.linalg.norm(C, axis=1, keepdims=True)
        nrm[nrm == 0] = 1.0
        assign = _nearest(X, (C / nrm).astype(np.float32), ip)
    else:
        assign = _nearest(X, C.astype(np.float32), ip)
    sums, counts = _group_means(X, assign, L)
    cm64 = np.where(counts[:, None] > 0, sums / np.maximum(counts, 1)[:, None], C)
    cm = cm64.astype(np.float32)
    if ip:
        nrm = np.sqrt((cm.astype(np.float64) ** 2).sum(axis=1, keepdims=True))
        nrm[nrm == 0] = 1.0
        cp = (cm.astype(np.float64) / nrm).astype(np.float32)
    else:
        cp = cm.copy()

    dsub = d // m
    resid = X - cm[assign]
    prng = rng_for(cfg, STREAM_PQ)
    ptr = resid[prng.choice(n, size=min(n, pq_train), replace=False)]
    codebooks = np.empty((m, KSUB, dsub), dtype=np.float32)
    for j in range(m):
        sub = np.ascontiguousarray(ptr[:, j * dsub:(j + 1) * dsub])
        codebooks[j] = _kmeans(sub, KSUB, pq_iters, prng, False).astype(np.float32)
    codes = encode(resid, codebooks)

    order = np.argsort(assign, kind="stable")
    list_offsets = np.zeros(L + 1, dtype=np.int64)
    list_offsets[1:] = np.cumsum(np.bincount(assign, minlength=L))
    return dict(cm=cm, cp=cp, codebooks=codebooks, codes=codes,
                list_offsets=list_offsets, list_ids=order.astype(np.int32),
                metric=cfg.metric)


def encode(resid: np.ndarray, codebooks: np.ndarray, chunk: int = 16384):
    """Nearest codeword per subspace (squared L2, ties to the lowest index)."""
    n, d = resid.shape
    m, K, dsub = codebooks.shape
    codes = np.empty((n, m), dtype=np.uint8)
    for s in range(0, n, chunk):
        r = resid[s:s + chunk].reshape(-1, m, 1, dsub)
        dist = ((r - codebooks[None]) ** 2).sum(axis=3)
        codes[s:s + chunk] = np.argmin(dist, axis=2).astype(np.uint8)
    return codes
