"""IVF + residual-PQ index construction on the GPU (Alg. 1).

KMeans over the lists, PQ codebooks per subspace, Quantize. The heavy steps
run in the library's kernels: nearest-list assignment (`ivf_assign`, the
coarse-scoring kernels with top-1 selection), the codeword assignment of the
PQ k-means and the residual encoding (`ivf_encode`). The k-means mean
updates are small reductions done on the host in float64 so the trained
index is reproducible. Lists are selected with
normalised centroids for inner product and residuals use the mean centroids
(section 4.6.1).
"""

from __future__ import annotations

import numpy as np

from . import assign_lists, assign_spill, encode_codes

KSUB = 16


def _group_means(X, a, k, chunk=1 << 20):
    """Per-group float64 sums and counts, in chunks of the group-sorted order."""
    order = np.argsort(a, kind="stable")
    counts = np.bincount(a, minlength=k)
    sums = np.zeros((k, X.shape[1]), dtype=np.float64)
    for s in range(0, len(order), chunk):
        idx = order[s:s + chunk]
        lab = a[idx]
        starts = np.concatenate(([0], np.nonzero(np.diff(lab))[0] + 1))
        sums[lab[starts]] += np.add.reduceat(X[idx].astype(np.float64), starts, axis=0)
    return sums, counts


def _normalise(C):
    nrm = np.linalg.norm(C, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    return C / nrm


def _pq_kmeans_gpu(resid, m, iters, rng, device):
    """16-codeword k-means of every PQ subspace at once: the assignment step is
    the encoding kernel (ivf_encode with one all-zero centroid, so the
    residual it quantises is the row itself), the means are float64 sums on
    the host; an empty codeword is reseeded from a random row."""
    import torch
    nt, d = resid.shape
    dsub = d // m
    sub = resid.reshape(nt, m, dsub)
    cb = np.empty((m, KSUB, dsub), dtype=np.float64)
    for j in range(m):
        cb[j] = sub[rng.choice(nt, size=KSUB, replace=nt < KSUB), j]
    Rd = torch.from_numpy(np.ascontiguousarray(resid, dtype=np.float32)).to(device)
    zero = torch.zeros((1, d), dtype=torch.float32, device=device)
    lists = torch.zeros(nt, dtype=torch.int32, device=device)
    for _ in range(iters):
        cbd = torch.from_numpy(cb.astype(np.float32)).to(device)
        codes = encode_codes(Rd, zero, lists, cbd).cpu().numpy().astype(np.int64)
        for j in range(m):
            a = codes[:, j]
            counts = np.bincount(a, minlength=KSUB)
            sums = np.stack([np.bincount(a, weights=sub[:, j, u].astype(np.float64),
                                         minlength=KSUB) for u in range(dsub)], axis=1)
            live = counts > 0
            cb[j][live] = sums[live] / counts[live][:, None]
            if (~live).any():
                cb[j][~live] = sub[rng.choice(nt, size=int((~live).sum())), j]
    return cb.astype(np.float32)


def component_filter(X: np.ndarray, threshold: float, chunk: int = 1 << 18) -> np.ndarray:
    """Statistical component filtration (section 4.3, Alg. 1 FilterComponents):
    per dimension the mean and (population) standard deviation over all rows,
    then the share of components equal to 0 or within one standard deviation
    of the mean; dimensions whose share exceeds `threshold` are dropped.
    Host FP64 in row chunks (a build step, like the k-means means). Returns
    the kept dimensions, ascending."""
    n, d = X.shape
    s1 = np.zeros(d, dtype=np.float64)
    for r in range(0, n, chunk):
        s1 += X[r:r + chunk].astype(np.float64).sum(axis=0)
    mu = s1 / n
    s2 = np.zeros(d, dtype=np.float64)
    for r in range(0, n, chunk):
        s2 += ((X[r:r + chunk].astype(np.float64) - mu) ** 2).sum(axis=0)
    sd = np.sqrt(s2 / n)
    quiet = np.zeros(d, dtype=np.int64)
    for r in range(0, n, chunk):
        x = X[r:r + chunk].astype(np.float64)
        quiet += ((x == 0.0) | (np.abs(x - mu) <= sd)).sum(axis=0)
    return np.nonzero(quiet / n <= threshold)[0].astype(np.int64)


def train_index_gpu(X: np.ndarray, L: int, m: int, metric: str, seed: int = 0,
                    iters: int = 10, pq_iters: int = 12, train_per_list: int = 64,
                    pq_train: int = 65536, coarse: str = "bf16", widen: int = 4,
                    device: str = "cuda", log=None, dims=None, soar=None):
    """Train an IVF-PQ index over X (float32 [n, d], host). Returns the same
    dict layout as the host trainer; `codes` and `list_ids` stay on the GPU
    (torch tensors), everything else is numpy. dims: kept columns of a
    component filtration; the index is built over X[:, dims] with m scaled
    to keep d', and carries "dims" and "d_base". soar: weight lam of a SOAR
    spilled assignment (section 4.6.2): every row also goes to its spill list
    (ivf_assign_spill), codes are per list entry and "copies" is 2."""
    import torch
    if dims is not None:
        dims = np.asarray(dims, dtype=np.int64)
        mf = m * len(dims) // X.shape[1]
        index = train_index_gpu(np.ascontiguousarray(X[:, dims]), L, mf, metric, seed, iters,
                                pq_iters, train_per_list, pq_train, coarse, widen, device, log,
                                soar=soar)
        index.update(dims=dims, d_base=X.shape[1])
        return index

    n, d = X.shape
    assert d % m == 0
    ip = metric == "ip"
    rng = np.random.default_rng(seed)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device)

    nt = min(n, max(train_per_list * L, L))
    tidx = np.sort(rng.choice(n, size=nt, replace=False)) if nt < n else np.arange(n)
    Xt = X[tidx]
    Xtd = Xd[torch.from_numpy(tidx).to(device)]
    C = Xt[rng.choice(nt, size=L, replace=nt < L)].astype(np.float64)
    for it in range(iters):
        if log:
            log(f"k-means iteration {it + 1} of {iters}")
        Cs = _normalise(C) if ip else C
        Cd = torch.from_numpy(Cs.astype(np.float32)).to(device)
        a = assign_lists(Cd, Xtd, metric, coarse=coarse, widen=widen).cpu().numpy().astype(np.int64)
        sums, counts = _group_means(Xt, a, L)
        C = np.where(counts[:, None] > 0, sums / np.maximum(counts, 1)[:, None], C)
        empty = counts == 0
        if empty.any():
            C[empty] = Xt[rng.choice(nt, size=int(empty.sum()))]
    Cs = _normalise(C) if ip else C
    Cd = torch.from_numpy(Cs.astype(np.float32)).to(device)
    assign_d = assign_lists(Cd, Xd, metric, coarse=coarse, widen=widen)
    assign = assign_d.cpu().numpy().astype(np.int64)
    if log:
        log("list means over all rows")
    sums, counts = _group_means(X, assign, L)
    cm64 = np.where(counts[:, None] > 0, sums / np.maximum(counts, 1)[:, None], C)
    cm = cm64.astype(np.float32)
    cp = _normalise(cm.astype(np.float64)).astype(np.float32) if ip else cm.copy()

    pidx = rng.choice(n, size=min(n, pq_train), replace=False)
    resid = X[pidx] - cm[assign[pidx]]
    if log:
        log(f"PQ codebooks: {m} subspaces")
    codebooks = _pq_kmeans_gpu(resid, m, pq_iters, rng, device)
    cmd = torch.from_numpy(cm).to(device)
    cbd = torch.from_numpy(codebooks).to(device)
    codes = encode_codes(Xd, cmd, assign_d, cbd)

    if soar is not None:
        if log:
            log(f"SOAR spill lists (lambda {soar})")
        spill_d = assign_spill(cmd, Xd, assign_d, soar)
        codes_s = encode_codes(Xd, cmd, spill_d, cbd)
        spill = spill_d.cpu().numpy().astype(np.int64)
        ent_list = np.concatenate([assign, spill])
        ent_id = np.concatenate([np.arange(n), np.arange(n)])
        order = np.lexsort((ent_id, ent_list))
        offsets = np.zeros(L + 1, dtype=np.int64)
        offsets[1:] = np.cumsum(np.bincount(ent_list, minlength=L))
        order_d = torch.from_numpy(order).to(device)
        return dict(cm=cm, cp=cp, codebooks=codebooks,
                    codes=torch.cat([codes, codes_s])[order_d].contiguous(),
                    list_offsets=offsets,
                    list_ids=torch.from_numpy(ent_id[order].astype(np.int32)).to(device),
                    metric=metric, assign=assign, spill=spill, copies=2,
                    soar_lambda=float(soar))

    order = np.argsort(assign, kind="stable")
    offsets = np.zeros(L + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    return dict(cm=cm, cp=cp, codebooks=codebooks, codes=codes,
                list_offsets=offsets,
                list_ids=torch.from_numpy(order.astype(np.int32)).to(device),
                metric=metric, assign=assign)
