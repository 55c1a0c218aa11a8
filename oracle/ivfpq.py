"""Plain CPU oracle of the IVF-PQ search path (test infrastructure only).

What it computes follows the search procedure (Alg. 2) with static
parameters and the brute-force branch of SearchInCluster (Alg. 3):

  1. coarse scores of the query against every list centroid and the
     nprobe nearest lists (TopNClusters);
  2. per probed list the asymmetric-distance lookup table of Eq. (1)
     (section 2.4), over residuals of the list (section 4.1);
  3. 8-bit quantisation of that table (sections 2.5 and 4.5.1);
  4. the approximate distance of every point of every probed list by table
     lookups over its 4-bit codes (CalculatePQDistances);
  5. the `reorder` best candidates over all probed lists (UpdateNNPool);
  6. exact re-ranking of the candidates against the query and the top k.

Stages 1-5 are computed in float32 ("canonical32"): every intermediate is a
float32 value produced by elementwise numpy float32 operations, each rounded
on its own, in the order written below, so that an independent
implementation can reproduce them bit for bit. No numpy reduction
(sum/dot/matmul) is used in those stages because their summation order is
unspecified. Stage 6 and the brute-force search are float64 ("exact64").

Readings where the paper is silent (all also listed in the design notes):
  * L2 uses one table per (query, list) built on the residual q - c_l; inner
    product uses one table per query plus a per-list bias -<q, c_l>, with c_l
    the arithmetic-mean centroid, while lists are *selected* with the
    normalised centroid (section 4.6.1).
  * Inner product is handled as the distance -<q, x>; re-ranked results are
    returned as <q, x>, largest first.
  * Quantisation: per-subspace offset lo_j = min_i T[j,i], one scale per
    (query, list) from the largest per-subspace range, round half to even,
    clamp at 255. The constant part B = (tree sum of lo_j) + bias.
  * Ties are broken by the smaller list index / point id everywhere.
  * Adaptive nprobe / reorder (section 4.2, Eq. 2): the trained classifier
    is replaced by a closed form of its "centroid distances" feature,
    p = e_1 / e_K (see hardness); Eq. 2 is read as
    min(v_max, v_min + floor(D * ReLU(p - p0) * (p + p1))).
  * Spilled assignment (section 4.6.2 integrates SOAR): each point also
    goes to one spill list chosen by SOAR's loss with weight lam; in the
    search a point scanned in several probed lists enters the pool once, at
    the smallest of its approximate distances.
"""

from __future__ import annotations

from typing import Optional

import numpy as np

F32 = np.float32
ZERO = F32(0.0)


# --------------------------------------------------------------------------
# Summation orders used by the canonical float32 stages.
# --------------------------------------------------------------------------

def seq_sum(terms: np.ndarray) -> np.ndarray:
    """Sequential float32 sum over the last axis: acc = 0; acc = acc + t_u."""
    terms = np.asarray(terms, dtype=F32)
    acc = np.zeros(terms.shape[:-1], dtype=F32)
    for u in range(terms.shape[-1]):
        acc = acc + terms[..., u]
    return acc


def tree_sum(terms: np.ndarray) -> np.ndarray:
    """Pairwise float32 sum over the last axis.

    The length is padded with +0.0 to a power of two, then adjacent pairs are
    added level by level: (t0+t1), (t2+t3), ... until one value remains.
    """
    v = np.asarray(terms, dtype=F32)
    n = v.shape[-1]
    p = 1
    while p < n:
        p *= 2
    if p != n:
        pad = np.zeros(v.shape[:-1] + (p - n,), dtype=F32)
        v = np.concatenate([v, pad], axis=-1)
    while v.shape[-1] > 1:
        v = v[..., 0::2] + v[..., 1::2]
    return v[..., 0]


def _plus_zero(x):
    """Map -0.0 to +0.0 (x + 0.0 is exact otherwise)."""
    return x + ZERO


# --------------------------------------------------------------------------
# Stage 1: coarse scoring and top-nprobe (Alg. 2, TopNClusters).
# --------------------------------------------------------------------------

def coarse_scores(q: np.ndarray, cp: np.ndarray, metric: str) -> np.ndarray:
    """Score of the query against every probe centroid, smaller is nearer.

    L2: s_l = sum_t (q_t - c_{l,t})^2, squared Euclidean (sections 2.4, 4.5.3).
    IP: s_l = -sum_t q_t * c_{l,t} with normalised centroids (section 4.6.1).
    Sums are sequential over t in float32.
    """
    q = np.asarray(q, dtype=F32)
    cp = np.asarray(cp, dtype=F32)
    if metric == "l2":
        diff = q[None, :] - cp
        return seq_sum(diff * diff)
    return _plus_zero(-seq_sum(q[None, :] * cp))


def select_probes(scores: np.ndarray, nprobe: int) -> np.ndarray:
    """The nprobe lists with the smallest (score, list index), in that order."""
    L = len(scores)
    order = np.lexsort((np.arange(L), scores))
    return order[:nprobe].astype(np.int64)


# --------------------------------------------------------------------------
# Stage 2: the lookup table of Eq. (1) for one (query, list).
# --------------------------------------------------------------------------

def lut_float(q: np.ndarray, cm_l: np.ndarray, codebooks: np.ndarray,
              metric: str) -> np.ndarray:
    """Float32 table T[j, i] = d(q^j, c_i^j) over residual PQ (Eq. 1, section 4.1).

    L2: r = q - cm_l; T[j,i] = sum_u (r_{j d'+u} - B[j,i,u])^2, sequential in u.
    IP: T[j,i] = -sum_u q_{j d'+u} * B[j,i,u] (independent of the list).
    """
    q = np.asarray(q, dtype=F32)
    m, K, dsub = codebooks.shape
    if metric == "l2":
        r = q - np.asarray(cm_l, dtype=F32)
        diff = r.reshape(m, 1, dsub) - codebooks
        return seq_sum(diff * diff)
    prod = q.reshape(m, 1, dsub) * codebooks
    return _plus_zero(-seq_sum(prod))


def list_bias(q: np.ndarray, cm_l: np.ndarray, metric: str) -> F32:
    """Per-list constant of the ADC value: 0 for L2, -<q, cm_l> for IP.

    For inner product the residual decomposition x = cm_l + r gives
    -<q, x> = -<q, cm_l> - <q, r>; the first term is this bias.
    """
    if metric == "l2":
        return ZERO
    prod = np.asarray(q, dtype=F32) * np.asarray(cm_l, dtype=F32)
    return _plus_zero(-seq_sum(prod[None, :])[0])


# --------------------------------------------------------------------------
# Stage 3: 8-bit quantisation of the table (sections 2.5, 4.5.1).
# --------------------------------------------------------------------------

def quantize_lut(T: np.ndarray, bias):
    """Quantise a float32 table to u8 entries with one affine map per table.

    lo_j  = min_i T[j,i]
    rng   = max_j max_i (T[j,i] - lo_j)
    delta = rng / 255, s = 255 / rng (both correctly rounded float32)
    q8    = min(255, rint((T[j,i] - lo_j) * s))   (round half to even)
    B     = tree_sum_j(lo_j) + bias
    If rng == 0 the table is constant: delta = 0 and q8 = 0.
    The approximate value of code vector c is then B + delta * sum_j q8[j, c_j].
    Returns (q8 [m,16] uint8, lo [m] f32, delta f32, B f32).
    """
    T = np.asarray(T, dtype=F32)
    lo = T.min(axis=1)
    D = T - lo[:, None]
    rng = D.max()
    if rng > ZERO:
        s = F32(255.0) / rng
        delta = rng / F32(255.0)
        q8 = np.minimum(F32(255.0), np.rint(D * s)).astype(np.uint8)
    else:
        delta = ZERO
        q8 = np.zeros(T.shape, dtype=np.uint8)
    B = tree_sum(lo[None, :])[0] + F32(bias)
    return q8, lo, F32(delta), F32(B)


# --------------------------------------------------------------------------
# Stage 4: ADC scan of one list (Alg. 3, CalculatePQDistances).
# --------------------------------------------------------------------------

def scan_list(q8: np.ndarray, delta, B, codes_rows: np.ndarray):
    """Approximate values of the points whose codes are ``codes_rows`` [n_l, m].

    S(x) = sum_j q8[j, code_j(x)] is an exact integer (at most 255 m < 2^16);
    a(x) = B + delta * float(S), product and sum each rounded in float32.
    Returns (S int64 [n_l], a float32 [n_l]).
    """
    m = q8.shape[0]
    codes_rows = np.asarray(codes_rows)
    S = np.zeros(len(codes_rows), dtype=np.int64)
    for j in range(m):
        S += q8[j, codes_rows[:, j]].astype(np.int64)
    a = _plus_zero(F32(B) + F32(delta) * S.astype(F32))
    return S, a


# --------------------------------------------------------------------------
# Stage 5: candidate pool of size `reorder` (Alg. 3, UpdateNNPool).
# --------------------------------------------------------------------------

def top_r(a: np.ndarray, ids: np.ndarray, R: int):
    """The min(R, len) smallest (a, id) pairs in lexicographic order."""
    order = np.lexsort((ids, a))[:R]
    return a[order], ids[order]


def top_r_unique(a: np.ndarray, ids: np.ndarray, R: int):
    """Pool over a spilled index, where one point may be scanned in several
    probed lists (section 4.6.2): a point's approximate distance is the
    smallest of its copies, and the pool is the min(R, #points) smallest
    (distance, id) pairs over distinct points."""
    best = {}
    for v, i in zip(a.tolist(), ids.tolist()):
        if i not in best or v < best[i]:
            best[i] = v
    pairs = sorted((v, i) for i, v in best.items())[:R]
    return (np.array([v for v, _ in pairs], dtype=F32),
            np.array([i for _, i in pairs], dtype=np.int64))


# --------------------------------------------------------------------------
# Stage 6: exact re-rank (Alg. 2, final step) -- float64.
# --------------------------------------------------------------------------

def rerank(q: np.ndarray, X: np.ndarray, cand_ids: np.ndarray, k: int,
           metric: str):
    """Exact distances of the candidates and the top k.

    L2: e = sum_t (q_t - x_t)^2, ascending; IP: e = <q, x>, descending; ties
    by the smaller id. Missing results are (-1, +inf) for L2 / (-1, -inf) IP.
    """
    q64 = np.asarray(q, dtype=np.float64)
    ids = np.asarray(cand_ids, dtype=np.int64)
    ids = ids[ids >= 0]
    # Gather the candidate rows first, then widen them (not the whole base).
    rows = np.asarray(X[ids], dtype=np.float64) if len(ids) else np.zeros((0, len(q)))
    if metric == "l2":
        e = ((rows - q64[None, :]) ** 2).sum(axis=1)
        order = np.lexsort((ids, e))
        pad = np.inf
    else:
        e = rows @ q64
        order = np.lexsort((ids, -e))
        pad = -np.inf
    order = order[:k]
    out_ids = np.full(k, -1, dtype=np.int64)
    out_d = np.full(k, pad, dtype=np.float64)
    out_ids[:len(order)] = ids[order]
    out_d[:len(order)] = e[order]
    return out_ids, out_d


# --------------------------------------------------------------------------
# Component filtration (section 4.3; Alg. 1 FilterComponents, Alg. 2).
# --------------------------------------------------------------------------

def component_filter(X: np.ndarray, threshold: float):
    """Dimensions kept by the statistical filtration of section 4.3.

    For every dimension t over all rows: mean mu_t and standard deviation
    sigma_t (population, FP64), and the share of components that are zero or
    lie within one standard deviation of the mean, |x_t - mu_t| <= sigma_t.
    A dimension whose share exceeds `threshold` is dropped. Returns the kept
    dimension indices (ascending) and the shares."""
    X64 = np.asarray(X, dtype=np.float64)
    n, d = X64.shape
    share = np.empty(d, dtype=np.float64)
    for t in range(d):
        col = X64[:, t]
        mu = col.sum() / n
        sigma = np.sqrt(((col - mu) ** 2).sum() / n)
        quiet = (col == 0.0) | (np.abs(col - mu) <= sigma)
        share[t] = quiet.sum() / n
    keep = np.nonzero(share <= threshold)[0].astype(np.int64)
    return keep, share


# --------------------------------------------------------------------------
# Adaptive probing depth and re-rank size (section 4.2, Eq. 2).
# --------------------------------------------------------------------------

def hardness(sorted_scores: np.ndarray, K: int, metric: str):
    """Closed-form stand-in for the trained easy/hard classifier of section
    4.2.1, from its "centroid distances" feature (Table 3): the ratio of the
    nearest to the K-th nearest centroid distance, p = e_1 / e_K in [0, 1]
    (near 1: many lists about as near as the nearest one, a hard query).
    e_i = s_i for L2 (squared distances); for inner product e_i = 1 + s_i,
    which is half the squared distance to a normalised centroid for a unit
    query. FP32, in this order: e = (1 + s); p = e_1 / e_K if e_K > 0 else 1;
    clamped to [0, 1]."""
    s1 = F32(sorted_scores[0])
    sK = F32(sorted_scores[K - 1])
    if metric == "ip":
        e1, eK = F32(1.0) + s1, F32(1.0) + sK
    else:
        e1, eK = s1, sK
    with np.errstate(divide="ignore", invalid="ignore"):
        p = e1 / eK if eK > F32(0.0) else F32(1.0)
    p = F32(p)
    if not (p >= F32(0.0)):  # NaN or negative
        p = F32(0.0) if p < F32(0.0) else F32(1.0)
    return F32(min(p, F32(1.0)))


def eq2(p, vmin: int, vmax: int, p0, p1) -> int:
    """Eq. 2: min(v_max, v_min + floor(D * ReLU(p - p0) * (p + p1))), with
    D = v_max - v_min, the products taken in this order in FP32; v_min is
    first clamped to [1, v_max]."""
    vmin = max(1, min(int(vmin), int(vmax)))
    relu = F32(max(F32(p) - F32(p0), F32(0.0)))
    g = F32(relu * (F32(p) + F32(p1)))
    x = F32(F32(vmax - vmin) * g)
    return int(min(vmax, vmin + int(np.floor(x))))


def adaptive_params(scores: np.ndarray, nprobe_max: int, metric: str, nprobe_init: int,
                    nprobe_min: int, reorder_min: int, R: int, k: int, p0, p1):
    """Per-query (nprobe, reorder) of Alg. 2 (nprob from the initial clusters,
    reorder from the same hardness): the coarse scores sorted by (score,
    list), K = min(nprobe_init, nprobe_max) of them feed p, then Eq. 2 with
    nprob_max = nprobe_max and reorder_max = R (reorder_min clamped to
    [k, R])."""
    P = select_probes(scores, nprobe_max)
    K = max(1, min(int(nprobe_init), int(nprobe_max)))
    p = hardness(scores[P], K, metric)
    npb = eq2(p, nprobe_min, nprobe_max, p0, p1)
    rmin = max(int(k), min(int(reorder_min), int(R)))
    reo = eq2(p, rmin, R, p0, p1) if R > 0 else 0
    return npb, reo, p


# --------------------------------------------------------------------------
# The whole search and the exhaustive reference.
# --------------------------------------------------------------------------

def search(index: dict, X: np.ndarray, Q: np.ndarray, nprobe, k: int, R: int,
           want_stages: bool = False, adaptive: Optional[dict] = None):
    """Run stages 1-6 for every query.

    index: dict with cm, cp [L,d] f32, codebooks [m,16,d'] f32, codes [n,m]
    u8, list_offsets [L+1], list_ids [n], metric. nprobe: int or per-query
    array. Returns dict with ids [nq,k] int64, dist [nq,k] f64, cand_a
    [nq,R] f32 (+inf padded), cand_id [nq,R] int64 (-1 padded) and, when
    want_stages, probes (list of arrays) and luts {(qi, list): (q8, lo, delta, B)}.
    index["copies"] (optional, default 1): a spilled index (section 4.6.2),
    where a point lies in up to `copies` lists; codes are then per list entry
    ([list_offsets[L], m], aligned with list_ids) and the pool keeps each
    point once, at its best copy (top_r_unique).
    index["dims"] (optional): kept dimensions of component filtration; the
    index lives in that subspace, stages 1-5 use q[dims] and the re-rank the
    full query against the full rows X (Alg. 2).
    adaptive: dict(nprobe_init, nprobe_min, reorder_min, p0, p1) -- per query,
    nprobe[qi] is nprob_max and R is reorder_max of Eq. 2; the pool keeps the
    R best as always and the re-rank takes its reorder best (the same set a
    pool of size reorder would hold). Adds nprobe_used, reorder_used.
    """
    metric = index["metric"]
    cm, cp = index["cm"], index["cp"]
    codebooks = np.asarray(index["codebooks"], dtype=F32)
    codes = index["codes"]
    off, lid = index["list_offsets"], index["list_ids"]
    nq = len(Q)
    nprobe = np.broadcast_to(np.asarray(nprobe), (nq,))
    out_ids = np.full((nq, k), -1, dtype=np.int64)
    out_d = np.zeros((nq, k), dtype=np.float64)
    cand_a = np.full((nq, R), np.inf, dtype=F32)
    cand_id = np.full((nq, R), -1, dtype=np.int64)
    probes, luts = [], {}
    np_used = np.zeros(nq, dtype=np.int64)
    reo_used = np.full(nq, R, dtype=np.int64)
    dims = index.get("dims")
    spilled = int(index.get("copies", 1)) > 1
    for qi in range(nq):
        q_init = np.asarray(Q[qi], dtype=F32)
        q = q_init[np.asarray(dims)] if dims is not None else q_init
        s = coarse_scores(q, cp, metric)
        npq = int(nprobe[qi])
        if adaptive is not None:
            npq, reo_used[qi], _ = adaptive_params(
                s, npq, metric, adaptive["nprobe_init"], adaptive["nprobe_min"],
                adaptive["reorder_min"], R, k, adaptive["p0"], adaptive["p1"])
        np_used[qi] = npq
        P = select_probes(s, npq)
        if want_stages:
            probes.append(P)
        T_ip = lut_float(q, None, codebooks, metric) if metric == "ip" else None
        all_a, all_id = [], []
        for l in P:
            T = T_ip if T_ip is not None else lut_float(q, cm[l], codebooks, metric)
            q8, lo, delta, B = quantize_lut(T, list_bias(q, cm[l], metric))
            if want_stages:
                luts[(qi, int(l))] = (q8, lo, delta, B)
            ids = np.asarray(lid[off[l]:off[l + 1]], dtype=np.int64)
            rows = codes[off[l]:off[l + 1]] if spilled else codes[ids]
            _, a = scan_list(q8, delta, B, rows)
            all_a.append(a)
            all_id.append(ids)
        a = np.concatenate(all_a) if all_a else np.zeros(0, F32)
        ids = np.concatenate(all_id) if all_id else np.zeros(0, np.int64)
        ca, cid = top_r_unique(a, ids, R) if spilled else top_r(a, ids, R)
        cand_a[qi, :len(ca)] = ca
        cand_id[qi, :len(cid)] = cid
        out_ids[qi], out_d[qi] = rerank(q_init, X, cid[:reo_used[qi]], k, metric)
    res = dict(ids=out_ids, dist=out_d, cand_a=cand_a, cand_id=cand_id)
    if adaptive is not None:
        res["nprobe_used"] = np_used
        res["reorder_used"] = reo_used
    if want_stages:
        res["probes"] = probes
        res["luts"] = luts
    return res


# --------------------------------------------------------------------------
# Index construction steps (Alg. 1: list assignment and Quantize).
# --------------------------------------------------------------------------

def assign_lists(X: np.ndarray, cp: np.ndarray, metric: str) -> np.ndarray:
    """Nearest list of every row: the top-1 of step 1 (canonical FP32 score,
    ties to the smaller list index)."""
    return np.array([select_probes(coarse_scores(x, cp, metric), 1)[0] for x in X],
                    dtype=np.int64)


def encode(X: np.ndarray, cm: np.ndarray, lists: np.ndarray, codebooks: np.ndarray) -> np.ndarray:
    """PQ codes of the residuals x - cm[list(x)] (Alg. 1 Quantize, section 2.3).

    code_j(x) = argmin_i sum_u (r_{j d'+u} - B[j,i,u])^2 with the residual
    component rounded once and the sum sequential in u (FP32); ties go to the
    smallest i.
    """
    X = np.asarray(X, dtype=F32)
    cb = np.asarray(codebooks, dtype=F32)
    m, K, dsub = cb.shape
    r = X - np.asarray(cm, dtype=F32)[np.asarray(lists)]
    diff = r.reshape(len(X), m, 1, dsub) - cb[None]
    dist = seq_sum(diff * diff)                      # [n, m, K]
    return np.argmin(dist, axis=2).astype(np.uint8)  # first minimum


def spill_assign(X: np.ndarray, cm: np.ndarray, primary: np.ndarray, lam: float) -> np.ndarray:
    """Spilled (secondary) list of every row, SOAR (section 4.6.2 integrates
    it for points near list boundaries; the loss is the one SOAR defines).

    With r = x - c_p the residual to the row's primary list p (mean
    centroids, the residual origin) and r' = x - c_l for a candidate list
    l != p, the spill list minimises
        loss(l) = ||r'||^2 + lam * <r', r>^2 / ||r||^2,
    the squared residual plus lam times the squared length of its projection
    on r, so that the second residual is pushed towards being orthogonal to
    the first (a query badly served by one list is then better served by
    the other). A row equal to its centroid (r = 0) takes the nearest other
    list. Ties go to the smaller list index. float64."""
    X64 = np.asarray(X, dtype=np.float64)
    C64 = np.asarray(cm, dtype=np.float64)
    out = np.empty(len(X64), dtype=np.int64)
    for i, x in enumerate(X64):
        p = int(primary[i])
        r = x - C64[p]
        rr = float(r @ r)
        dev = x[None, :] - C64
        loss = (dev * dev).sum(axis=1)
        if rr > 0.0:
            proj = dev @ r
            loss = loss + lam * proj * proj / rr
        loss[p] = np.inf
        out[i] = int(np.argmin(loss))  # first minimum
    return out


def brute_force_knn(X: np.ndarray, Q: np.ndarray, k: int, metric: str):
    """Exact k-NN (section 1 problem statement) by exhaustive float64 search.

    Ordered by (squared L2 ascending | inner product descending, id ascending).
    """
    X64 = np.asarray(X, dtype=np.float64)
    ids = np.arange(len(X64), dtype=np.int64)
    out_ids = np.zeros((len(Q), k), dtype=np.int64)
    out_d = np.zeros((len(Q), k), dtype=np.float64)
    for qi, q in enumerate(np.asarray(Q, dtype=np.float64)):
        if metric == "l2":
            e = ((X64 - q[None, :]) ** 2).sum(axis=1)
            order = np.lexsort((ids, e))[:k]
        else:
            e = X64 @ q
            order = np.lexsort((ids, -e))[:k]
        out_ids[qi], out_d[qi] = ids[order], e[order]
    return out_ids, out_d
