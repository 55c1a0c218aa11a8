"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: brute-force
k-NN (section 1 problem statement), the reconstructed-vector identity of
Eq. (1) with residual PQ (sections 2.4, 4.1), constructed lossless cases in
which the 8-bit table is exact, error bounds, plain-Python sorts, and a
hand-worked example.
"""

import dataclasses
import json
import math
import os

import numpy as np
import pytest

import oracle
from conftest import cached_workload, make_rng

EPS32 = 2.0 ** -24
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- summation

def test_seq_and_tree_sum_orders():
    # 1e8 has float32 spacing 8, so the result depends on the order.
    v = np.array([1e8, 1.0, -1e8, 1.0], dtype=np.float32)
    # ((1e8 + 1) - 1e8) + 1: 1e8 + 1 rounds to 1e8 -> 0 + 1 = 1.
    assert oracle.seq_sum(v[None, :])[0] == np.float32(1.0)
    # (1e8 + 1) + (-1e8 + 1) = 1e8 + (-1e8) = 0.
    assert oracle.tree_sum(v[None, :])[0] == np.float32(0.0)
    # Exactly representable integers: both equal the exact sum.
    r = make_rng(1).integers(-1000, 1000, size=(7, 37)).astype(np.float32)
    exact = np.array([math.fsum(row) for row in r.astype(np.float64)])
    assert np.array_equal(oracle.seq_sum(r).astype(np.float64), exact)
    assert np.array_equal(oracle.tree_sum(r).astype(np.float64), exact)


# ---------------------------------------------------------- golden example

def test_hand_worked_lut_example():
    g = json.load(open(os.path.join(GOLDEN, "lut_worked_example.json")))
    # The expected table follows closed forms derived by hand (see the
    # fixture's derivation): rint(i^2/2) with ties to even, and i^2 + 2i.
    half_even = [(i * i) // 2 + (1 if (i * i) % 2 and ((i * i) // 2) % 2 else 0)
                 for i in range(16)]
    assert g["expected_q8"][0] == half_even
    assert g["expected_q8"][1] == [i * i + 2 * i for i in range(16)]
    q = np.array(g["q"], dtype=np.float32)
    cm = np.array(g["cm"], dtype=np.float32)
    cb = np.array(g["codebooks"], dtype=np.float32)
    T = oracle.lut_float(q, cm, cb, g["metric"])
    q8, lo, delta, B = oracle.quantize_lut(T, oracle.list_bias(q, cm, g["metric"]))
    assert q8.tolist() == g["expected_q8"]
    assert lo.tolist() == g["expected_lo"]
    assert float(delta) == g["expected_delta"]
    assert float(B) == g["expected_B"]
    S, a = oracle.scan_list(q8, delta, B, np.array(g["points_codes"]))
    assert S.tolist() == g["expected_S"]
    assert a.tolist() == g["expected_a"]
    # Quantisation error stays within m * delta / 2 of the exact value.
    exact = np.array(g["exact_reconstruction_dist"])
    assert np.all(np.abs(a - exact) <= 2 * float(delta) / 2)


def test_hand_worked_pairwise_lo_sum():
    # m = 4 subspace minima (1, 2^-24, 2^-24, 2^-24): the pairwise sum that
    # forms B is 1 + 2^-23, a sequential one would be 1 (fixture derivation).
    g = json.load(open(os.path.join(GOLDEN, "lut_pairwise_lo_sum.json")))
    i = np.arange(16)
    assert g["expected_q8"] == [(i * i + 2 * i).tolist(), (i * i).tolist(),
                                ((i * i + 2) // 4).tolist(), ((i * i + 8) // 16).tolist()]
    assert g["expected_lo"] == [1.0] + [2.0 ** -24] * 3
    assert g["expected_B"] == 1.0 + 2.0 ** -23
    q = np.array(g["q"], dtype=np.float32)
    cm = np.array(g["cm"], dtype=np.float32)
    cb = np.array(g["codebooks"], dtype=np.float32)
    T = oracle.lut_float(q, cm, cb, g["metric"])
    q8, lo, delta, B = oracle.quantize_lut(T, oracle.list_bias(q, cm, g["metric"]))
    assert q8.tolist() == g["expected_q8"]
    assert lo.tolist() == g["expected_lo"]
    assert float(delta) == g["expected_delta"]
    assert int(np.float32(B).view(np.uint32)) == int(g["expected_B_bits"], 16)
    S, a = oracle.scan_list(q8, delta, B, np.array(g["points_codes"]))
    assert S.tolist() == g["expected_S"]
    assert a.tolist() == g["expected_a"]
    # The exact squared distance to the reconstructed vector (cm = 0, so
    # x^ = concatenated codewords), in float64, within m * delta / 2.
    for c, av in zip(g["points_codes"], a.tolist()):
        xh = np.array([cb[j, c[j], 0] for j in range(4)], dtype=np.float64)
        exact = float(((q.astype(np.float64) - xh) ** 2).sum())
        assert abs(av - exact) <= 4 * float(delta) / 2


# ------------------------------------------------ brute force (section 1)

@pytest.mark.parametrize("name", ["c1", "c3"])
def test_all_lists_full_rerank_equals_brute_force(name):
    cfg, X, Q, _, index = cached_workload(name, 3000, 12, L=16, ncomp=12)
    res = oracle.search(index, X, Q, cfg.L, cfg.k, len(X))
    ids, dist = oracle.brute_force_knn(X, Q, cfg.k, cfg.metric)
    assert np.array_equal(res["ids"], ids)
    np.testing.assert_allclose(res["dist"], dist, rtol=1e-12, atol=1e-12)


def test_duplicates_tie_by_id():
    cfg, X, Q, _, index = cached_workload("c1", 2000, 5, L=8, ncomp=8)
    # Duplicate some rows; ties in both the approximate and exact distances
    # must resolve to the smaller id.
    X2 = X.copy()
    X2[1::2] = X2[0::2][: len(X2[1::2])]
    index2 = dict(index)
    index2["codes"] = index["codes"].copy()
    index2["codes"][1::2] = index["codes"][0::2][: len(X2[1::2])]
    # Put every point in the list of its duplicate source so ties are scanned.
    res = oracle.search(index2, X2, Q, cfg.L, 20, len(X2))
    ids, _ = oracle.brute_force_knn(X2, Q, 20, cfg.metric)
    assert np.array_equal(res["ids"], ids)
    # Candidate pool: equal (a, .) pairs appear with ascending ids.
    for qi in range(len(Q)):
        a, cid = res["cand_a"][qi], res["cand_id"][qi]
        same = a[1:] == a[:-1]
        assert np.all(cid[1:][same] > cid[:-1][same])


# ------------------------------------------ Eq. (1) reconstruction identity

@pytest.mark.parametrize("name", ["c1", "c3", "c2"])
def test_adc_equals_distance_to_reconstruction(name):
    cfg, X, Q, _, index = cached_workload(name, 4000, 6, L=12, ncomp=10)
    cb = index["codebooks"].astype(np.float64)
    m, K, dsub = cb.shape
    rng = make_rng(2, cfg.index)
    for qi in range(len(Q)):
        q = Q[qi]
        for l in rng.choice(cfg.L, size=3, replace=False):
            ids = index["list_ids"][index["list_offsets"][l]:index["list_offsets"][l + 1]]
            if len(ids) == 0:
                continue
            T = oracle.lut_float(q, index["cm"][l], index["codebooks"], cfg.metric).astype(np.float64)
            b = float(oracle.list_bias(q, index["cm"][l], cfg.metric))
            codes = index["codes"][ids].astype(np.int64)
            # Reconstruction x_hat = cm_l + concat_j B[j, code_j] in float64.
            xh = index["cm"][l].astype(np.float64)[None, :] + \
                cb[np.arange(m)[None, :], codes].reshape(len(ids), -1)
            q64 = q.astype(np.float64)
            adc = T[np.arange(m)[None, :], codes].sum(axis=1) + b
            if cfg.metric == "l2":
                ref = ((xh - q64) ** 2).sum(axis=1)
                scale = ((np.abs(q64) + np.abs(index["cm"][l]))[None, :] +
                         np.abs(cb[np.arange(m)[None, :], codes].reshape(len(ids), -1))) ** 2
            else:
                ref = -(xh @ q64)
                scale = np.abs(q64)[None, :] * (np.abs(index["cm"][l])[None, :] +
                                                 np.abs(cb[np.arange(m)[None, :], codes].reshape(len(ids), -1)))
            bound = 16 * (dsub + 2 + (cfg.d if cfg.metric == "ip" else 0)) * EPS32 * scale.sum(axis=1)
            assert np.all(np.abs(adc - ref) <= bound), (name, qi, l)


# --------------------------------------------------- quantisation (step 3)

@pytest.mark.parametrize("name", ["c1", "c3"])
def test_quantisation_error_bound(name):
    cfg, X, Q, _, index = cached_workload(name, 4000, 6, L=12, ncomp=10)
    m = cfg.m
    for qi in range(len(Q)):
        q = Q[qi]
        for l in range(cfg.L):
            ids = index["list_ids"][index["list_offsets"][l]:index["list_offsets"][l + 1]]
            T = oracle.lut_float(q, index["cm"][l], index["codebooks"], cfg.metric)
            bias = oracle.list_bias(q, index["cm"][l], cfg.metric)
            q8, lo, delta, B = oracle.quantize_lut(T, bias)
            # Table shape facts: every subspace has a 0 entry; the widest has 255.
            assert np.all(q8.min(axis=1) == 0)
            assert q8.max() == 255
            codes = index["codes"][ids].astype(np.int64)
            S, a = oracle.scan_list(q8, delta, B, codes)
            exact = T.astype(np.float64)[np.arange(m)[None, :], codes].sum(axis=1) + float(bias)
            slack = 8 * EPS32 * (np.abs(lo).astype(np.float64).sum() * 2 + abs(float(bias))
                                 + float(delta) * 255 * m)
            assert np.all(np.abs(a - exact) <= m * float(delta) / 2 * (1 + 1e-5) + slack)


def _grid_index(metric, L=4, per_list=60, d=12, seed=3):
    """Lossless grid case: d' = 1, codewords B[j,i] = i, integer data.

    Every residual component is an integer in 0..15 and equals a codeword,
    so the reconstruction is exact; the query is chosen so that each table's
    widest subspace range is exactly 255 (scale 1), so the 8-bit table is
    exact too and a(x) equals the exact distance.
    """
    rng = make_rng(seed)
    cm = rng.integers(20, 30, size=(L, d)).astype(np.float32)
    codes = rng.integers(0, 16, size=(L * per_list, d)).astype(np.uint8)
    assign = np.repeat(np.arange(L), per_list)
    X = cm[assign] + codes.astype(np.float32)
    cb = np.tile(np.arange(16, dtype=np.float32)[None, :, None], (d, 1, 1))
    nq = 6
    if metric == "l2":
        # Residual q - cm_l = -1 in dimension 0 for every list (range 255);
        # other residual components stay within [-1, 15] (ranges <= 255).
        cm[:, 0] = 30.0
        X = cm[assign] + codes.astype(np.float32)
        Q = np.zeros((nq, d), dtype=np.float32)
        Q[:, 0] = 29.0
        for t in range(1, d):
            lo_t = cm[:, t].max() - 1
            hi_t = cm[:, t].min() + 15
            Q[:, t] = rng.integers(int(lo_t), int(hi_t) + 1, size=nq) if hi_t >= lo_t else lo_t
        cp = cm.copy()
    else:
        # -q_j * i has range 15 |q_j|; max |q_j| = 17 gives range 255.
        Q = rng.integers(-17, 18, size=(nq, d)).astype(np.float32)
        Q[:, 0] = 17.0
        nrm = np.sqrt((cm.astype(np.float64) ** 2).sum(axis=1, keepdims=True))
        cp = (cm / nrm).astype(np.float32)
    order = np.argsort(assign, kind="stable")
    off = np.zeros(L + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.bincount(assign, minlength=L))
    index = dict(cm=cm, cp=cp, codebooks=cb, codes=codes, list_offsets=off,
                 list_ids=order.astype(np.int32), metric=metric)
    return index, X, Q


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_lossless_grid_is_exact(metric):
    index, X, Q = _grid_index(metric)
    L = len(index["cm"])
    k = 15
    for qi, q in enumerate(Q):
        for l in range(L):
            ids = index["list_ids"][index["list_offsets"][l]:index["list_offsets"][l + 1]]
            T = oracle.lut_float(q, index["cm"][l], index["codebooks"], metric)
            q8, lo, delta, B = oracle.quantize_lut(T, oracle.list_bias(q, index["cm"][l], metric))
            assert delta == np.float32(1.0)
            _, a = oracle.scan_list(q8, delta, B, index["codes"][ids])
            rows = X[ids].astype(np.float64)
            exact = ((rows - q) ** 2).sum(1) if metric == "l2" else -(rows @ q.astype(np.float64))
            assert np.array_equal(a.astype(np.float64), exact)
    # With every list probed and a pool of exactly k, the candidate pool is
    # already the exact answer (before any re-ranking).
    res = oracle.search(index, X, Q, L, k, k)
    ids, dist = oracle.brute_force_knn(X, Q, k, metric)
    assert np.array_equal(res["cand_id"], ids)
    assert np.array_equal(res["ids"], ids)


# ------------------------------------------------- coarse selection (step 1)

@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_coarse_ranking_matches_float64(name):
    cfg, X, Q, _, index = cached_workload(name, 6000, 20, L=64, ncomp=40)
    cp = index["cp"].astype(np.float64)
    n = 7
    for q in Q:
        s32 = oracle.coarse_scores(q, index["cp"], cfg.metric).astype(np.float64)
        q64 = q.astype(np.float64)
        if cfg.metric == "l2":
            s64 = ((cp - q64) ** 2).sum(1)
            mag = ((np.abs(cp) + np.abs(q64)) ** 2).sum(1)
        else:
            s64 = -(cp @ q64)
            mag = (np.abs(cp) * np.abs(q64)).sum(1)
        bound = (cfg.d + 2) * EPS32 * mag
        assert np.all(np.abs(s32 - s64) <= bound)
        P = oracle.select_probes(s32, n)
        P64 = np.lexsort((np.arange(len(s64)), s64))[:n]
        kth = s64[P64[-1]]
        for l in set(P.tolist()) ^ set(P64.tolist()):
            assert abs(s64[l] - kth) <= 2 * bound.max()
        assert np.all(np.diff(s32[P]) >= 0)


# ----------------------------------------------- scan and pool (steps 4-5)

def test_scan_and_pool_against_plain_python():
    rng = make_rng(4)
    m, n = 9, 300
    q8 = rng.integers(0, 256, size=(m, 16)).astype(np.uint8)
    codes = rng.integers(0, 16, size=(n, m)).astype(np.uint8)
    delta, B = np.float32(0.37), np.float32(-12.5)
    S, a = oracle.scan_list(q8, delta, B, codes)
    for x in range(n):
        s = sum(int(q8[j][codes[x][j]]) for j in range(m))
        assert S[x] == s
        assert a[x] == np.float32(B + np.float32(delta * np.float32(s)))
    # Pool: many exact ties on a; plain sorted() over (a, id) tuples.
    a_t = rng.integers(0, 20, size=500).astype(np.float32)
    ids = rng.permutation(10_000)[:500].astype(np.int64)
    for R in (1, 7, 100, 500, 800):
        ra, rid = oracle.top_r(a_t, ids, R)
        ref = sorted(zip(a_t.tolist(), ids.tolist()))[:R]
        assert list(zip(ra.tolist(), rid.tolist())) == ref


# ------------------------------------------------------------- edge cases

def test_edge_cases_small_pools_and_empty_lists():
    cfg, X, Q, _, index = cached_workload("c1", 1500, 4, L=10, ncomp=4)
    # Empty lists: drop all points of two lists.
    idx = dict(index)
    off = index["list_offsets"].copy()
    lid = index["list_ids"]
    keep = np.ones(len(lid), bool)
    for l in (0, 3):
        keep[off[l]:off[l + 1]] = False
    counts = np.diff(off).copy()
    counts[[0, 3]] = 0
    idx["list_offsets"] = np.concatenate(([0], np.cumsum(counts)))
    idx["list_ids"] = lid[keep]
    present = idx["list_ids"]
    # R larger than the probed points: pool holds every scanned point.
    res = oracle.search(idx, X, Q, 1, 5, 10_000)
    for qi in range(len(Q)):
        got = res["cand_id"][qi]
        n_valid = int((got >= 0).sum())
        assert np.all(got[n_valid:] == -1)
        assert np.all(np.isinf(res["cand_a"][qi][n_valid:]))
        assert set(got[:n_valid].tolist()) <= set(present.tolist())
    # k == R and nprobe == L with empty lists: equals brute force over the kept points.
    res = oracle.search(idx, X, Q, cfg.L, 5, len(X))
    ids_bf, _ = oracle.brute_force_knn(X[present], Q, 5, cfg.metric)
    assert np.array_equal(res["ids"], present[ids_bf])
    # Fewer candidates than k: padded with (-1, +inf).
    res = oracle.search(idx, X, Q, 1, 5, 3)
    assert np.all(res["ids"][:, 3:] == -1) and np.all(np.isinf(res["dist"][:, 3:]))


# ------------------------------------------- index construction (Alg. 1)

def test_encode_against_plain_python_and_reconstruction():
    rng = make_rng(5)
    n, m, dsub, L = 40, 6, 3, 4
    cb = rng.normal(size=(m, 16, dsub)).astype(np.float32)
    cm = rng.normal(size=(L, m * dsub)).astype(np.float32)
    lists = rng.integers(0, L, size=n)
    X = rng.normal(size=(n, m * dsub)).astype(np.float32)
    # Exact ties: make codeword 5 a copy of codeword 2 in every subspace.
    cb[:, 5] = cb[:, 2]
    codes = oracle.encode(X, cm, lists, cb)
    X64, cb64, cm64 = X.astype(np.float64), cb.astype(np.float64), cm.astype(np.float64)
    for x in range(n):
        r = X64[x] - cm64[lists[x]]
        for j in range(m):
            d = [sum((r[j * dsub + u] - cb64[j, i, u]) ** 2 for u in range(dsub)) for i in range(16)]
            best = min(d)
            # The FP32 choice is a minimiser up to rounding, never 5 (tie -> 2).
            assert d[codes[x, j]] <= best * (1 + 1e-5) + 1e-6
            assert codes[x, j] != 5
    # Lossless case: rows equal to a centroid plus codewords encode to them.
    want = rng.integers(0, 16, size=(n, m))
    want[want == 5] = 2
    Xl = cm[lists] + cb[np.arange(m)[None, :], want].reshape(n, -1)
    assert np.array_equal(oracle.encode(Xl.astype(np.float32), cm, lists, cb), want)


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_assign_lists_is_top1_of_float64_ranking(metric):
    cfg, X, Q, _, index = cached_workload("c1" if metric == "l2" else "c3", 3000, 4, L=16, ncomp=12)
    a = oracle.assign_lists(X[:300], index["cp"], metric)
    cp = index["cp"].astype(np.float64)
    for x, l in zip(X[:300].astype(np.float64), a):
        s64 = ((cp - x) ** 2).sum(1) if metric == "l2" else -(cp @ x)
        mag = ((np.abs(cp) + np.abs(x)) ** 2).sum(1) if metric == "l2" else (np.abs(cp) * np.abs(x)).sum(1)
        assert s64[l] <= s64.min() + 2 * (cfg.d + 2) * EPS32 * mag.max()


# ---------------------------------------------------------------------------
# Adaptive probing depth and re-rank size (section 4.2, Eq. 2).
# ---------------------------------------------------------------------------

def test_eq2_hand_worked_values_and_limits():
    F = np.float32
    # v_min 8, v_max 64, p0 0.25, p1 0.5, p 0.75: ReLU(0.5) * 1.25 = 0.625,
    # 56 * 0.625 = 35 (all exact in binary) -> 8 + 35 = 43.
    assert oracle.eq2(F(0.75), 8, 64, 0.25, 0.5) == 43
    # p <= p0: ReLU is 0 -> v_min.
    for p in (0.0, 0.1, 0.25):
        assert oracle.eq2(F(p), 8, 64, 0.25, 0.5) == 8
    # p = 1, p0 = 0, p1 = 0: the full range -> v_max; the min() caps overshoot.
    assert oracle.eq2(F(1.0), 8, 64, 0.0, 0.0) == 64
    assert oracle.eq2(F(1.0), 8, 64, 0.0, 3.0) == 64
    # v_min is clamped into [1, v_max]; the result never leaves [v_min, v_max].
    assert oracle.eq2(F(0.0), 0, 10, 0.5, 0.0) == 1
    assert oracle.eq2(F(0.9), 20, 10, 0.0, 0.0) == 10
    prev = 0
    for p in np.linspace(0, 1, 101, dtype=F):
        v = oracle.eq2(p, 4, 256, 0.2, 0.3)
        assert 4 <= v <= 256 and v >= prev  # non-decreasing in p for p1 >= -p0
        prev = v
    # floor, not rounding: 0.5 * (0.5 + 0.0) * 10 = 2.5 -> 2.
    assert oracle.eq2(F(0.5), 0 + 1, 11, 0.0, 0.0) == 1 + 2


def test_hardness_closed_form():
    F = np.float32
    # L2: ratio of nearest to K-th squared distance.
    assert oracle.hardness(np.array([1, 2, 4, 8], F), 3, "l2") == F(0.25)
    assert oracle.hardness(np.array([3, 3, 3], F), 3, "l2") == F(1.0)
    # K = 1: the nearest against itself -> 1 (hardest) unless it is 0.
    assert oracle.hardness(np.array([5, 9], F), 1, "l2") == F(1.0)
    assert oracle.hardness(np.array([0, 9], F), 2, "l2") == F(0.0)
    # IP: e = 1 + s (s = -<q, c_hat>), half the squared distance for unit q.
    p = oracle.hardness(np.array([-0.9, -0.5], F), 2, "ip")
    assert abs(float(p) - 0.2) < 1e-6
    # Negative e (non-unit query) clamps to 0; e_K <= 0 gives 1.
    assert oracle.hardness(np.array([-1.5, -0.5], F), 2, "ip") == F(0.0)
    assert oracle.hardness(np.array([-1.5, -1.2], F), 2, "ip") == F(1.0)


def test_adaptive_params_hand_worked():
    F = np.float32
    # Six lists scored out of order: sorted by (score, list) they are lists
    # 1, 3, 4, 0, 5, 2 with scores 1, 2, 4, 5, 8, 9.
    row = np.array([5.0, 1.0, 9.0, 2.0, 4.0, 8.0], F)
    # nprobe_init 3: e_1 = 1, e_3 = 4, p = 1/4. Eq. 2 with p0 = 0, p1 = 1:
    # ReLU(1/4) * (1/4 + 1) = 5/16 (exact).
    #   nprobe:  v_min 2, v_max 6:  2 + floor(4 * 5/16 = 1.25) = 3
    #   reorder: v_min 20 (reorder_min, within [k, R] = [10, 100]), v_max 100:
    #            20 + floor(80 * 5/16 = 25) = 45
    npb, reo, p = oracle.adaptive_params(row, 6, "l2", 3, 2, 20, 100, 10, 0.0, 1.0)
    assert (npb, reo, float(p)) == (3, 45, 0.25)
    # nprobe_init above nprobe_max: K = nprobe_max = 2, e_2 = 2, p = 1/2,
    # ReLU(1/2) * 3/2 = 3/4; nprobe has v_min = v_max = 2; reorder
    # 20 + floor(80 * 3/4 = 60) = 80.
    npb, reo, p = oracle.adaptive_params(row, 2, "l2", 3, 2, 20, 100, 10, 0.0, 1.0)
    assert (npb, reo, float(p)) == (2, 80, 0.5)
    # reorder_min below k is raised to k = 10: 10 + floor(90 * 5/16 = 28.125) = 38.
    npb, reo, p = oracle.adaptive_params(row, 6, "l2", 3, 2, 4, 100, 10, 0.0, 1.0)
    assert (npb, reo) == (3, 38)
    # Inner product: e = 1 + s. Sorted scores -0.75, -0.5, 0 (lists 1, 3, 2):
    # e_1 = 1/4, e_3 = 1, p = 1/4 as above -> (3, 45). Read as L2 (e = s),
    # e_3 = 0 would give p = 1 and (6, 100).
    row_ip = np.array([0.5, -0.75, 0.0, -0.5, 0.25, 0.75], F)
    npb, reo, p = oracle.adaptive_params(row_ip, 6, "ip", 3, 2, 20, 100, 10, 0.0, 1.0)
    assert (npb, reo, float(p)) == (3, 45, 0.25)


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_adaptive_search_is_static_search_at_chosen_parameters(name):
    cfg, X, Q, nprobe, index = cached_workload(name, 3000, 10, L=24, ncomp=16)
    ad = dict(nprobe_init=3, nprobe_min=2, reorder_min=cfg.k, p0=0.3, p1=0.5)
    npmax = np.full(len(Q), 12, dtype=np.int64)
    res = oracle.search(index, X, Q, npmax, cfg.k, 60, adaptive=ad)
    used, reo = res["nprobe_used"], res["reorder_used"]
    assert ((used >= 2) & (used <= 12)).all() and ((reo >= cfg.k) & (reo <= 60)).all()
    assert len(set(used.tolist())) > 1  # the queries differ in difficulty
    # The same pools as the static search with the chosen nprobe, and the
    # re-rank over the reorder best of them.
    st = oracle.search(index, X, Q, used, cfg.k, 60)
    assert np.array_equal(st["cand_id"], res["cand_id"])
    for qi in range(len(Q)):
        ids, _ = oracle.rerank(Q[qi], X, st["cand_id"][qi][:reo[qi]], cfg.k, index["metric"])
        assert np.array_equal(ids, res["ids"][qi])
    # Limits: p0 above every p -> the minima; p0 below, p1 large -> static.
    lo = oracle.search(index, X, Q, npmax, cfg.k, 60,
                       adaptive=dict(ad, p0=2.0))
    assert (lo["nprobe_used"] == 2).all() and (lo["reorder_used"] == cfg.k).all()
    hi = oracle.search(index, X, Q, npmax, cfg.k, 60,
                       adaptive=dict(ad, p0=-1.0, p1=100.0))
    full = oracle.search(index, X, Q, npmax, cfg.k, 60)
    assert (hi["nprobe_used"] == 12).all() and (hi["reorder_used"] == 60).all()
    assert np.array_equal(hi["ids"], full["ids"])


# ---------------------------------------------------------------------------
# Component filtration (section 4.3).
# ---------------------------------------------------------------------------

def test_component_filter_hand_example():
    X = np.array([[0, 1, 5, 2], [0, 2, 5, 0], [0, 3, 5, 4], [1, 4, 5, 6]], np.float32)
    # col 0: mu 0.25, sigma 0.433, three zeros, |1-mu| > sigma -> 3/4
    # col 1: mu 2.5, sigma 1.118, 2 and 3 within -> 2/4
    # col 2: constant, sigma 0 -> every component within -> 4/4
    # col 3: mu 3, sigma 2.236, one zero, 2 and 4 within, 6 outside -> 3/4
    keep, share = oracle.component_filter(X, 0.75)
    assert np.allclose(share, [0.75, 0.5, 1.0, 0.75])
    assert keep.tolist() == [0, 1, 3]
    assert oracle.component_filter(X, 0.7)[0].tolist() == [1]


def test_component_filter_distributions_and_product_agree():
    from paper_2511_03298_amd.train import component_filter as product_filter
    rng = make_rng(7)
    n = 200_000
    X = np.stack([rng.standard_normal(n),                      # Gaussian: ~68.3 % within 1 sigma
                  rng.uniform(-1, 1, n),                       # uniform: 1/sqrt(3) ~ 57.7 %
                  np.full(n, 3.0),                             # constant: 100 %
                  np.where(rng.random(n) < 0.96, 0.0, 5.0),    # 96 % zeros
                  ], axis=1).astype(np.float32)
    keep, share = oracle.component_filter(X, 0.9)
    assert abs(share[0] - 0.6827) < 0.005 and abs(share[1] - 1 / np.sqrt(3)) < 0.005
    assert share[2] == 1.0 and share[3] >= 0.95
    assert keep.tolist() == [0, 1]
    assert product_filter(X, 0.9).tolist() == keep.tolist()
    from workloads import make_workload, scaled
    cfg = scaled("c6", 8000, 4, L=16, ncomp=16)
    Xw, _, _ = make_workload(cfg)
    kw = oracle.component_filter(Xw, 0.9)[0]
    assert kw.tolist() == list(range(cfg.d - cfg.background))
    assert product_filter(Xw, 0.9).tolist() == kw.tolist()


def test_filtered_search_all_lists_equals_brute_force_on_full_rows():
    # Dropped dimensions that are exactly 0 carry no distance: with every
    # list probed and a full re-rank against the full rows, the filtered
    # search is exact k-NN on the full data.
    from workloads import train_index
    cfg, X, Q, _, _ = cached_workload("c1", 2500, 8, L=12, ncomp=10)
    Xz = np.concatenate([X, np.zeros((len(X), 8), np.float32)], axis=1)
    Qz = np.concatenate([Q, np.zeros((len(Q), 8), np.float32)], axis=1)
    keep, _ = oracle.component_filter(Xz, 0.9)
    assert keep.tolist() == list(range(X.shape[1]))
    idx = train_index(Xz, dataclasses.replace(cfg, d=Xz.shape[1], m=cfg.m * Xz.shape[1] // cfg.d),
                      dims=keep)
    res = oracle.search(idx, Xz, Qz, cfg.L, cfg.k, len(Xz))
    bf_ids, bf_d = oracle.brute_force_knn(Xz, Qz, cfg.k, cfg.metric)
    assert np.array_equal(res["ids"], bf_ids)


# ---------------------------------- spilled assignment (section 4.6.2, SOAR)

def test_spill_assign_hand_example():
    # x = (1, 0) in list 0 (c = origin), so r = (1, 0). List 1 at (2, 0) leaves
    # r' = (-1, 0), parallel to r: loss 1 + lam * 1. List 2 at (1, 1.5) leaves
    # r' = (0, -1.5), orthogonal to r: loss 2.25. lam = 0 takes the nearer
    # list 1; lam = 1.5 (loss 2.5) or more takes the orthogonal list 2.
    X = np.array([[1.0, 0.0]], np.float32)
    cm = np.array([[0.0, 0.0], [2.0, 0.0], [1.0, 1.5]], np.float32)
    prim = np.array([0])
    assert oracle.spill_assign(X, cm, prim, 0.0).tolist() == [1]
    assert oracle.spill_assign(X, cm, prim, 1.0).tolist() == [1]
    assert oracle.spill_assign(X, cm, prim, 1.5).tolist() == [2]
    assert oracle.spill_assign(X, cm, prim, 4.0).tolist() == [2]
    # Exact tie (mirror-image lists): the smaller list index.
    X = np.array([[0.0, 1.0]], np.float32)
    cm = np.array([[0.0, 0.0], [1.0, 1.0], [-1.0, 1.0]], np.float32)
    assert oracle.spill_assign(X, cm, prim, 1.0).tolist() == [1]
    # A row on its centroid (r = 0): the nearest other list.
    X = np.array([[0.0, 0.0]], np.float32)
    cm = np.array([[0.0, 0.0], [3.0, 0.0], [0.0, 2.0]], np.float32)
    assert oracle.spill_assign(X, cm, prim, 1.0).tolist() == [2]


def test_spill_assign_brute_force_projection_form():
    rng = make_rng(8)
    X = rng.standard_normal((40, 6))
    cm = rng.standard_normal((9, 6))
    prim = rng.integers(0, 9, size=40)
    for lam in (0.0, 0.7, 1.0, 3.0):
        got = oracle.spill_assign(X, cm, prim, lam)
        for i in range(len(X)):
            r = X[i] - cm[prim[i]]
            P = np.outer(r, r) / float(r @ r)      # projection onto r
            losses = []
            for l in range(len(cm)):
                if l == prim[i]:
                    continue
                rp = X[i] - cm[l]
                pr = P @ rp
                losses.append((float(rp @ rp) + lam * float(pr @ pr), l))
            assert got[i] == min(losses)[1]
        if lam == 0.0:
            # lam = 0: the second-nearest list (the nearest other than p).
            d = ((X[:, None, :] - cm[None]) ** 2).sum(axis=2)
            d[np.arange(len(X)), prim] = np.inf
            assert got.tolist() == np.argmin(d, axis=1).tolist()
    # Larger lam: the chosen second residuals are less aligned with r.
    cos0, cos3 = [], []
    for lam, acc in ((0.0, cos0), (3.0, cos3)):
        sp = oracle.spill_assign(X, cm, prim, lam)
        for i in range(len(X)):
            r, rp = X[i] - cm[prim[i]], X[i] - cm[sp[i]]
            acc.append(abs(r @ rp) / np.linalg.norm(r) / np.linalg.norm(rp))
    assert np.mean(cos3) < np.mean(cos0)


def test_spill_lists_of_the_trainer_agree_with_oracle():
    from workloads.train import _spill_lists
    cfg, X, Q, _, index = cached_workload("c1", 3000, 4, L=16, ncomp=12)
    off = index["list_offsets"]
    prim = np.empty(len(X), np.int64)
    prim[index["list_ids"]] = np.repeat(np.arange(cfg.L), np.diff(off))
    ref = oracle.spill_assign(X, index["cm"], prim, 1.0)
    got = _spill_lists(X, index["cm"], prim, 1.0)
    assert (got == ref).mean() >= 0.99
    assert (got != prim).all()


def test_unique_pool_against_greedy_selection():
    # Repeated ids with different and equal values; the pool keeps each id
    # once at its smallest value. Greedy reference: take the smallest
    # remaining (a, id) pair, then drop every entry of that id.
    rng = make_rng(9)
    a = rng.integers(0, 30, size=400).astype(np.float32)
    ids = rng.integers(0, 150, size=400).astype(np.int64)
    for R in (1, 5, 60, 150, 400):
        ra, rid = oracle.top_r_unique(a, ids, R)
        rest = sorted(zip(a.tolist(), ids.tolist()))
        ref = []
        while rest and len(ref) < R:
            v, i = rest[0]
            ref.append((v, i))
            rest = [(w, j) for w, j in rest if j != i]
        assert list(zip(ra.tolist(), rid.tolist())) == ref
        assert len(set(rid.tolist())) == len(rid)


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_spilled_search_all_lists_equals_brute_force(name):
    from workloads import spill_index
    cfg, X, Q, _, index = cached_workload(name, 2500, 8, L=12, ncomp=10)
    sp = spill_index(X, index, 1.0)
    assert len(sp["list_ids"]) == 2 * len(X) and sp["codes"].shape[0] == 2 * len(X)
    res = oracle.search(sp, X, Q, cfg.L, cfg.k, len(X))
    ids, dist = oracle.brute_force_knn(X, Q, cfg.k, cfg.metric)
    assert np.array_equal(res["ids"], ids)
    for qi in range(len(Q)):
        assert sorted(res["cand_id"][qi].tolist()) == list(range(len(X)))


def test_spilled_pool_is_best_copy_of_each_point():
    # Every pooled point's value is the smaller of its copies' values in the
    # probed lists, recomputed from the stage tables and the entry codes;
    # points in no probed list are absent, and nothing better is left out.
    from workloads import spill_index
    cfg, X, Q, _, index = cached_workload("c1", 3000, 6, L=16, ncomp=12)
    sp = spill_index(X, index, 1.0)
    off, lid, codes = sp["list_offsets"], sp["list_ids"], sp["codes"]
    R = 150
    res = oracle.search(sp, X, Q, 4, cfg.k, R, want_stages=True)
    for qi in range(len(Q)):
        best = {}
        for l in res["probes"][qi]:
            q8, lo, delta, B = res["luts"][(qi, int(l))]
            for e in range(off[l], off[l + 1]):
                s = sum(int(q8[j][codes[e][j]]) for j in range(codes.shape[1]))
                v = np.float32(B + np.float32(delta * np.float32(s)))
                i = int(lid[e])
                best[i] = min(best.get(i, np.float32(np.inf)), v)
        ref = sorted((v, i) for i, v in best.items())[:R]
        got = list(zip(res["cand_a"][qi].tolist(), res["cand_id"][qi].tolist()))
        assert got[:len(ref)] == [(float(v), i) for v, i in ref]
