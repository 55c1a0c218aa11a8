"""GPU parity: every stage of the HIP path against the CPU oracle.

Probe sets, quantised tables (bytes, offsets, scale, constant), candidate
pools (value, id) are compared bit for bit; re-ranked distances within 1e-5
relative of FP64, final ids equal up to the FP64 tie band. All calls go
through the C ABI (libivfpq.so) via the Python binding.
"""

import dataclasses
import sys

import numpy as np
import pytest

import oracle
from conftest import cached_workload
from gpu_helpers import check_final, oracle_stages, unpack_tables

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_03298_amd as ivf
    return ivf


# name -> (workload, n, nq, L, ncomp, overrides)
CASES = {
    "c1": ("c1", 10_000, 100, None, None, {}),
    "c2s": ("c2", 40_000, 40, 64, 40, dict(nprobe=(6, 6))),
    "c3s": ("c3", 30_000, 40, 80, 80, dict(nprobe=(8, 32))),
    "c4s": ("c4", 40_000, 20, 64, 64, dict(nprobe=(8, 8))),
    "c5s": ("c5", 12_000, 12, 32, 32, dict(nprobe=(4, 16))),
    # L2 with 64 < m <= 128: two subspaces per lane in the batched table
    # build, 8-query items (m = 128) and 16-query items (m = 96).
    "c6u": ("c6", 20_000, 30, 32, 32, dict(nprobe=(6, 6))),
    "c2w": ("c2", 20_000, 30, 32, 32, dict(nprobe=(6, 6), d=192, m=96)),
}

_STATE = {}


def case(name):
    if name not in _STATE:
        ivf = _gpu()
        wl, n, nq, L, ncomp, kw = CASES[name]
        cfg, X, Q, nprobe, index = cached_workload(wl, n, nq, L=L, ncomp=ncomp, **kw)
        print(f"[case {name}] n={cfg.n} d={cfg.d} L={cfg.L} m={cfg.m} nq={cfg.nq} "
              f"R={cfg.R} k={cfg.k} metric={cfg.metric}", flush=True)
        g = ivf.GpuIndex.from_index(index, X, base_dtype=cfg.base_dtype)
        res = oracle_stages(index, X, Q, nprobe, cfg.k, cfg.R)
        _STATE[name] = (cfg, X, Q, nprobe, index, g, res)
    return _STATE[name]


def probes_tensor(res, nprobe):
    mx = int(max(nprobe))
    P = np.full((len(nprobe), mx), -1, dtype=np.int32)
    for qi, p in enumerate(res["probes"]):
        P[qi, :len(p)] = p
    return torch.from_numpy(P)


@pytest.mark.parametrize("name", list(CASES))
def test_pack_roundtrip(name):
    cfg, X, Q, nprobe, index, g, res = case(name)
    lay = g.layout()
    tables = g.tables.cpu().numpy()
    codes, slot_ids, pad = unpack_tables(tables, lay, cfg.m)
    assert np.all(pad == 0)
    boff = tables[lay.block_offsets:lay.block_offsets + (cfg.L + 1) * 4].view(np.int32)
    off, lid = index["list_offsets"], index["list_ids"]
    for l in range(cfg.L):
        ids = lid[off[l]:off[l + 1]]
        s0 = boff[l] * 64
        nblk = boff[l + 1] - boff[l]
        assert nblk == (len(ids) + 63) // 64
        assert np.array_equal(slot_ids[s0:s0 + len(ids)], ids)
        assert np.all(slot_ids[s0 + len(ids):s0 + nblk * 64] == -1)
        assert np.array_equal(codes[s0:s0 + len(ids)], index["codes"][ids])


@pytest.mark.parametrize("name", list(CASES))
def test_probe_sets_bit_exact(name):
    cfg, X, Q, nprobe, index, g, res = case(name)
    got = g.debug_probes(Q, nprobe).cpu().numpy()
    for qi, p in enumerate(res["probes"]):
        assert np.array_equal(got[qi, :len(p)], p), qi
        assert np.all(got[qi, len(p):] == -1)


@pytest.mark.parametrize("name", list(CASES))
def test_luts_bit_exact(name):
    cfg, X, Q, nprobe, index, g, res = case(name)
    P = probes_tensor(res, nprobe)
    lut, lo, delta, B = [t.cpu().numpy() for t in g.debug_luts(Q, P, nprobe)]
    for qi, p in enumerate(res["probes"]):
        for pi, l in enumerate(p):
            q8, lo_o, d_o, B_o = res["luts"][(qi, int(l))]
            assert np.array_equal(lut[qi, pi], q8), (qi, l)
            assert np.array_equal(lo[qi, pi].view(np.uint32), lo_o.view(np.uint32)), (qi, l)
            assert delta[qi, pi].view(np.uint32) == np.float32(d_o).view(np.uint32), (qi, l)
            assert B[qi, pi].view(np.uint32) == np.float32(B_o).view(np.uint32), (qi, l)


@pytest.mark.parametrize("name", list(CASES))
def test_batched_luts_bit_exact(name):
    # The batched form's own table builders (per-item L2 builders for every
    # word count used here, the per-query IP table plus list bias), per
    # (query, probed list), against the oracle's tables.
    cfg, X, Q, nprobe, index, g, res = case(name)
    P = probes_tensor(res, nprobe)
    lut, delta, B = [t.cpu().numpy() for t in g.debug_batched_luts(Q, P, nprobe)]
    for qi, p in enumerate(res["probes"]):
        for pi, l in enumerate(p):
            q8, lo_o, d_o, B_o = res["luts"][(qi, int(l))]
            assert np.array_equal(lut[qi, pi], q8), (qi, l)
            assert delta[qi, pi].view(np.uint32) == np.float32(d_o).view(np.uint32), (qi, l)
            assert B[qi, pi].view(np.uint32) == np.float32(B_o).view(np.uint32), (qi, l)


@pytest.mark.parametrize("name", list(CASES))
def test_candidates_bit_exact(name):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    P = probes_tensor(res, nprobe)
    keys = g.debug_candidates(Q, P, nprobe, cfg.R).cpu().numpy()
    a, ids = ivf.decode_keys(keys)
    assert np.array_equal(ids, res["cand_id"])
    assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32))


@pytest.mark.parametrize("name", list(CASES))
def test_search_end_to_end(name):
    cfg, X, Q, nprobe, index, g, res = case(name)
    ids, dist = g.search(Q, nprobe, cfg.k, cfg.R)
    torch.cuda.synchronize()
    assert g.device_error() == 0
    check_final(ids.cpu().numpy(), dist.cpu().numpy(), res, X, Q, cfg.metric,
                exact_ids=(cfg.dist == "int255"))


def test_u8_and_f32_rows_rerank_identically():
    # Byte-valued rows stored as u8 are widened exactly: the same search on
    # FP32 rows gives bit-identical distances (integer sums stay below 2^24).
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case("c2s")
    assert cfg.dist == "int255" and cfg.base_dtype == "f32"
    g8 = ivf.GpuIndex.from_index(index, X, base_dtype="u8")
    for opts in (ivf.make_opts(), ivf.make_opts(form="batched", coarse="bf16")):
        i8, d8 = g8.search(Q, nprobe, cfg.k, cfg.R, opts=opts)
        i32, d32 = g.search(Q, nprobe, cfg.k, cfg.R, opts=opts)
        assert torch.equal(i8, i32) and torch.equal(d8.view(torch.int32), d32.view(torch.int32))
    check_final(i8.cpu().numpy(), d8.cpu().numpy(), res, X, Q, cfg.metric, exact_ids=True)


@pytest.mark.parametrize("form,rounds", [("plain", 0), ("batched", 1), ("batched", 3)])
@pytest.mark.parametrize("name", ["c1", "c3s"])
def test_repeat_runs_bit_identical(name, form, rounds):
    # Ten runs, bit for bit: the survivors' append order varies from run to
    # run in the batched form, the selected keys and the results do not.
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    opts = ivf.make_opts(form=form, coarse="bf16", rounds=rounds)
    outs = []
    for _ in range(10):
        ids, dist = g.search(Q, nprobe, cfg.k, cfg.R, opts=opts)
        outs.append((ids.cpu().numpy(), dist.cpu().numpy().view(np.uint32)))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


@pytest.mark.parametrize("form", ["plain", "batched"])
def test_two_streams_in_flight(form):
    # One index searched on two streams at once, each search with its own
    # workspace (the binding keeps one per stream): both equal the oracle.
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case("c3s")
    opts = ivf.make_opts(form=form)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    outs = []
    for s in streams:
        with torch.cuda.stream(s):
            outs.append(g.search(Q, nprobe, cfg.k, cfg.R, opts=opts))
    torch.cuda.synchronize()
    got = [(ids.cpu().numpy(), dist.cpu().numpy()) for ids, dist in outs]
    for ids, dist in got:
        check_final(ids, dist, res, X, Q, cfg.metric)
    assert np.array_equal(got[0][0], got[1][0])
    assert np.array_equal(got[0][1].view(np.uint32), got[1][1].view(np.uint32))
    assert g.device_error() == 0


def test_query_count_limit():
    # More than 2^20 queries per call are rejected on the host before any
    # device work; 2^20 itself is a valid size.
    import ctypes
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case("c1")
    o = ivf.make_opts()
    lib = ivf.lib()
    assert lib.ivf_search_workspace_bytes(g._h, 1 << 20, 1, 1, 1, ctypes.byref(o)) > 0
    assert lib.ivf_search_workspace_bytes(g._h, (1 << 20) + 1, 1, 1, 1, ctypes.byref(o)) == 0
    assert "2^20" in ivf.last_error()


def test_nprobe_one_and_all_lists():
    cfg, X, Q, nprobe, index, g, _ = case("c1")
    for npb in (1, cfg.L):
        res = oracle.search(index, X, Q[:20], npb, cfg.k, cfg.R)
        ids, dist = g.search(Q[:20], npb, cfg.k, cfg.R)
        check_final(ids.cpu().numpy(), dist.cpu().numpy(), res, X, Q[:20], cfg.metric)


def test_pool_larger_than_probed_points_and_k_equals_R():
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, _ = case("c1")
    R = 2048
    res = oracle.search(index, X, Q[:10], 1, 7, R)
    P = torch.from_numpy(np.stack([oracle.select_probes(
        oracle.coarse_scores(q, index["cp"], cfg.metric), 1) for q in Q[:10]]).astype(np.int32))
    keys = g.debug_candidates(Q[:10], P, 1, R).cpu().numpy()
    a, ids = ivf.decode_keys(keys)
    assert np.array_equal(ids, res["cand_id"])
    assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32))
    # k == R: every candidate comes back, ordered by exact distance.
    res = oracle.search(index, X, Q[:10], 2, 50, 50)
    gi, gd = g.search(Q[:10], 2, 50, 50)
    check_final(gi.cpu().numpy(), gd.cpu().numpy(), res, X, Q[:10], cfg.metric)


def test_empty_lists_and_tiny_index():
    ivf = _gpu()
    cfg, X, Q, nprobe, index, _, _ = case("c1")
    idx = dict(index)
    off = index["list_offsets"]
    counts = np.diff(off).copy()
    keep = np.ones(len(index["list_ids"]), bool)
    for l in (0, 5, 9):
        keep[off[l]:off[l + 1]] = False
        counts[l] = 0
    idx["list_offsets"] = np.concatenate(([0], np.cumsum(counts)))
    idx["list_ids"] = index["list_ids"][keep]
    # The index covers fewer points than X; ids still index rows of X.
    g = ivf.GpuIndex(X, idx["cm"], idx["codebooks"], idx["codes"], idx["list_offsets"],
                     idx["list_ids"], cfg.metric, probe_centroids=idx["cp"])
    for npb in (1, 3, cfg.L):
        res = oracle.search(idx, X, Q[:16], npb, cfg.k, cfg.R)
        ids, dist = g.search(Q[:16], npb, cfg.k, cfg.R)
        check_final(ids.cpu().numpy(), dist.cpu().numpy(), res, X, Q[:16], cfg.metric)
    # A tiny index: fewer points than one 64-point block, fewer than k.
    small = dict(index)
    sel = index["list_ids"][:5]
    small_off = np.zeros(cfg.L + 1, dtype=np.int64)
    small_off[1:] = 5
    small["list_offsets"] = small_off
    small["list_ids"] = np.sort(sel).astype(np.int32)
    g2 = ivf.GpuIndex(X, small["cm"], small["codebooks"], small["codes"], small_off,
                      small["list_ids"], cfg.metric, probe_centroids=small["cp"])
    res = oracle.search(small, X, Q[:4], cfg.L, 10, 100)
    ids, dist = g2.search(Q[:4], cfg.L, 10, 100)
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    assert np.all(ids[:, 5:] == -1) and np.all(np.isinf(dist[:, 5:]))
    check_final(ids, dist, res, X, Q[:4], cfg.metric)


def test_invalid_nprobe_sets_error_word():
    cfg, X, Q, nprobe, index, g, _ = case("c1")
    npb = np.full(8, 4, dtype=np.int32)
    npb[3] = 0
    npb[5] = 99
    ids, dist = g.search(Q[:8], npb, cfg.k, cfg.R, max_nprobe=8)
    torch.cuda.synchronize()
    assert g.device_error() == 1
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    for qi in (3, 5):
        assert np.all(ids[qi] == -1) and np.all(np.isnan(dist[qi]))
    res = oracle.search(index, X, Q[:8], 4, cfg.k, cfg.R)
    for qi in (0, 1, 2, 4, 6, 7):
        assert np.array_equal(ids[qi][ids[qi] >= 0].shape, res["ids"][qi][res["ids"][qi] >= 0].shape)
    assert g.device_error() == 0  # cleared by the read


@pytest.mark.parametrize("form", ["plain", "batched"])
def test_bad_probe_rows_rejected(form):
    # Caller-given probe rows: a list named twice or outside [0, L) sets bit 2
    # of the error word; that row is answered as (-1, NaN), the others are
    # searched normally.
    ivf = _gpu()
    cfg, X, Q, nprobe, index, g, res = case("c1")
    nq = 6
    P = probes_tensor({"probes": res["probes"][:nq]}, nprobe[:nq]).clone()
    npb = np.asarray(nprobe[:nq], dtype=np.int32)
    P[1, 2] = P[1, 0]          # repeated list
    P[4, 1] = cfg.L            # out of range
    opts = ivf.make_opts(form=form)
    ids, dist = g.search_with_probes(Q[:nq], P, npb, cfg.k, cfg.R, opts=opts)
    torch.cuda.synchronize()
    assert g.device_error() == 2
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    for qi in (1, 4):
        assert np.all(ids[qi] == -1) and np.all(np.isnan(dist[qi]))
    ok = [0, 2, 3, 5]
    sub = {k: v[ok] for k, v in res.items() if k in ("ids", "dist")}
    check_final(ids[ok], dist[ok], sub, X, Q[ok], cfg.metric)
    assert g.device_error() == 0


def test_list_id_out_of_range_rejected_at_build():
    # An unspilled index whose list names a row outside [0, n): the build
    # reports it instead of reading codes out of bounds.
    ivf = _gpu()
    cfg, X, Q, nprobe, index, g, _ = case("c1")
    lid = index["list_ids"].copy()
    off = index["list_offsets"]
    lid[off[1]] = len(X) + 5
    with pytest.raises(ivf.IvfError, match="outside"):
        ivf.GpuIndex(X, index["cm"], index["codebooks"], index["codes"], off, lid,
                     cfg.metric, probe_centroids=index["cp"])
    lid[off[1]] = -3
    with pytest.raises(ivf.IvfError, match="outside"):
        ivf.GpuIndex(X, index["cm"], index["codebooks"], index["codes"], off, lid,
                     cfg.metric, probe_centroids=index["cp"])


@pytest.mark.parametrize("name", ["c2s", "c4s"])
def test_multiple_probed_lists_ragged_batch(name):
    # nq not a multiple of any tile, per-query nprobe spanning 1..L.
    cfg, X, Q, nprobe, index, g, _ = case(name)
    rng = np.random.default_rng(7)
    nq = 13
    npb = rng.integers(1, cfg.L + 1, size=nq).astype(np.int32)
    res = oracle.search(index, X, Q[:nq], npb, cfg.k, cfg.R)
    ids, dist = g.search(Q[:nq], npb, cfg.k, cfg.R, max_nprobe=cfg.L)
    check_final(ids.cpu().numpy(), dist.cpu().numpy(), res, X, Q[:nq], cfg.metric,
                exact_ids=(cfg.dist == "int255"))


# ---------------------------------------------------------------------------
# MFMA coarse forms: approximate scores, widened pre-selection, canonical
# re-score.
# ---------------------------------------------------------------------------

UNIT = {"f32": 2.0 ** -22, "bf16": 2.0 ** -7, "fp8": 2.0 ** -3}


@pytest.mark.parametrize("coarse", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("name", ["c1", "c2s", "c3s", "c5s"])
def test_mfma_scores_within_operand_rounding(name, coarse):
    cfg, X, Q, nprobe, index, g, res = case(name)
    S = g.debug_coarse_scores(Q, coarse).cpu().numpy().astype(np.float64)
    cp = index["cp"].astype(np.float64)
    q64 = Q.astype(np.float64)
    dot = q64 @ cp.T
    ref = (cp ** 2).sum(1)[None, :] - 2 * dot if cfg.metric == "l2" else -dot
    mag = np.abs(q64) @ np.abs(cp).T
    fac = 2.0 if cfg.metric == "l2" else 1.0
    err = np.abs(S - ref)
    # |c|^2 is exact FP32 (any order), so the error is the product's.
    slack = 1e-5 * (np.abs(ref) + 1e-30) + cfg.d * 2.0 ** -23 * fac * mag
    assert np.all(err <= fac * UNIT[coarse] * mag + slack)
    # Low precision: typical error far below the worst case (catches a
    # wrong operand scale or FP8 format, which shift every product).
    if coarse != "f32":
        assert np.median(err / (fac * mag + 1e-30)) <= UNIT[coarse] / 4


def canonical_sorted(index, q, metric, lists):
    s = oracle.coarse_scores(q, index["cp"], metric)
    return s[np.asarray(lists, dtype=np.int64)]


@pytest.mark.parametrize("coarse", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("name", ["c1", "c2s", "c3s", "c4s", "c5s"])
def test_mfma_probe_sets(name, coarse):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    # Widening to every list: the canonical re-score decides alone -> exact.
    full = g.debug_probes(Q, nprobe, opts=ivf.make_opts(coarse=coarse, widen=cfg.L)).cpu().numpy()
    for qi, p in enumerate(res["probes"]):
        assert np.array_equal(full[qi, :len(p)], p), qi
    got = g.debug_probes(Q, nprobe, opts=ivf.make_opts(coarse=coarse, widen=2)).cpu().numpy()
    differ = 0
    for qi, p in enumerate(res["probes"]):
        mine = got[qi, :len(p)]
        if np.array_equal(mine, p):
            continue
        differ += 1
        # Still a valid widened choice: distinct lists in canonical order,
        # each rank no better than the true canonical top-nprobe.
        assert len(set(mine.tolist())) == len(p)
        sm = canonical_sorted(index, Q[qi], cfg.metric, mine)
        so = canonical_sorted(index, Q[qi], cfg.metric, p)
        assert np.all(np.diff(sm) >= 0) and np.all(sm >= so)
    print(f"[{name}/{coarse}] probe sets differing from the canonical top-nprobe: "
          f"{differ}/{len(Q)}")
    if coarse == "f32":
        assert differ == 0
    else:
        assert differ <= max(1, len(Q) // 10)


@pytest.mark.parametrize("coarse", ["bf16", "fp8"])
@pytest.mark.parametrize("name", ["c1", "c3s", "c5s"])
def test_mfma_additive_margin(name, coarse):
    # widen 1 plus a margin of lists: min(L, nprobe + add) lists re-scored.
    # A margin covering every list is exact; a smaller one gives valid sets
    # (distinct lists in canonical order, none better than the true ones).
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    full = g.debug_probes(Q, nprobe, opts=ivf.make_opts(coarse=coarse, widen=1,
                                                        widen_add=cfg.L)).cpu().numpy()
    for qi, p in enumerate(res["probes"]):
        assert np.array_equal(full[qi, :len(p)], p), qi
    for add in (0, 4):
        got = g.debug_probes(Q, nprobe, opts=ivf.make_opts(coarse=coarse, widen=1,
                                                           widen_add=add)).cpu().numpy()
        for qi, p in enumerate(res["probes"]):
            mine = got[qi, :len(p)]
            assert len(set(mine.tolist())) == len(p) and np.all(got[qi, len(p):] == -1)
            sm = canonical_sorted(index, Q[qi], cfg.metric, mine)
            so = canonical_sorted(index, Q[qi], cfg.metric, p)
            assert np.all(np.diff(sm) >= 0) and np.all(sm >= so)
    with pytest.raises(ivf.IvfError, match="widen_add"):
        g.debug_probes(Q, nprobe, opts=ivf.make_opts(coarse=coarse, widen=1, widen_add=-1))


@pytest.mark.parametrize("coarse", ["bf16", "fp8"])
@pytest.mark.parametrize("name", ["c2s", "c3s"])
def test_mfma_search_matches_oracle_on_equal_probe_sets(name, coarse):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    opts = ivf.make_opts(coarse=coarse, widen=4)
    probes = g.debug_probes(Q, nprobe, opts=opts).cpu().numpy()
    ids, dist = g.search(Q, nprobe, cfg.k, cfg.R, opts=opts)
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    same = [qi for qi, p in enumerate(res["probes"]) if np.array_equal(probes[qi, :len(p)], p)]
    assert len(same) >= len(Q) * 0.9
    sub = {k_: v[same] for k_, v in res.items() if k_ in ("ids", "dist")}
    check_final(ids[same], dist[same], sub, X, Q[same], cfg.metric,
                exact_ids=(cfg.dist == "int255"))


# ---------------------------------------------------------------------------
# Batched form (list-major persistent scan) and hipGraph replay.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(CASES))
def test_batched_candidates_bit_exact(name):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    P = probes_tensor(res, nprobe)
    keys = g.debug_candidates(Q, P, nprobe, cfg.R, opts=ivf.make_opts(form="batched")).cpu().numpy()
    a, ids = ivf.decode_keys(keys)
    assert np.array_equal(ids, res["cand_id"])
    assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32))


@pytest.mark.parametrize("name", list(CASES))
def test_batched_search_identical_to_plain(name):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    ip, dp = g.search(Q, nprobe, cfg.k, cfg.R)
    ib, db = g.search(Q, nprobe, cfg.k, cfg.R, opts=ivf.make_opts(form="batched"))
    assert np.array_equal(ip.cpu().numpy(), ib.cpu().numpy())
    assert np.array_equal(dp.cpu().numpy().view(np.uint32), db.cpu().numpy().view(np.uint32))
    check_final(ib.cpu().numpy(), db.cpu().numpy(), res, X, Q, cfg.metric,
                exact_ids=(cfg.dist == "int255"))


@pytest.mark.parametrize("rounds,depth", [(2, 0), (3, 0), (4, 0), (1, 1), (3, 1), (1, 2),
                                          (2, 8)])
@pytest.mark.parametrize("name", ["c1", "c3s", "c4s", "c5s", "c6u", "c2w"])
def test_batched_rounds_candidates_bit_exact(name, rounds, depth):
    # Rounds over probe ranks [0,4), [4,16), [16,64), ... tighten the
    # threshold between them, and the first-list pass (at least `depth`
    # lists) sets the first one; the pool is still the exact R smallest keys.
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    P = probes_tensor(res, nprobe)
    opts = ivf.make_opts(form="batched", rounds=rounds, first_lists=depth)
    keys = g.debug_candidates(Q, P, nprobe, cfg.R, opts=opts).cpu().numpy()
    a, ids = ivf.decode_keys(keys)
    assert np.array_equal(ids, res["cand_id"])
    assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32))
    ib, db = g.search(Q, nprobe, cfg.k, cfg.R, opts=opts)
    ip, dp = g.search(Q, nprobe, cfg.k, cfg.R)
    assert torch.equal(ib, ip) and torch.equal(db.view(torch.int32), dp.view(torch.int32))
    assert g.device_error() == 0


@pytest.mark.parametrize("query_order,list_order", [(1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("name", ["c1", "c3s", "c5s", "c2w"])
def test_launch_orders_change_no_result(name, query_order, list_order):
    # Longest-first (the default) or index-order launches of the per-query
    # scans and of the batched work items: the same pools and results.
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    P = probes_tensor(res, nprobe)
    ip, dp = g.search(Q, nprobe, cfg.k, cfg.R)
    for form in ("plain", "batched"):
        opts = ivf.make_opts(form=form, query_order=query_order, list_order=list_order)
        keys = g.debug_candidates(Q, P, nprobe, cfg.R, opts=opts).cpu().numpy()
        a, ids = ivf.decode_keys(keys)
        assert np.array_equal(ids, res["cand_id"])
        assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32))
        io, do = g.search(Q, nprobe, cfg.k, cfg.R, opts=opts)
        assert torch.equal(io, ip) and torch.equal(do.view(torch.int32), dp.view(torch.int32))
    assert g.device_error() == 0


@pytest.mark.parametrize("rounds,spill_cap", [(1, 1024), (3, 1024), (3, 2048), (1, 0), (3, 0)])
def test_batched_survivor_overflow_recomputes(rounds, spill_cap):
    # The first probed list is the farthest one and the first-list pass stops
    # after it (one list), so the phase-1 threshold is loose and the near
    # lists' survivors overflow a 1024-key buffer: those queries go through
    # the plain recompute. With the automatic capacity nothing overflows and
    # the merge takes its large-LDS launch.
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, _ = case("c2s")
    nq = 6
    rows = []
    for q in Q[:nq]:
        s = oracle.coarse_scores(q, index["cp"], cfg.metric)
        order = oracle.select_probes(s, cfg.L)
        rows.append(np.concatenate(([order[-1]], order[:20])))
    P = torch.from_numpy(np.stack(rows).astype(np.int32))
    npb = np.full(nq, P.shape[1], dtype=np.int32)
    lens = np.diff(index["list_offsets"])
    assert all(lens[r[1:]].sum() > 1024 for r in rows)
    kp = g.debug_candidates(Q[:nq], P, npb, cfg.R).cpu().numpy()
    kb = g.debug_candidates(Q[:nq], P, npb, cfg.R,
                            opts=ivf.make_opts(form="batched", rounds=rounds,
                                               spill_cap=spill_cap,
                                               first_lists=1)).cpu().numpy()
    assert np.array_equal(kp, kb)
    res = oracle.search(index, X, Q[:nq], 1, cfg.k, cfg.R)  # shape only
    # Pool against the oracle on the same visiting order.
    for qi, r in enumerate(rows):
        all_a, all_i = [], []
        for l in r:
            T = oracle.lut_float(Q[qi], index["cm"][l], index["codebooks"], cfg.metric)
            q8, lo, d, B = oracle.quantize_lut(T, oracle.list_bias(Q[qi], index["cm"][l], cfg.metric))
            ids = index["list_ids"][index["list_offsets"][l]:index["list_offsets"][l + 1]].astype(np.int64)
            all_a.append(oracle.scan_list(q8, d, B, index["codes"][ids])[1])
            all_i.append(ids)
        ca, ci = oracle.top_r(np.concatenate(all_a), np.concatenate(all_i), cfg.R)
        a, ids = ivf.decode_keys(kb[qi])
        assert np.array_equal(ids[:len(ci)], ci)
        assert np.array_equal(a[:len(ca)].view(np.uint32), ca.view(np.uint32))
    del res


@pytest.mark.parametrize("form,rounds", [("plain", 0), ("batched", 1), ("batched", 3)])
def test_graph_replays_match_eager(form, rounds):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case("c3s")
    stream = torch.cuda.Stream()
    Qd = torch.from_numpy(Q).cuda()
    npd = torch.from_numpy(nprobe).cuda()
    eager = ivf.make_opts(form=form, coarse="bf16", widen=4, rounds=rounds)
    graph = ivf.make_opts(form=form, coarse="bf16", widen=4, use_graph=True, rounds=rounds)
    ids = torch.empty((len(Q), cfg.k), dtype=torch.int64, device="cuda")
    dist = torch.empty((len(Q), cfg.k), dtype=torch.float32, device="cuda")
    with torch.cuda.stream(stream):
        ie, de = g.search(Qd, npd, cfg.k, cfg.R, opts=eager)
        ie, de = ie.clone(), de.clone()
        for rep in range(4):
            ids.fill_(-7)
            dist.fill_(0.5)
            g.search(Qd, npd, cfg.k, cfg.R, opts=graph, out=(ids, dist))
            stream.synchronize()
            assert torch.equal(ids, ie), rep
            assert torch.equal(dist.view(torch.int32), de.view(torch.int32)), rep
            # eager work between replays
            g.search(Qd[:5], npd[:5], cfg.k, cfg.R, opts=eager)
            stream.synchronize()


def test_stage_profile_sums_rounds():
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case("c3s")
    Qd = torch.from_numpy(Q).cuda()
    npd = torch.from_numpy(nprobe).cuda()
    g.profile(True)
    try:
        g.profile_read()
        for form, rounds in (("plain", 0), ("batched", 1), ("batched", 3)):
            opts = ivf.make_opts(form=form, rounds=rounds)
            for _ in range(3):
                g.search(Qd, npd, cfg.k, cfg.R, opts=opts)
            g.debug_candidates(Q, probes_tensor(res, nprobe), nprobe, cfg.R, opts=opts)
            ms, cnt = g.profile_read()
            assert cnt == 3, (form, rounds, cnt)
            for st in ("coarse", "select", "prep", "scan", "rerank"):
                assert ms[st] > 0.0, (form, rounds, st)
            assert (ms["merge"] > 0.0) == (form == "batched")
    finally:
        g.profile(False)


# ---------------------------------------------------------------------------
# Adaptive probing depth and re-rank size (section 4.2, Eq. 2).
# ---------------------------------------------------------------------------

ADAPT = dict(nprobe_init=3, nprobe_min=2, reorder_min=1, p0=0.3, p1=0.5)


@pytest.mark.parametrize("name", list(CASES))
def test_adaptive_choice_and_search(name):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    ad = dict(ADAPT, reorder_min=max(cfg.k, cfg.R // 4))
    # Per-query choice: integers decided in FP32 from canonical scores.
    n_used, r_used = g.debug_adaptive(Q, nprobe, cfg.k, cfg.R, opts=ivf.make_opts(adaptive=ad))
    n_used, r_used = n_used.cpu().numpy(), r_used.cpu().numpy()
    want_n, want_r = [], []
    for qi in range(len(Q)):
        s = oracle.coarse_scores(np.asarray(Q[qi], np.float32), index["cp"], cfg.metric)
        npq, reo, _ = oracle.adaptive_params(s, int(nprobe[qi]), cfg.metric, ad["nprobe_init"],
                                             ad["nprobe_min"], ad["reorder_min"], cfg.R, cfg.k,
                                             ad["p0"], ad["p1"])
        want_n.append(npq)
        want_r.append(reo)
    assert np.array_equal(n_used, want_n) and np.array_equal(r_used, want_r)
    # Probe export: the chosen count, then -1.
    P = g.debug_probes(Q, nprobe, opts=ivf.make_opts(adaptive=ad)).cpu().numpy()
    for qi in range(len(Q)):
        assert (P[qi, want_n[qi]:] == -1).all()
    # Search: plain and batched identical; the oracle's adaptive search.
    ip, dp = g.search(Q, nprobe, cfg.k, cfg.R, opts=ivf.make_opts(form="plain", adaptive=ad))
    ib, db = g.search(Q, nprobe, cfg.k, cfg.R, opts=ivf.make_opts(form="batched", adaptive=ad))
    assert torch.equal(ip, ib) and torch.equal(dp.view(torch.int32), db.view(torch.int32))
    ores = oracle.search(index, X, Q, nprobe, cfg.k, cfg.R, adaptive=ad)
    assert np.array_equal(ores["nprobe_used"], want_n)
    check_final(ib.cpu().numpy(), db.cpu().numpy(), ores, X, Q, cfg.metric,
                exact_ids=(cfg.dist == "int255"))
    assert g.device_error() == 0


def test_adaptive_limits_and_rejections():
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case("c3s")
    # p0 above every hardness: the minima; the pools are the static ones at
    # nprobe_min and the re-rank uses reorder_min of them.
    ad = dict(ADAPT, p0=2.0, reorder_min=cfg.k)
    n_used, r_used = g.debug_adaptive(Q, nprobe, cfg.k, cfg.R, opts=ivf.make_opts(adaptive=ad))
    assert (n_used.cpu() == ADAPT["nprobe_min"]).all() and (r_used.cpu() == cfg.k).all()
    ia, da = g.search(Q, nprobe, cfg.k, cfg.R, opts=ivf.make_opts(adaptive=ad))
    ores = oracle.search(index, X, Q, np.full(len(Q), ADAPT["nprobe_min"]), cfg.k, cfg.R)
    for qi in range(len(Q)):
        ids, _ = oracle.rerank(Q[qi], X, ores["cand_id"][qi][:cfg.k], cfg.k, cfg.metric)
        assert set(ia[qi].cpu().numpy().tolist()) == set(ids.tolist())
    # Caller-given probes have no coarse scores: rejected.
    with pytest.raises(ivf.IvfError):
        g.search_with_probes(Q, probes_tensor(res, nprobe), nprobe, cfg.k, cfg.R,
                             opts=ivf.make_opts(adaptive=ad))


# ---------------------------------------------------------------------------
# Component filtration (section 4.3): the index over the kept columns.
# ---------------------------------------------------------------------------

def _filtered_case():
    if "c6s" not in _STATE:
        ivf = _gpu()
        from workloads import make_workload, scaled, train_index
        cfg = scaled("c6", 20_000, 30, L=32, ncomp=32, nprobe=(6, 6))
        X, Q, nprobe = make_workload(cfg)
        keep, _ = oracle.component_filter(X, 0.9)
        index = train_index(X, cfg, dims=keep)
        print(f"[case c6s] n={cfg.n} d_base={cfg.d} kept={len(keep)} m={index['codebooks'].shape[0]}",
              flush=True)
        g = ivf.GpuIndex.from_index(index, X)
        res = oracle_stages(index, X, Q, nprobe, cfg.k, cfg.R)
        _STATE["c6s"] = (cfg, X, Q, nprobe, index, g, res)
    return _STATE["c6s"]


def test_filtered_index_parity():
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = _filtered_case()
    assert g.d == len(index["dims"]) < g.d_base == X.shape[1]
    # Steps 1-4 on the kept components: probes, tables and pools bit-exact.
    P = g.debug_probes(Q, nprobe).cpu().numpy()
    for qi, p in enumerate(res["probes"]):
        assert np.array_equal(P[qi, :len(p)], p), qi
    Pt = probes_tensor(res, nprobe)
    lut, lo, delta, B = g.debug_luts(Q, Pt, nprobe)
    qi, p = 3, 2
    q8, lo_o, d_o, B_o = res["luts"][(qi, int(res["probes"][qi][p]))]
    assert np.array_equal(lut[qi, p].cpu().numpy(), q8)
    assert np.float32(delta[qi, p].item()) == d_o and np.float32(B[qi, p].item()) == B_o
    for form in ("plain", "batched"):
        keys = g.debug_candidates(Q, Pt, nprobe, cfg.R, opts=ivf.make_opts(form=form)).cpu().numpy()
        a, ids = ivf.decode_keys(keys)
        assert np.array_equal(ids, res["cand_id"]), form
        assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32)), form
    # The re-rank against the full rows and queries (Alg. 2).
    for form, coarse in (("plain", "exact"), ("batched", "bf16")):
        ids, dist = g.search(Q, nprobe, cfg.k, cfg.R, opts=ivf.make_opts(form=form, coarse=coarse))
        check_final(ids.cpu().numpy(), dist.cpu().numpy(), res, X, Q, cfg.metric, exact_ids=True)
    assert g.device_error() == 0


# ---------------------------------------------------------------------------
# Index construction on the GPU (Alg. 1): assignment and encoding.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["c1", "c2s", "c3s", "c5s"])
def test_gpu_assign_and_encode_bit_exact(name):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    rows = X[:3000]
    Xd = torch.from_numpy(np.ascontiguousarray(rows)).cuda()
    cpd = torch.from_numpy(index["cp"]).cuda()
    want = oracle.assign_lists(rows, index["cp"], cfg.metric)
    got = ivf.assign_lists(cpd, Xd, cfg.metric, coarse="exact", chunk=1000).cpu().numpy()
    assert np.array_equal(got, want)
    # MFMA pre-selection widened to every list is exact; widened by 4 it is
    # a valid choice and almost always the canonical one.
    got = ivf.assign_lists(cpd, Xd, cfg.metric, coarse="bf16", widen=cfg.L, chunk=777).cpu().numpy()
    assert np.array_equal(got, want)
    got = ivf.assign_lists(cpd, Xd, cfg.metric, coarse="bf16", widen=4).cpu().numpy()
    assert (got != want).mean() <= 0.01
    lists = want.astype(np.int32)
    codes = ivf.encode_codes(Xd, torch.from_numpy(index["cm"]).cuda(),
                             torch.from_numpy(lists).cuda(),
                             torch.from_numpy(index["codebooks"]).cuda()).cpu().numpy()
    assert np.array_equal(codes, oracle.encode(rows, index["cm"], lists, index["codebooks"]))


def test_gpu_trained_index_searches_well():
    import paper_2511_03298_amd as ivf
    from paper_2511_03298_amd.train import train_index_gpu
    from workloads import exact_knn, recall_at_k
    cfg, X, Q, nprobe, index, _, _ = case("c3s")
    tr = train_index_gpu(X, cfg.L, cfg.m, cfg.metric, seed=1)
    lens = np.diff(tr["list_offsets"])
    assert lens.sum() == len(X) and lens.min() >= 0
    ids_sorted = np.sort(tr["list_ids"].cpu().numpy())
    assert np.array_equal(ids_sorted, np.arange(len(X)))
    g = ivf.GpuIndex.from_index(tr, X)
    ids, _ = g.search(Q, 16, cfg.k, cfg.R)
    gt, _ = exact_knn(X, Q, cfg.k, cfg.metric)
    assert recall_at_k(ids.cpu().numpy(), gt, cfg.k) >= 0.8


def test_autotuner_picks_measured_schedule_and_caches(tmp_path):
    import paper_2511_03298_amd as ivf
    from paper_2511_03298_amd.tune import autotune
    cfg, X, Q, nprobe, index, g, res = case("c2s")
    space = [dict(form="plain", coarse="exact", widen=2, pool_cap=0),
             dict(form="batched", coarse="exact", widen=2, grid=2),
             dict(form="batched", coarse="bf16", widen=4, grid=0, rounds=3)]
    path = str(tmp_path / "tune.json")
    opts, rep = autotune(g, Q, nprobe, cfg.k, cfg.R, space=space, reps=2, cache_path=path)
    assert not rep["cached"] and len(rep["trials"]) >= 2
    assert rep["best_ms"] == min(t["ms"] for t in rep["trials"])
    opts2, rep2 = autotune(g, Q, nprobe, cfg.k, cfg.R, space=space, cache_path=path)
    assert rep2["cached"] and ivf.opts_dict(opts2) == ivf.opts_dict(opts)
    # The tuned schedule gives the same results as the plain exact one.
    a = g.search(Q, nprobe, cfg.k, cfg.R)
    b = g.search(Q, nprobe, cfg.k, cfg.R, opts=opts)
    if ivf.opts_dict(opts)["coarse"] == "exact":
        assert torch.equal(a[0], b[0])


# ---------------------------------------------------------------------------
# Spilled assignment (section 4.6.2, SOAR): two copies per point, the pool
# keeps each point once at its best copy.
# ---------------------------------------------------------------------------

SPILL_BASE = {"c2x": "c2s", "c3x": "c3s"}


def _spilled_case(name):
    if name not in _STATE:
        ivf = _gpu()
        from workloads import spill_index
        cfg, X, Q, nprobe, index, _, _ = case(SPILL_BASE[name])
        sp = spill_index(X, index, 1.0)
        print(f"[case {name}] spilled {SPILL_BASE[name]}: entries={len(sp['list_ids'])} "
              f"n={len(X)} R={cfg.R} pool={2 * cfg.R}", flush=True)
        g = ivf.GpuIndex.from_index(sp, X, base_dtype=cfg.base_dtype)
        res = oracle_stages(sp, X, Q, nprobe, cfg.k, cfg.R)
        _STATE[name] = (cfg, X, Q, nprobe, sp, g, res)
    return _STATE[name]


@pytest.mark.parametrize("name", list(SPILL_BASE))
def test_spilled_tables(name):
    cfg, X, Q, nprobe, sp, g, res = _spilled_case(name)
    lay = g.layout()
    tables = g.tables.cpu().numpy()
    codes, slot, pad = unpack_tables(tables, lay, cfg.m)
    boff = tables[lay.block_offsets:lay.block_offsets + (cfg.L + 1) * 4].view(np.int32)
    off, lid = sp["list_offsets"], sp["list_ids"]
    seen = {}
    for l in range(cfg.L):
        n_l = off[l + 1] - off[l]
        s0 = boff[l] * 64
        v = slot[s0:s0 + n_l]
        assert np.array_equal(v // 2, lid[off[l]:off[l + 1]])
        assert np.array_equal(codes[s0:s0 + n_l], sp["codes"][off[l]:off[l + 1]])
        for sl, val in zip(range(s0, s0 + n_l), v.tolist()):
            seen.setdefault(val // 2, []).append((sl, val % 2))
    # Each point: two slots numbered 0 then 1 in slot order.
    assert len(seen) == len(X)
    for i, ent in seen.items():
        assert [c for _, c in sorted(ent)] == [0, 1], i


@pytest.mark.parametrize("form,rounds", [("plain", 0), ("batched", 1), ("batched", 3)])
@pytest.mark.parametrize("name", list(SPILL_BASE))
def test_spilled_candidates_bit_exact(name, form, rounds):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, sp, g, res = _spilled_case(name)
    P = probes_tensor(res, nprobe)
    keys = g.debug_candidates(Q, P, nprobe, cfg.R,
                              opts=ivf.make_opts(form=form, rounds=rounds)).cpu().numpy()
    a, ids = ivf.decode_keys(keys)
    assert np.array_equal(ids, res["cand_id"])
    assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32))
    for row in ids:
        v = row[row >= 0]
        assert len(np.unique(v)) == len(v)
    assert g.device_error() == 0


@pytest.mark.parametrize("name", list(SPILL_BASE))
def test_spilled_search(name):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, sp, g, res = _spilled_case(name)
    ip, dp = g.search(Q, nprobe, cfg.k, cfg.R)
    check_final(ip.cpu().numpy(), dp.cpu().numpy(), res, X, Q, cfg.metric,
                exact_ids=(cfg.dist == "int255"))
    for opts in (ivf.make_opts(form="batched"), ivf.make_opts(form="batched", rounds=3),
                 ivf.make_opts(form="plain", pool_cap=256)):
        ib, db = g.search(Q, nprobe, cfg.k, cfg.R, opts=opts)
        assert torch.equal(ib, ip) and torch.equal(db.view(torch.int32), dp.view(torch.int32))
    # Adaptive re-rank size on the de-duplicated pool.
    ad = dict(nprobe_init=4, nprobe_min=2, reorder_min=cfg.R // 2, p0=0.3, p1=0.5)
    ra = oracle.search(sp, X, Q, nprobe, cfg.k, cfg.R, adaptive=ad)
    ia, da = g.search(Q, nprobe, cfg.k, cfg.R,
                      opts=ivf.make_opts(form="batched", coarse="exact", adaptive=ad))
    check_final(ia.cpu().numpy(), da.cpu().numpy(), ra, X, Q, cfg.metric,
                exact_ids=(cfg.dist == "int255"))
    assert g.device_error() == 0


def test_spilled_survivor_overflow_recomputes():
    # Far list first and a first-list pass of one list: a loose first
    # threshold, survivors overflow a 1024-key buffer and those queries are
    # recomputed; pools equal the plain form's and the oracle's best-copy
    # pool over the same lists.
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, sp, g, _ = _spilled_case("c2x")
    nq = 6
    rows = []
    for q in Q[:nq]:
        s = oracle.coarse_scores(q, sp["cp"], cfg.metric)
        order = oracle.select_probes(s, cfg.L)
        rows.append(np.concatenate(([order[-1]], order[:20])))
    P = torch.from_numpy(np.stack(rows).astype(np.int32))
    npb = np.full(nq, P.shape[1], dtype=np.int32)
    kp = g.debug_candidates(Q[:nq], P, npb, cfg.R).cpu().numpy()
    for rounds in (1, 3):
        kb = g.debug_candidates(Q[:nq], P, npb, cfg.R,
                                opts=ivf.make_opts(form="batched", rounds=rounds,
                                                   spill_cap=1024,
                                                   first_lists=1)).cpu().numpy()
        assert np.array_equal(kp, kb), rounds
    off, lid = sp["list_offsets"], sp["list_ids"]
    for qi, r in enumerate(rows):
        all_a, all_i = [], []
        for l in r:
            T = oracle.lut_float(Q[qi], sp["cm"][l], sp["codebooks"], cfg.metric)
            q8, lo, d, B = oracle.quantize_lut(T, oracle.list_bias(Q[qi], sp["cm"][l], cfg.metric))
            all_a.append(oracle.scan_list(q8, d, B, sp["codes"][off[l]:off[l + 1]])[1])
            all_i.append(lid[off[l]:off[l + 1]].astype(np.int64))
        ca, ci = oracle.top_r_unique(np.concatenate(all_a), np.concatenate(all_i), cfg.R)
        a, ids = ivf.decode_keys(kp[qi])
        assert np.array_equal(ids[:len(ci)], ci)
        assert np.array_equal(a[:len(ca)].view(np.uint32), ca.view(np.uint32))


def test_spilled_index_rejections():
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, sp, g, _ = _spilled_case("c2x")
    # rerank * copies above 2048.
    with pytest.raises(ivf.IvfError):
        g.search(Q[:2], 4, 10, 1500)
    # A point in three lists with copies = 2, and an id outside [0, n).
    off, lid = sp["list_offsets"], sp["list_ids"].copy()
    for bad_id, what in ((int(lid[off[1]]), "three lists"), (len(X), "out of range")):
        l = 0
        ids0 = lid[off[l]:off[l + 1]]
        if bad_id in ids0.tolist():
            l = 2
            ids0 = lid[off[l]:off[l + 1]]
        new0 = np.sort(np.concatenate([ids0, [bad_id]])).astype(np.int32)
        pos = int(np.searchsorted(new0, bad_id))
        lid2 = np.concatenate([lid[:off[l]], new0, lid[off[l + 1]:]])
        codes2 = np.insert(sp["codes"], off[l] + pos, sp["codes"][off[l]], axis=0)
        off2 = off.copy()
        off2[l + 1:] += 1
        with pytest.raises(ivf.IvfError):
            ivf.GpuIndex(X, sp["cm"], sp["codebooks"], codes2, off2, lid2, cfg.metric,
                         probe_centroids=sp["cp"], copies=2)


@pytest.mark.parametrize("name", ["c2s", "c3s"])
def test_gpu_spill_assignment(name):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g, res = case(name)
    rows = X[:3000]
    prim = np.empty(len(X), np.int64)
    prim[index["list_ids"]] = np.repeat(np.arange(cfg.L), np.diff(index["list_offsets"]))
    prim = prim[:3000]
    Xd = torch.from_numpy(np.ascontiguousarray(rows)).cuda()
    cmd = torch.from_numpy(index["cm"]).cuda()
    pd = torch.from_numpy(prim.astype(np.int32)).cuda()
    C64 = index["cm"].astype(np.float64)
    for lam in (0.0, 1.0, 2.5):
        want = oracle.spill_assign(rows, index["cm"], prim, lam)
        got = ivf.assign_spill(cmd, Xd, pd, lam, chunk=1111).cpu().numpy()
        assert (got != prim).all()
        assert (got == want).mean() >= 0.99, lam
        for i in np.nonzero(got != want)[0]:
            x = rows[i].astype(np.float64)
            r = x - C64[prim[i]]

            def loss(l):
                dv = x - C64[l]
                return dv @ dv + lam * (dv @ r) ** 2 / (r @ r)
            assert loss(got[i]) <= loss(want[i]) * (1 + 1e-5) + 1e-6, (lam, i)
    bad = pd.clone()
    bad[5] = cfg.L
    bad[9] = -3
    got = ivf.assign_spill(cmd, Xd, bad, 1.0).cpu().numpy()
    assert got[5] == -1 and got[9] == -1 and (got[:5] >= 0).all()


def test_gpu_trained_spilled_index():
    import paper_2511_03298_amd as ivf
    from paper_2511_03298_amd.train import train_index_gpu
    from workloads import exact_knn, recall_at_k
    cfg, X, Q, nprobe, index, _, _ = case("c3s")
    tr = train_index_gpu(X, cfg.L, cfg.m, cfg.metric, seed=1)
    sp = train_index_gpu(X, cfg.L, cfg.m, cfg.metric, seed=1, soar=1.0)
    assert sp["copies"] == 2 and len(sp["list_ids"]) == 2 * len(X)
    lid = sp["list_ids"].cpu().numpy()
    assert np.array_equal(np.bincount(lid, minlength=len(X)), np.full(len(X), 2))
    assert (sp["spill"] != sp["assign"]).all()
    gt, _ = exact_knn(X, Q, cfg.k, cfg.metric)
    g1 = ivf.GpuIndex.from_index(tr, X)
    g2 = ivf.GpuIndex.from_index(sp, X)
    r1 = recall_at_k(g1.search(Q, 4, cfg.k, cfg.R)[0].cpu().numpy(), gt, cfg.k)
    r2 = recall_at_k(g2.search(Q, 4, cfg.k, cfg.R)[0].cpu().numpy(), gt, cfg.k)
    print(f"[spilled] recall@{cfg.k} nprobe 4: one copy {r1:.3f}, two copies {r2:.3f}", flush=True)
    assert r2 >= r1 - 0.02
    # The GPU-trained spilled index against the oracle on a few queries.
    spn = dict(sp, codes=sp["codes"].cpu().numpy(), list_ids=lid)
    res = oracle_stages(spn, X, Q[:8], 6, cfg.k, cfg.R)
    keys = g2.debug_candidates(Q[:8], probes_tensor(res, np.full(8, 6)), np.full(8, 6, np.int32),
                               cfg.R).cpu().numpy()
    a, ids = ivf.decode_keys(keys)
    assert np.array_equal(ids, res["cand_id"])
    assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32))


# ---------------------------------------------------------------------------
# Probe selection on long score rows (L > 2048: keys held in registers,
# 4-bit radix passes, ties by list order).
# ---------------------------------------------------------------------------

def _long_row_index(ivf, L, d, metric, seed, groups=None):
    """An index with one point per list (only the centroids matter here).
    groups: the centroids are drawn from L / groups distinct rows, so scores
    tie exactly."""
    rng = np.random.default_rng(seed)
    if groups:
        base = rng.standard_normal((L // groups + 1, d)).astype(np.float32)
        C = base[rng.integers(0, len(base), size=L)]
    else:
        C = rng.standard_normal((L, d)).astype(np.float32)
    if metric == "ip":
        C = (C / np.linalg.norm(C, axis=1, keepdims=True)).astype(np.float32)
    m = 4
    cb = rng.standard_normal((m, 16, d // m)).astype(np.float32)
    codes = rng.integers(0, 16, size=(L, m)).astype(np.uint8)
    g = ivf.GpuIndex(C.copy(), C, cb, codes, np.arange(L + 1), np.arange(L, dtype=np.int32),
                     metric, probe_centroids=C)
    return g, C


@pytest.mark.parametrize("L,metric,groups", [(1024, "l2", 7), (1500, "l2", None),
                                             (2048, "ip", 16), (3000, "l2", None),
                                             (3000, "l2", 7), (9000, "ip", None),
                                             (4100, "ip", 16), (16384, "l2", None)])
def test_long_row_selection_bit_exact(L, metric, groups):
    import paper_2511_03298_amd as ivf
    _gpu()
    d = 16
    g, C = _long_row_index(ivf, L, d, metric, seed=L + (groups or 0), groups=groups)
    rng = np.random.default_rng(5)
    nq = 24
    Q = rng.standard_normal((nq, d)).astype(np.float32)
    if groups:
        Q[:4] = C[[0, 1, 2, 3]]  # queries on a repeated centroid: ties at the top
    nprobe = rng.choice([1, 2, 7, 64, 300, 1000], size=nq).astype(np.int32)
    print(f"[long rows] L={L} metric={metric} groups={groups} nprobe={sorted(set(nprobe.tolist()))}",
          flush=True)
    want = []
    for qi in range(nq):
        s = oracle.coarse_scores(Q[qi], C, metric)
        want.append(oracle.select_probes(s, int(nprobe[qi])))
    got = g.debug_probes(Q, nprobe).cpu().numpy()
    for qi, p in enumerate(want):
        assert np.array_equal(got[qi, :len(p)], p), qi
        assert np.all(got[qi, len(p):] == -1)
    # MFMA pre-selection widened to every list, then the canonical re-score.
    if L <= 8192:
        got = g.debug_probes(Q, nprobe, opts=ivf.make_opts(coarse="bf16", widen=L)).cpu().numpy()
        for qi, p in enumerate(want):
            assert np.array_equal(got[qi, :len(p)], p), qi
    # Adaptive counts read the sorted canonical scores of the long row.
    ad = dict(nprobe_init=8, nprobe_min=1, reorder_min=50, p0=0.2, p1=0.5)
    used, reo = g.debug_adaptive(Q, np.full(nq, 64, np.int32), 10, 100,
                                 opts=ivf.make_opts(adaptive=ad))
    for qi in range(nq):
        s = oracle.coarse_scores(Q[qi], C, metric)
        npq, rq, _ = oracle.adaptive_params(s, 64, metric, 8, 1, 50, 100, 10, 0.2, 0.5)
        assert int(used[qi]) == npq and int(reo[qi]) == rq, qi


def test_largest_m_plain_form():
    # m = 256 subspaces (d' = 1), the largest the tables allow: 32 code words
    # per point. The plain form matches the oracle bit for bit; the batched
    # form (tables for up to 192 subspaces) refuses it.
    import paper_2511_03298_amd as ivf
    _gpu()
    cfg, X, Q, nprobe, index = cached_workload("c6", 6000, 10, L=16, ncomp=16, m=256,
                                               nprobe=(4, 4))
    assert index["codebooks"].shape[0] == 256
    print(f"[m=256] n={len(X)} d={X.shape[1]} L={cfg.L}", flush=True)
    g = ivf.GpuIndex.from_index(index, X, base_dtype=cfg.base_dtype)
    res = oracle_stages(index, X, Q, nprobe, cfg.k, cfg.R)
    P = probes_tensor(res, nprobe)
    lut, lo, delta, B = [t.cpu().numpy() for t in g.debug_luts(Q, P, nprobe)]
    for qi, p in enumerate(res["probes"]):
        for pi, l in enumerate(p):
            q8, lo_o, d_o, B_o = res["luts"][(qi, int(l))]
            assert np.array_equal(lut[qi, pi], q8)
            assert B[qi, pi].view(np.uint32) == np.float32(B_o).view(np.uint32)
    keys = g.debug_candidates(Q, P, nprobe, cfg.R).cpu().numpy()
    a, ids = ivf.decode_keys(keys)
    assert np.array_equal(ids, res["cand_id"])
    assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32))
    ids, dist = g.search(Q, nprobe, cfg.k, cfg.R)
    check_final(ids.cpu().numpy(), dist.cpu().numpy(), res, X, Q, cfg.metric, exact_ids=True)
    with pytest.raises(ivf.IvfError):
        g.search(Q, nprobe, cfg.k, cfg.R, opts=ivf.make_opts(form="batched"))


def test_gpu_pq_kmeans():
    # PQ codebook k-means with the encoding kernel as its assignment step:
    # each iteration's codes are the oracle's nearest codewords, and the
    # quantisation error does not grow with more iterations.
    from paper_2511_03298_amd.train import _pq_kmeans_gpu
    cfg, X, Q, nprobe, index, g, res = case("c2s")
    off = index["list_offsets"]
    lists = np.repeat(np.arange(cfg.L), np.diff(off))
    rows = index["list_ids"].astype(np.int64)
    resid = (X[rows] - index["cm"][lists]).astype(np.float32)[:8000]
    errs = []
    for iters in (1, 4, 10):
        cb = _pq_kmeans_gpu(resid, cfg.m, iters, np.random.default_rng(3), "cuda")
        codes = oracle.encode(resid, np.zeros((1, resid.shape[1]), np.float32),
                              np.zeros(len(resid), np.int64), cb)
        rec = np.concatenate([cb[j][codes[:, j]] for j in range(cfg.m)], axis=1)
        errs.append(float(((resid.astype(np.float64) - rec) ** 2).sum(axis=1).mean()))
    print(f"[pq k-means] mean squared error after 1/4/10 iterations: {errs}", flush=True)
    assert errs[1] <= errs[0] * (1 + 1e-6) and errs[2] <= errs[1] * (1 + 1e-6)


def test_filtered_and_spilled_index_from_the_gpu_trainer():
    # Component filtration and spilled assignment together, both built by the
    # GPU trainer: pools bit-exact against the oracle on the same index, the
    # re-rank on the full rows.
    import paper_2511_03298_amd as ivf
    from paper_2511_03298_amd.train import train_index_gpu
    _gpu()
    from workloads import make_workload, scaled
    cfg = scaled("c6", 12_000, 16, L=24, ncomp=24, nprobe=(4, 4))
    X, Q, nprobe = make_workload(cfg)
    keep, _ = oracle.component_filter(X, 0.9)
    tr = train_index_gpu(X, cfg.L, cfg.m, cfg.metric, seed=2, dims=keep, soar=1.0)
    assert tr["copies"] == 2 and len(tr["dims"]) == len(keep) < X.shape[1]
    idx = dict(tr, codes=tr["codes"].cpu().numpy(), list_ids=tr["list_ids"].cpu().numpy())
    print(f"[filtered+spilled] kept {len(keep)} of {X.shape[1]} dims, "
          f"{len(idx['list_ids'])} entries for {len(X)} rows", flush=True)
    g = ivf.GpuIndex.from_index(idx, X, base_dtype=cfg.base_dtype)
    res = oracle_stages(idx, X, Q, nprobe, cfg.k, cfg.R)
    P = probes_tensor(res, nprobe)
    for form in ("plain", "batched"):
        keys = g.debug_candidates(Q, P, nprobe, cfg.R, opts=ivf.make_opts(form=form)).cpu().numpy()
        a, ids = ivf.decode_keys(keys)
        assert np.array_equal(ids, res["cand_id"]), form
        assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32)), form
    ids, dist = g.search(Q, nprobe, cfg.k, cfg.R, opts=ivf.make_opts(form="batched"))
    check_final(ids.cpu().numpy(), dist.cpu().numpy(), res, X, Q, cfg.metric, exact_ids=True)
    assert g.device_error() == 0


@pytest.mark.parametrize("max_np", [1030, 600])
def test_ip_list_constants_long_probe_rows(max_np):
    # Inner product: with probe rows of at most 1024 slots the scan kernel
    # computes the list constants -<q, cm_l> itself, with longer rows a
    # separate kernel does; both give the oracle's pools bit-exactly.
    import paper_2511_03298_amd as ivf
    _gpu()
    L, k, R = 1100, 5, 64
    cfg, X, Q, nprobe, index = cached_workload("c3", 8000, 6, L=L, ncomp=300, d=20, m=10,
                                               nprobe=(max_np, max_np), k=k, R=R)
    print(f"[long probe rows] {cfg.metric} L={cfg.L} nprobe={nprobe.tolist()}", flush=True)
    assert cfg.metric == "ip" and int(max(nprobe)) == max_np
    g = ivf.GpuIndex.from_index(index, X)
    res = oracle_stages(index, X, Q, nprobe, k, R)
    P = probes_tensor(res, nprobe)
    for opts in (ivf.make_opts(), ivf.make_opts(form="batched")):
        keys = g.debug_candidates(Q, P, nprobe, R, opts=opts).cpu().numpy()
        a, ids = ivf.decode_keys(keys)
        assert np.array_equal(ids, res["cand_id"]), ivf.opts_dict(opts)
        assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32))
        ids, dist = g.search(Q, nprobe, k, R, opts=opts)
        check_final(ids.cpu().numpy(), dist.cpu().numpy(), res, X, Q, cfg.metric)
    assert g.device_error() == 0


@pytest.mark.parametrize("seed", range(8))
def test_fuzz_shapes(seed):
    # Random shapes inside the supported range: d not a multiple of 16, any
    # divisor m, L not a multiple of the tiles, per-query nprobe in [1, L],
    # R in [k, n]. Probe sets and pools bit-exact in both forms; re-rank
    # within the tolerance.
    import paper_2511_03298_amd as ivf
    _gpu()
    rng = np.random.default_rng(1000 + seed)
    name = ("c1", "c3")[seed % 2]
    d = int(rng.choice([12, 20, 36, 60, 100]))
    m = int(rng.choice([v for v in range(1, min(d, 128) + 1) if d % v == 0]))
    L = int(rng.integers(5, 150))
    n = int(rng.integers(2000, 6000))
    k = int(rng.integers(1, 20))
    R = int(rng.integers(k, min(n, 1024) + 1))
    cfg, X, Q, nprobe, index = cached_workload(name, n, 12, L=L, ncomp=max(4, L // 2), d=d, m=m,
                                               nprobe=(1, L), k=k, R=R)
    print(f"[fuzz {seed}] {cfg.metric} n={n} d={d} m={m} L={L} k={k} R={R} "
          f"nprobe={nprobe.tolist()}", flush=True)
    g = ivf.GpuIndex.from_index(index, X)
    res = oracle_stages(index, X, Q, nprobe, k, R)
    got = g.debug_probes(Q, nprobe).cpu().numpy()
    for qi, p in enumerate(res["probes"]):
        assert np.array_equal(got[qi, :len(p)], p), qi
    P = probes_tensor(res, nprobe)
    for opts in (ivf.make_opts(), ivf.make_opts(form="batched"),
                 ivf.make_opts(form="batched", rounds=3)):
        keys = g.debug_candidates(Q, P, nprobe, R, opts=opts).cpu().numpy()
        a, ids = ivf.decode_keys(keys)
        assert np.array_equal(ids, res["cand_id"]), ivf.opts_dict(opts)
        assert np.array_equal(a.view(np.uint32), res["cand_a"].view(np.uint32))
    ids, dist = g.search(Q, nprobe, k, R, opts=ivf.make_opts(form="batched"))
    check_final(ids.cpu().numpy(), dist.cpu().numpy(), res, X, Q, cfg.metric)
    assert g.device_error() == 0
