"""Autotuner for the search schedule.

For one index and one query-batch shape it measures a set of schedules on the
device and keeps the fastest admissible one:
  * form: plain (one workgroup per query) or batched (persistent list-major);
  * coarse precision: exact FP32, or FP32/BF16/FP8 MFMA pre-selection with
    widening x1, x2 or x4 or an additive margin of 16-64 lists -- admitted
    only when its probe sets agree with the exact ones on at least
    `min_agree` of the queries (results are otherwise bit-identical, the
    forms only change the schedule);
  * plain candidate-buffer size (pool_cap), batched persistent grid size,
    number of threshold-tightening rounds and lists of the first-list pass
    (first_lists);
  * for the fastest of those, the launch orders: longest-first or index
    order of the per-query scans (query_order) and of the batched work items
    (list_order);
  * then the fastest schedule captured into a hipGraph and replayed on a
    side stream (use_graph), kept when faster.
Results are cached in a JSON file keyed by the device architecture and the
shape (n, d, L, m, metric, nq, max_nprobe, k, rerank).
"""

from __future__ import annotations

import json
import os
import time
from typing import Optional

from . import COARSE, GpuIndex, make_opts, opts_dict

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ivfpq", "tune.json")


def shape_key(g: GpuIndex, nq: int, max_nprobe: int, k: int, rerank: int) -> str:
    import torch
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    return f"{arch}|n{g.n}|d{g.d}|L{g.L}|m{g.m}|{g.metric}|nq{nq}|p{max_nprobe}|k{k}|R{rerank}"


COARSE_SPACE = (("exact", 2, 0), ("bf16", 1, 0), ("bf16", 1, 16), ("bf16", 1, 32),
                ("bf16", 1, 64), ("bf16", 2, 0), ("bf16", 4, 0), ("fp8", 1, 64), ("fp8", 4, 0),
                ("f32", 2, 0))


def default_space():
    space = []
    for coarse, widen, add in COARSE_SPACE:
        c = dict(coarse=coarse, widen=widen, widen_add=add)
        for pool in (0, 2048, 4096):
            space.append(dict(c, form="plain", pool_cap=pool))
        for rounds in (1, 2, 3):
            for depth in (1, 2, 4, 8):
                for grid, pool in ((0, 0), (4, 0)):
                    space.append(dict(c, form="batched", grid=grid, pool_cap=pool, rounds=rounds,
                                      first_lists=depth))
    return space


def _time(g, Qd, npd, k, rerank, max_nprobe, opts, ids, dist, reps, stream=None):
    """Milliseconds per search; graph-captured schedules run on `stream`."""
    import torch
    stream = stream or torch.cuda.current_stream()
    with torch.cuda.stream(stream):
        g.search(Qd, npd, k, rerank, max_nprobe=max_nprobe, opts=opts, out=(ids, dist))
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(reps):
            g.search(Qd, npd, k, rerank, max_nprobe=max_nprobe, opts=opts, out=(ids, dist))
        stop.record(stream)
        torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps


def autotune(g: GpuIndex, queries, nprobe, k: int, rerank: int,
             max_nprobe: Optional[int] = None, space=None, reps: int = 3,
             min_agree: float = 0.995, cache_path: Optional[str] = DEFAULT_CACHE,
             refresh: bool = False, log=None):
    """Return (opts, report) for the fastest admissible schedule."""
    import torch
    Qd = g._queries(queries)
    nq = Qd.shape[0]
    npd = g._nprobe(nprobe, nq)
    if max_nprobe is None:
        max_nprobe = max(1, min(int(npd.max().item()), g.L))
    key = shape_key(g, nq, max_nprobe, k, rerank)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if not refresh and key in cache:
        best = cache[key]["best"]
        return make_opts(**best), dict(cache[key], cached=True)

    exact = g.debug_probes(Qd, npd, max_nprobe=max_nprobe).cpu()
    agree = {}
    ids = torch.empty((nq, k), dtype=torch.int64, device=g.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=g.device)
    trials = []
    t0 = time.time()
    for cand in space or default_space():
        ck = (cand["coarse"], cand["widen"], cand.get("widen_add", 0))
        if ck not in agree:
            if cand["coarse"] == "exact":
                agree[ck] = 1.0
            else:
                o = make_opts(coarse=cand["coarse"], widen=cand["widen"],
                              widen_add=cand.get("widen_add", 0))
                p = g.debug_probes(Qd, npd, max_nprobe=max_nprobe, opts=o).cpu()
                agree[ck] = float((p == exact).all(dim=1).float().mean())
        if agree[ck] < min_agree:
            continue
        opts = make_opts(**cand)
        ms = _time(g, Qd, npd, k, rerank, max_nprobe, opts, ids, dist, reps)
        trials.append(dict(cand, ms=ms, probe_agreement=agree[ck]))
        if log:
            log(f"tune {cand}: {ms:.3f} ms")
    best = min(trials, key=lambda r: r["ms"])
    best_opts = {k_: best[k_] for k_ in ("form", "coarse", "widen", "widen_add", "pool_cap",
                                         "grid", "rounds", "first_lists") if k_ in best}
    # Launch orders of the fastest schedule (the defaults, longest first,
    # were measured above).
    lists = (0, 1) if best_opts["form"] == "batched" else (0,)
    for qo in (0, 1):
        for lo in lists:
            if qo == 0 and lo == 0:
                continue
            cand = dict(best_opts, query_order=qo, list_order=lo)
            ms = _time(g, Qd, npd, k, rerank, max_nprobe, make_opts(**cand), ids, dist, reps)
            trials.append(dict(cand, ms=ms, probe_agreement=best["probe_agreement"]))
            if log:
                log(f"tune {cand}: {ms:.3f} ms")
            if ms < best["ms"]:
                best = trials[-1]
    best_opts = {k_: best[k_] for k_ in ("form", "coarse", "widen", "widen_add", "pool_cap",
                                         "grid", "rounds", "first_lists", "query_order",
                                         "list_order") if k_ in best}
    # The same schedule captured into a hipGraph and replayed (a side stream:
    # capture needs one), kept when faster.
    side = torch.cuda.Stream()
    gms = _time(g, Qd, npd, k, rerank, max_nprobe, make_opts(**best_opts, use_graph=True), ids,
                dist, reps, stream=side)
    trials.append(dict(best_opts, use_graph=True, ms=gms, probe_agreement=best["probe_agreement"]))
    if log:
        log(f"tune {best_opts} graph-captured: {gms:.3f} ms (eager {best['ms']:.3f} ms)")
    if gms < best["ms"]:
        best_opts["use_graph"] = True
        best = trials[-1]
    report = dict(key=key, best=opts_dict(make_opts(**best_opts)), best_ms=best["ms"],
                  trials=trials, seconds=round(time.time() - t0, 2))
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        cache[key] = report
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return make_opts(**best_opts), dict(report, cached=False)


__all__ = ["autotune", "default_space", "shape_key", "DEFAULT_CACHE", "COARSE"]
