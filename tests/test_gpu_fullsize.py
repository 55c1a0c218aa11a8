"""Parity at the benchmark's full sizes, in the launch configurations
bench.py times; sampled queries are recomputed by the oracle one by one.

* 1M x 128 integer L2 data, 1024 lists, m = 64, 10k queries, nprobe 32,
  k 10, R 200 (plain + exact coarse, batched + BF16 coarse, batched + exact
  coarse, and the batched schedule the autotuner picks there).
* The 10M x 768 workload's shape at a tenth of its points: 1M x 768 BF16
  unit vectors (inner product), 8192 lists, m = 192 (8-query work items),
  a 4096-query batch with per-query nprobe 4..256 (register-held selection
  over 8192-list rows, the 2 GiB survivor budget), k 10, R 256.

Candidate pools come from one launch over the whole batch (not a re-launch
for the sampled queries), so the thresholds, work items and merges are the
benchmark's.
"""

import numpy as np
import pytest

import oracle
from gpu_helpers import check_final

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_FULL = {}


def _full(which):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if which not in _FULL:
        import paper_2511_03298_amd as ivf
        from workloads import CONFIGS, make_workload, scaled, train_index
        if which == "c2":
            cfg = CONFIGS["c2"]
            print("[fullsize] generating and training 1M x 128", flush=True)
            X, Q, nprobe = make_workload(cfg)
            index = train_index(X, cfg)
        else:
            from paper_2511_03298_amd.train import train_index_gpu
            cfg = scaled("c5", n=1_000_000, nq=4096, L=8192, ncomp=8192)
            print("[fullsize] generating and training 1M x 768, 8192 lists", flush=True)
            X, Q, nprobe = make_workload(cfg)
            index = train_index_gpu(X, cfg.L, cfg.m, cfg.metric, seed=cfg.index)
            index = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in index.items()}
        g = ivf.GpuIndex.from_index(index, X, base_dtype=cfg.base_dtype)
        _FULL[which] = dict(cfg=cfg, X=X, Q=Q, nprobe=nprobe, index=index, g=g)
    return _FULL[which]


SAMPLES = {"c2": [0, 1, 997, 4242, 7777, 9999],
           "c5": [0, 1, 511, 1024, 2047, 2500, 3333, 4000, 4094, 4095]}


def _check_sampled(which, opts, exact_ids):
    import paper_2511_03298_amd as ivf
    f = _full(which)
    cfg, X, Q, nprobe, index, g = f["cfg"], f["X"], f["Q"], f["nprobe"], f["index"], f["g"]
    sample = SAMPLES[which]
    Qd = torch.from_numpy(Q).cuda()
    npd = torch.from_numpy(nprobe).cuda()
    max_np = int(nprobe.max())
    print(f"[fullsize {which}] {ivf.opts_dict(opts)} nq={len(Q)} max_nprobe={max_np}", flush=True)
    ids, dist = g.search(Qd, npd, cfg.k, cfg.R, max_nprobe=max_np, opts=opts)
    probes = g.debug_probes(Qd, npd, max_nprobe=max_np, opts=opts)
    # The pools of the whole batch in one launch of this schedule.
    keys = g.debug_candidates(Qd, probes, npd, cfg.R, opts=opts).cpu().numpy()
    probes = probes.cpu().numpy()
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    assert g.device_error() == 0
    res = oracle.search(index, X, Q[sample], nprobe[sample], cfg.k, cfg.R, want_stages=True)
    same = [i for i, qi in enumerate(sample)
            if np.array_equal(probes[qi, :nprobe[qi]], res["probes"][i])]
    if ivf.opts_dict(opts)["coarse"] == "exact":
        assert len(same) == len(sample)
    assert len(same) >= len(sample) - 1
    rows = [sample[i] for i in same]
    a, cid = ivf.decode_keys(keys[rows])
    assert np.array_equal(cid, res["cand_id"][same])
    assert np.array_equal(a.view(np.uint32), res["cand_a"][same].view(np.uint32))
    sub = {k: v[same] for k, v in res.items() if k in ("ids", "dist")}
    check_final(ids[rows], dist[rows], sub, X, Q[rows], cfg.metric, exact_ids=exact_ids)
    return f, rows, probes, res, same


@pytest.mark.parametrize("form,coarse,grid", [("plain", "exact", 0), ("batched", "bf16", 0),
                                              ("batched", "exact", 0), ("batched", "bf16", 4)])
def test_fullsize_1Mx128_sampled_queries(form, coarse, grid):
    import paper_2511_03298_amd as ivf
    _check_sampled("c2", ivf.make_opts(form=form, coarse=coarse, grid=grid), exact_ids=True)


def test_fullsize_1Mx128_forms_agree():
    import paper_2511_03298_amd as ivf
    f = _full("c2")
    cfg, Q, nprobe, g = f["cfg"], f["Q"], f["nprobe"], f["g"]
    Qd = torch.from_numpy(Q).cuda()
    npd = torch.from_numpy(nprobe).cuda()
    a = g.search(Qd, npd, cfg.k, cfg.R, opts=ivf.make_opts(form="plain"))
    b = g.search(Qd, npd, cfg.k, cfg.R, opts=ivf.make_opts(form="batched"))
    assert torch.equal(a[0], b[0]) and torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))


@pytest.mark.parametrize("form,coarse", [("batched", "bf16"), ("plain", "exact")])
def test_fullsize_768d_8192_lists_sampled_queries(form, coarse):
    import paper_2511_03298_amd as ivf
    f, rows, probes, res, same = _check_sampled("c5", ivf.make_opts(form=form, coarse=coarse),
                                                exact_ids=False)
    if form != "batched":
        return
    # The batched form's tables of the sampled queries' probed lists.
    g, Q, nprobe = f["g"], f["Q"], f["nprobe"]
    P = torch.from_numpy(probes[rows]).cuda()
    lut, delta, B = [t.cpu().numpy() for t in g.debug_batched_luts(Q[rows], P, nprobe[rows])]
    for r, i in enumerate(same):
        for pi, l in enumerate(res["probes"][i]):
            q8, _, d_o, B_o = res["luts"][(i, int(l))]
            assert np.array_equal(lut[r, pi], q8), (rows[r], l)
            assert delta[r, pi].view(np.uint32) == np.float32(d_o).view(np.uint32)
            assert B[r, pi].view(np.uint32) == np.float32(B_o).view(np.uint32)


def test_fullsize_768d_forms_agree():
    import paper_2511_03298_amd as ivf
    f = _full("c5")
    cfg, Q, nprobe, g = f["cfg"], f["Q"], f["nprobe"], f["g"]
    Qd = torch.from_numpy(Q).cuda()
    npd = torch.from_numpy(nprobe).cuda()
    a = g.search(Qd, npd, cfg.k, cfg.R, opts=ivf.make_opts(form="plain", coarse="bf16"))
    b = g.search(Qd, npd, cfg.k, cfg.R, opts=ivf.make_opts(form="batched", coarse="bf16"))
    assert torch.equal(a[0], b[0]) and torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))
