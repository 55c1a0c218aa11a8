"""Parity at the benchmark's full size: 1M x 128 integer L2 data, 1024 lists,
m = 64, 10k queries, nprobe 32, k 10, R 200, searched in the launch
configurations bench.py times (plain + exact coarse, batched + BF16 coarse,
batched + exact coarse);
sampled queries are recomputed by the oracle one by one.
"""

import numpy as np
import pytest

import oracle
from gpu_helpers import check_final

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_FULL = {}


def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not _FULL:
        import paper_2511_03298_amd as ivf
        from workloads import CONFIGS, make_workload, train_index
        cfg = CONFIGS["c2"]
        print("[fullsize] generating and training 1M x 128", flush=True)
        X, Q, nprobe = make_workload(cfg)
        index = train_index(X, cfg)
        g = ivf.GpuIndex.from_index(index, X)
        _FULL.update(cfg=cfg, X=X, Q=Q, nprobe=nprobe, index=index, g=g)
    return _FULL


SAMPLE = [0, 1, 997, 4242, 7777, 9999]


@pytest.mark.parametrize("form,coarse", [("plain", "exact"), ("batched", "bf16"),
                                        ("batched", "exact")])
def test_fullsize_sampled_queries(form, coarse):
    import paper_2511_03298_amd as ivf
    f = full()
    cfg, X, Q, nprobe, index, g = f["cfg"], f["X"], f["Q"], f["nprobe"], f["index"], f["g"]
    opts = ivf.make_opts(form=form, coarse=coarse)
    Qd = torch.from_numpy(Q).cuda()
    npd = torch.from_numpy(nprobe).cuda()
    ids, dist = g.search(Qd, npd, cfg.k, cfg.R, opts=opts)
    probes = g.debug_probes(Qd, npd, opts=opts).cpu().numpy()
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    assert g.device_error() == 0
    res = oracle.search(index, X, Q[SAMPLE], nprobe[SAMPLE], cfg.k, cfg.R, want_stages=True)
    same = [i for i, qi in enumerate(SAMPLE)
            if np.array_equal(probes[qi, :nprobe[qi]], res["probes"][i])]
    if coarse == "exact":
        assert len(same) == len(SAMPLE)
    assert len(same) >= len(SAMPLE) - 1
    sub = {k: v[same] for k, v in res.items() if k in ("ids", "dist")}
    rows = [SAMPLE[i] for i in same]
    check_final(ids[rows], dist[rows], sub, X, Q[rows], cfg.metric, exact_ids=True)
    # Candidate pools, in the same form, bit for bit.
    P = torch.from_numpy(probes[rows]).cuda()
    keys = g.debug_candidates(Qd[rows], P, npd[rows], cfg.R, opts=opts).cpu().numpy()
    a, cid = ivf.decode_keys(keys)
    assert np.array_equal(cid, res["cand_id"][same])
    assert np.array_equal(a.view(np.uint32), res["cand_a"][same].view(np.uint32))


def test_fullsize_forms_agree():
    import paper_2511_03298_amd as ivf
    f = full()
    cfg, Q, nprobe, g = f["cfg"], f["Q"], f["nprobe"], f["g"]
    Qd = torch.from_numpy(Q).cuda()
    npd = torch.from_numpy(nprobe).cuda()
    a = g.search(Qd, npd, cfg.k, cfg.R, opts=ivf.make_opts(form="plain"))
    b = g.search(Qd, npd, cfg.k, cfg.R, opts=ivf.make_opts(form="batched"))
    assert torch.equal(a[0], b[0]) and torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))
