"""ivf_search_static (the search with the library's fixed device scratch, for
callers that cannot allocate) against ivf_search with a caller workspace.

Both run the same kernels, so ids and distances must agree bit for bit; the
first call's re-ranked distances are also checked against the oracle. Two
calls in a row, the second with fewer queries, show that what the first one
left in the shared scratch does not leak into the second.
"""

import numpy as np
import pytest

from conftest import cached_workload
from gpu_helpers import check_final, oracle_stages

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    # name -> (workload, n, nq, L, ncomp, overrides)
    "c2s": ("c2", 40_000, 40, 64, 40, dict(nprobe=(6, 6))),
    "c3s": ("c3", 30_000, 40, 80, 80, dict(nprobe=(8, 32))),
}
_STATE = {}


def case(name):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_03298_amd as ivf
    if name not in _STATE:
        wl, n, nq, L, ncomp, kw = CASES[name]
        cfg, X, Q, nprobe, index = cached_workload(wl, n, nq, L=L, ncomp=ncomp, **kw)
        print(f"[no-alloc case {name}] n={cfg.n} d={cfg.d} L={cfg.L} m={cfg.m} nq={cfg.nq}",
              flush=True)
        g = ivf.GpuIndex.from_index(index, X, base_dtype=cfg.base_dtype)
        _STATE[name] = (cfg, X, Q, nprobe, index, g)
    return _STATE[name]


def _bits(ids, dist):
    return ids.cpu().numpy(), dist.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("form,coarse", [("plain", "exact"), ("batched", "bf16"),
                                         ("batched", "exact")])
@pytest.mark.parametrize("name", ["c2s", "c3s"])
def test_static_scratch_matches_workspace_search(name, form, coarse):
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g = case(name)
    opts = ivf.make_opts(form=form, coarse=coarse)
    max_np = int(np.max(nprobe))
    # Call 1: the whole batch. Call 2: a smaller batch of other queries.
    sizes = [(0, cfg.nq), (cfg.nq // 2, cfg.nq // 2 + 7)]
    for lo, hi in sizes:
        q = np.ascontiguousarray(Q[lo:hi])
        npb = np.ascontiguousarray(nprobe[lo:hi])
        print(f"[no-alloc] {name} {form}/{coarse} queries [{lo}, {hi})", flush=True)
        ref = _bits(*g.search(q, npb, cfg.k, cfg.R, max_nprobe=max_np, opts=opts))
        got = _bits(*g.search_static(q, npb, cfg.k, cfg.R, max_np, opts=opts))
        torch.cuda.synchronize()
        assert np.array_equal(got[0], ref[0])
        assert np.array_equal(got[1], ref[1])
        assert g.device_error() == 0
        if lo == 0:
            res = oracle_stages(index, X, q, npb, cfg.k, cfg.R)
            check_final(got[0], got[1].view(np.float32), res, X, q, cfg.metric)


def test_static_scratch_limits():
    import paper_2511_03298_amd as ivf
    cfg, X, Q, nprobe, index, g = case("c3s")
    # A batch whose workspace (the score matrix alone: nq x L x 4 bytes)
    # exceeds the scratch is refused on the host, before any work.
    nq = ivf.STATIC_SCRATCH_BYTES // (cfg.L * 4) + 1
    q = torch.zeros((nq, cfg.d), dtype=torch.float32, device="cuda")
    npb = torch.ones(nq, dtype=torch.int32, device="cuda")
    with pytest.raises(ivf.IvfError) as e:
        g.search_static(q, npb, cfg.k, cfg.R, 1)
    assert e.value.status == ivf.IVF_ERR_WORKSPACE
    assert "static scratch" in str(e.value)
    # Graph capture inside the call is not offered.
    with pytest.raises(ivf.IvfError) as e:
        g.search_static(Q, nprobe, cfg.k, cfg.R, int(np.max(nprobe)),
                        opts=ivf.make_opts(use_graph=True))
    assert e.value.status == ivf.IVF_ERR_INVALID_ARG
    # After the refusals a normal call still answers like ivf_search.
    max_np = int(np.max(nprobe))
    ref = _bits(*g.search(Q, nprobe, cfg.k, cfg.R, max_nprobe=max_np))
    got = _bits(*g.search_static(Q, nprobe, cfg.k, cfg.R, max_np))
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
