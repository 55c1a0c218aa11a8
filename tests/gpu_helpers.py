"""Shared helpers of the GPU parity tests (comparison against the oracle)."""

import numpy as np

import oracle

REL_TOL = 1e-5   # FP32 re-rank distance vs FP64, relative
TIE_BAND = 2e-5  # final ids may differ only among candidates this close


def oracle_stages(index, X, Q, nprobe, k, R):
    return oracle.search(index, X, Q, nprobe, k, R, want_stages=True)


def unpack_tables(tables_u8, layout, m):
    """Read the packed code blocks and slot ids back from table memory."""
    raw = np.asarray(tables_u8)
    W, blocks = layout.words_per_point, layout.blocks
    words = raw[layout.codes:layout.codes + blocks * W * 64 * 4].view(np.uint32).reshape(blocks, W, 64)
    slot_ids = raw[layout.slot_ids:layout.slot_ids + blocks * 64 * 4].view(np.int32).reshape(blocks * 64)
    codes = np.zeros((blocks * 64, W * 8), dtype=np.uint8)
    for w in range(W):
        for s in range(8):
            codes[:, w * 8 + s] = ((words[:, w, :] >> np.uint32(4 * s)) & np.uint32(15)).reshape(-1)
    return codes[:, :m], slot_ids, codes[:, m:]


def check_final(ids_g, dist_g, res, X, Q, metric, exact_ids=False):
    """GPU re-rank vs the oracle's FP64 re-rank of the same candidates."""
    ids_o, dist_o = res["ids"], res["dist"]
    for qi in range(len(Q)):
        g = ids_g[qi]
        o = ids_o[qi]
        assert (g >= 0).sum() == (o >= 0).sum(), qi
        valid = g >= 0
        rows = X[g[valid]].astype(np.float64)
        q64 = Q[qi].astype(np.float64)
        if metric == "l2":
            e64 = ((rows - q64) ** 2).sum(1)
            scale = np.abs(e64)
        else:
            e64 = rows @ q64
            scale = np.maximum(np.abs(e64), (np.abs(rows) * np.abs(q64)).sum(1))
        err = np.abs(dist_g[qi][valid].astype(np.float64) - e64)
        assert np.all(err <= REL_TOL * scale + 1e-30), (qi, err.max())
        if exact_ids:
            assert np.array_equal(g, o), qi
        else:
            # Same multiset of distances up to the tie band.
            do = dist_o[qi][o >= 0]
            band = TIE_BAND * np.maximum(np.abs(do), 1e-30)
            if metric == "ip":
                band = np.maximum(band, TIE_BAND * scale.max())
            assert np.all(np.abs(np.sort(e64) - np.sort(do)) <= band), qi
            mism = set(g[valid].tolist()) ^ set(o[o >= 0].tolist())
            if mism:
                kth = do[-1]
                for i in mism:
                    r = X[i].astype(np.float64)
                    e = ((r - q64) ** 2).sum() if metric == "l2" else r @ q64
                    assert abs(e - kth) <= TIE_BAND * max(abs(kth), 1e-30) + \
                        (TIE_BAND * scale.max() if metric == "ip" else 0), (qi, i)
