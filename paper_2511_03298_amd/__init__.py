"""Python binding of the gfx950 IVF-PQ search library (libivfpq.so).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the search runs in the library's HIP
kernels. The C ABI is declared in include/ivf.h. Loading fails loudly when
the library has not been built.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
# IVFPQ_LIB selects another build of the same library (the host-sanitizer
# build of the ABI tests); by default the in-tree one.
LIB_PATH = os.environ.get("IVFPQ_LIB") or os.path.join(PKG_DIR, "libivfpq.so")

IVF_OK, IVF_ERR_INVALID_ARG, IVF_ERR_DEVICE, IVF_ERR_WORKSPACE = 0, 1, 2, 3
IVF_ERR_UNSUPPORTED, IVF_ERR_INTERNAL = 4, 5
METRIC = {"l2": 0, "ip": 1}
DTYPE = {"f32": 0, "bf16": 1, "u8": 2}
COARSE = {"exact": 0, "f32": 1, "bf16": 2, "fp8": 3}
FORM = {"plain": 0, "batched": 1}
STATIC_SCRATCH_BYTES = 64 << 20  # IVF_STATIC_SCRATCH_BYTES of ivf.h

EXPORTED = [
    "ivf_default_opts", "ivf_tables_bytes", "ivf_build_tables", "ivf_search_workspace_bytes",
    "ivf_search", "ivf_search_with_probes", "ivf_debug_probes", "ivf_debug_luts",
    "ivf_debug_candidates", "ivf_get_table_layout", "ivf_get_device_error", "ivf_destroy",
    "ivf_last_error", "ivf_profile_enable", "ivf_profile_read", "ivf_debug_coarse_scores",
    "ivf_assign_workspace_bytes", "ivf_assign", "ivf_encode", "ivf_debug_adaptive",
    "ivf_assign_spill_workspace_bytes", "ivf_assign_spill", "ivf_debug_batched_luts",
    "ivf_search_static",
]
STAGES = ("coarse", "select", "prep", "scan", "merge", "rerank")


class IvfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"ivf status {status}: {message}")
        self.status = status


class IndexDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("L", ctypes.c_int32),
                ("m", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("base_dtype", ctypes.c_int32), ("base", ctypes.c_void_p),
                ("centroids", ctypes.c_void_p), ("probe_centroids", ctypes.c_void_p),
                ("codebooks", ctypes.c_void_p), ("codes", ctypes.c_void_p),
                ("list_offsets", ctypes.c_void_p), ("list_ids", ctypes.c_void_p),
                ("d_base", ctypes.c_int32), ("dims", ctypes.c_void_p),
                ("copies", ctypes.c_int32)]


class SearchOpts(ctypes.Structure):
    _fields_ = [("coarse", ctypes.c_int32), ("widen", ctypes.c_int32),
                ("form", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("pool_cap", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("spill_cap", ctypes.c_int32),
                ("adaptive", ctypes.c_int32), ("nprobe_init", ctypes.c_int32),
                ("nprobe_min", ctypes.c_int32), ("reorder_min", ctypes.c_int32),
                ("p0", ctypes.c_float), ("p1", ctypes.c_float),
                ("widen_add", ctypes.c_int32), ("first_lists", ctypes.c_int32),
                ("query_order", ctypes.c_int32), ("list_order", ctypes.c_int32)]


class TableLayout(ctypes.Structure):
    _fields_ = [(name, ctypes.c_size_t) for name in (
        "codes", "slot_ids", "block_offsets", "list_len", "centroids", "probe_centroids",
        "codebooks", "probe_norms", "probe_f32", "probe_bf16", "probe_fp8", "probe_fp8_scale",
        "dims", "total")] + \
        [(name, ctypes.c_int32) for name in (
            "words_per_point", "m_padded", "blocks", "L_padded", "d_padded", "reserved")]


_LIB = None


def _declare(lib):
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "ivf_default_opts": (None, [P]),
        "ivf_tables_bytes": (SZ, [P]),
        "ivf_build_tables": (I32, [P, P, SZ, P, P]),
        "ivf_search_workspace_bytes": (SZ, [P, I32, I32, I32, I32, P]),
        "ivf_search": (I32, [P, P, I32, P, I32, I32, I32, P, P, SZ, P, P, P]),
        "ivf_search_with_probes": (I32, [P, P, I32, P, P, I32, I32, I32, P, P, SZ, P, P, P]),
        "ivf_debug_probes": (I32, [P, P, I32, P, I32, P, P, SZ, P, P]),
        "ivf_debug_luts": (I32, [P, P, I32, P, P, I32, P, P, P, P, P]),
        "ivf_debug_coarse_scores": (I32, [P, P, I32, P, P, SZ, P, P]),
        "ivf_debug_candidates": (I32, [P, P, I32, P, P, I32, I32, P, P, SZ, P, P]),
        "ivf_get_table_layout": (I32, [P, P]),
        "ivf_get_device_error": (I32, [P, P, P, P]),
        "ivf_destroy": (None, [P]),
        "ivf_profile_enable": (I32, [P, I32]),
        "ivf_profile_read": (I32, [P, P, P]),
        "ivf_last_error": (ctypes.c_char_p, []),
        "ivf_assign_workspace_bytes": (SZ, [I32, I32, I32, I32]),
        "ivf_assign": (I32, [P, I32, I32, I32, P, I64, I32, I32, I32, P, SZ, P, P]),
        "ivf_encode": (I32, [P, I64, I32, P, P, P, I32, P, P]),
        "ivf_assign_spill_workspace_bytes": (SZ, [I32, I32, I32]),
        "ivf_assign_spill": (I32, [P, I32, I32, P, I64, P, ctypes.c_float, I32, P, SZ, P, P]),
        "ivf_debug_adaptive": (I32, [P, P, I32, P, I32, I32, I32, P, P, SZ, P, P, P]),
        "ivf_debug_batched_luts": (I32, [P, P, I32, P, P, I32, P, SZ, P, P, P, P]),
        "ivf_search_static": (I32, [P, P, I32, P, I32, I32, I32, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _ = I64


def lib():
    """Load libivfpq.so (built in-tree by __graft_entry__.build())."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        handle = ctypes.CDLL(LIB_PATH)
        _declare(handle)
        _LIB = handle
    return _LIB


def last_error() -> str:
    return lib().ivf_last_error().decode()


def check(status: int):
    if status != IVF_OK:
        raise IvfError(status, last_error())


def make_opts(coarse: str = "exact", widen: int = 2, form: str = "plain",
              use_graph: bool = False, pool_cap: int = 0, grid: int = 0,
              rounds: int = 0, spill_cap: int = 0,
              adaptive: Optional[dict] = None, widen_add: int = 0,
              first_lists: int = 0, query_order: int = 0,
              list_order: int = 0) -> SearchOpts:
    """adaptive: dict(nprobe_init, nprobe_min, reorder_min, p0, p1) turns on
    the per-query probe count and re-rank size of Eq. 2 (nprobe[q] and
    rerank are the maxima)."""
    o = SearchOpts()
    lib().ivf_default_opts(ctypes.byref(o))
    o.coarse, o.widen, o.form = COARSE[coarse], int(widen), FORM[form]
    o.use_graph, o.pool_cap, o.grid = int(bool(use_graph)), int(pool_cap), int(grid)
    o.rounds, o.spill_cap = int(rounds), int(spill_cap)
    o.widen_add = int(widen_add)
    o.first_lists = int(first_lists)
    o.query_order, o.list_order = int(query_order), int(list_order)
    if adaptive:
        o.adaptive = 1
        o.nprobe_init = int(adaptive["nprobe_init"])
        o.nprobe_min = int(adaptive["nprobe_min"])
        o.reorder_min = int(adaptive["reorder_min"])
        o.p0, o.p1 = float(adaptive["p0"]), float(adaptive["p1"])
    return o


def opts_dict(o: SearchOpts) -> dict:
    inv_c = {v: k for k, v in COARSE.items()}
    inv_f = {v: k for k, v in FORM.items()}
    d = dict(coarse=inv_c[o.coarse], widen=o.widen, form=inv_f[o.form],
             use_graph=bool(o.use_graph), pool_cap=o.pool_cap, grid=o.grid,
             rounds=o.rounds, spill_cap=o.spill_cap, widen_add=o.widen_add,
             first_lists=o.first_lists, query_order=o.query_order,
             list_order=o.list_order)
    if o.adaptive:
        d["adaptive"] = dict(nprobe_init=o.nprobe_init, nprobe_min=o.nprobe_min,
                             reorder_min=o.reorder_min, p0=o.p0, p1=o.p1)
    return d


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class GpuIndex:
    """An IVF-PQ index resident on the GPU.

    Inputs are the trained index arrays (numpy or torch); `base` rows are kept
    referenced by the library for the exact re-rank.
    """

    def __init__(self, base, centroids, codebooks, codes, list_offsets, list_ids,
                 metric: str, probe_centroids=None, base_dtype: str = "f32",
                 device: str = "cuda", dims=None, copies: int = 1):
        import numpy as np
        import torch
        L = lib()

        def dev(a, dtype):
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            return t.to(device=device, dtype=dtype).contiguous()

        if base_dtype == "bf16":
            self.base = dev(base, torch.bfloat16)
        elif base_dtype == "u8":
            # Byte vectors: the rows must be integers in [0, 255] (stored exactly).
            b = base if isinstance(base, torch.Tensor) else torch.from_numpy(np.asarray(base))
            if b.dtype != torch.uint8:
                bf = b.to(torch.float32)
                if not bool(((bf >= 0) & (bf <= 255) & (bf == torch.round(bf))).all()):
                    raise ValueError("base_dtype 'u8' needs integer components in [0, 255]")
            self.base = dev(b, torch.uint8)
        else:
            self.base = dev(base, torch.float32)
        self.centroids = dev(centroids, torch.float32)
        self.probe_centroids = None if probe_centroids is None else dev(probe_centroids, torch.float32)
        self.codebooks = dev(codebooks, torch.float32)
        codes_t = dev(codes, torch.uint8)
        ids_t = dev(list_ids, torch.int32)
        offs = np.ascontiguousarray(np.asarray(list_offsets, dtype=np.int64))
        n, d_base = self.base.shape
        Lc, d = self.centroids.shape
        m = self.codebooks.shape[0]
        # Component filtration: the index lives in the kept base columns.
        self.dims = None if dims is None else np.ascontiguousarray(np.asarray(dims, np.int32))
        self.n, self.d, self.L, self.m, self.metric = n, d, Lc, m, metric
        self.d_base = d_base
        # Spilled index (section 4.6.2): codes are per list entry.
        self.copies = int(copies)
        desc = IndexDesc(n=n, d=d, L=Lc, m=m, metric=METRIC[metric],
                         base_dtype=DTYPE[base_dtype], base=_ptr(self.base),
                         centroids=_ptr(self.centroids),
                         probe_centroids=_ptr(self.probe_centroids),
                         codebooks=_ptr(self.codebooks), codes=_ptr(codes_t),
                         list_offsets=offs.ctypes.data, list_ids=_ptr(ids_t),
                         d_base=d_base if self.dims is not None else 0,
                         dims=None if self.dims is None else self.dims.ctypes.data,
                         copies=self.copies)
        nbytes = L.ivf_tables_bytes(ctypes.byref(desc))
        if nbytes == 0:
            raise IvfError(IVF_ERR_INVALID_ARG, last_error())
        self.tables = torch.empty(nbytes, dtype=torch.uint8, device=device)
        handle = ctypes.c_void_p()
        check(L.ivf_build_tables(ctypes.byref(desc), self.tables.data_ptr(), nbytes, _stream(),
                                 ctypes.byref(handle)))
        self._h = handle
        self._ws = {}
        self.device = device

    @classmethod
    def from_index(cls, index: dict, X, base_dtype: str = "f32", device: str = "cuda"):
        return cls(X, index["cm"], index["codebooks"], index["codes"], index["list_offsets"],
                   index["list_ids"], index["metric"], probe_centroids=index["cp"],
                   base_dtype=base_dtype, device=device, dims=index.get("dims"),
                   copies=int(index.get("copies", 1)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.ivf_destroy(h)
            self._h = None

    # -- helpers ----------------------------------------------------------
    def layout(self) -> TableLayout:
        lay = TableLayout()
        check(lib().ivf_get_table_layout(self._h, ctypes.byref(lay)))
        return lay

    def workspace(self, nq, max_nprobe, k, rerank, opts):
        import torch
        nbytes = lib().ivf_search_workspace_bytes(self._h, nq, max_nprobe, k, rerank,
                                                  ctypes.byref(opts))
        if nbytes == 0:
            raise IvfError(IVF_ERR_INVALID_ARG, last_error())
        # One cached workspace per stream (a search enqueued on another stream
        # gets its own, so two streams never share one in flight); a stream's
        # workspace is replaced only when a call needs a different size.
        stream = torch.cuda.current_stream().cuda_stream
        ws = self._ws.get(stream)
        if ws is None or ws.numel() != nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._ws[stream] = ws
        self._last_ws = ws
        return ws

    def _queries(self, queries):
        import numpy as np
        import torch
        q = queries if isinstance(queries, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(queries, dtype=np.float32))
        return q.to(device=self.device, dtype=torch.float32).contiguous()

    def _nprobe(self, nprobe, nq):
        import numpy as np
        import torch
        if isinstance(nprobe, int):
            return torch.full((nq,), nprobe, dtype=torch.int32, device=self.device)
        t = nprobe if isinstance(nprobe, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(nprobe, dtype=np.int32))
        return t.to(device=self.device, dtype=torch.int32).contiguous()

    # -- the search -------------------------------------------------------
    def search(self, queries, nprobe, k: int, rerank: int, max_nprobe: Optional[int] = None,
               opts: Optional[SearchOpts] = None, out=None):
        """Return (ids int64 [nq,k], dist float32 [nq,k]) as device tensors."""
        import torch
        q = self._queries(queries)
        nq = q.shape[0]
        npb = self._nprobe(nprobe, nq)
        if max_nprobe is None:
            max_nprobe = int(npb.max().item()) if nq else 1
            max_nprobe = max(1, min(max_nprobe, self.L))
        opts = opts or make_opts()
        ws = self.workspace(nq, max_nprobe, k, rerank, opts)
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int64, device=self.device)
            dist = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        else:
            ids, dist = out
        check(lib().ivf_search(self._h, _ptr(q), nq, _ptr(npb), max_nprobe, k, rerank,
                               ctypes.byref(opts), ws.data_ptr(), ws.numel(), _ptr(ids),
                               _ptr(dist), _stream()))
        self._keep = (q, npb)
        return ids, dist

    def search_static(self, queries, nprobe, k: int, rerank: int, max_nprobe: int,
                      opts: Optional[SearchOpts] = None, out=None):
        """ivf_search_static: the search with the library's fixed device scratch
        instead of a workspace (outputs may be passed in through `out`)."""
        import torch
        q = self._queries(queries)
        nq = q.shape[0]
        npb = self._nprobe(nprobe, nq)
        opts = opts or make_opts()
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int64, device=self.device)
            dist = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        else:
            ids, dist = out
        check(lib().ivf_search_static(self._h, _ptr(q), nq, _ptr(npb), max_nprobe, k, rerank,
                                      ctypes.byref(opts), _ptr(ids), _ptr(dist), _stream()))
        self._keep = (q, npb)
        return ids, dist

    def search_with_probes(self, queries, probes, nprobe, k: int, rerank: int,
                           opts: Optional[SearchOpts] = None):
        import torch
        q = self._queries(queries)
        nq = q.shape[0]
        pr = probes.to(device=self.device, dtype=torch.int32).contiguous()
        max_nprobe = pr.shape[1]
        npb = self._nprobe(nprobe, nq)
        opts = opts or make_opts()
        ws = self.workspace(nq, max_nprobe, k, rerank, opts)
        ids = torch.empty((nq, k), dtype=torch.int64, device=self.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        check(lib().ivf_search_with_probes(self._h, _ptr(q), nq, _ptr(pr), _ptr(npb), max_nprobe,
                                           k, rerank, ctypes.byref(opts), ws.data_ptr(),
                                           ws.numel(), _ptr(ids), _ptr(dist), _stream()))
        return ids, dist

    def debug_adaptive(self, queries, nprobe, k: int, rerank: int, max_nprobe=None, opts=None):
        """Per-query (nprobe, reorder) the adaptive search would use."""
        import torch
        q = self._queries(queries)
        nq = q.shape[0]
        npb = self._nprobe(nprobe, nq)
        if max_nprobe is None:
            max_nprobe = max(1, min(int(npb.max().item()), self.L))
        ws = self.workspace(nq, max_nprobe, k, rerank, opts)
        out_n = torch.empty(nq, dtype=torch.int32, device=self.device)
        out_r = torch.empty(nq, dtype=torch.int32, device=self.device)
        check(lib().ivf_debug_adaptive(self._h, _ptr(q), nq, _ptr(npb), max_nprobe, k, rerank,
                                       ctypes.byref(opts), ws.data_ptr(), ws.numel(),
                                       _ptr(out_n), _ptr(out_r), _stream()))
        return out_n, out_r

    def debug_probes(self, queries, nprobe, max_nprobe=None, opts=None):
        import torch
        q = self._queries(queries)
        nq = q.shape[0]
        npb = self._nprobe(nprobe, nq)
        if max_nprobe is None:
            max_nprobe = max(1, min(int(npb.max().item()), self.L))
        opts = opts or make_opts()
        ws = self.workspace(nq, max_nprobe, 1, 1, opts)
        out = torch.empty((nq, max_nprobe), dtype=torch.int32, device=self.device)
        check(lib().ivf_debug_probes(self._h, _ptr(q), nq, _ptr(npb), max_nprobe,
                                     ctypes.byref(opts), ws.data_ptr(), ws.numel(), _ptr(out),
                                     _stream()))
        return out

    def debug_coarse_scores(self, queries, coarse: str):
        import torch
        q = self._queries(queries)
        nq = q.shape[0]
        opts = make_opts(coarse=coarse)
        ws = self.workspace(nq, 1, 1, 1, opts)
        out = torch.empty((nq, self.L), dtype=torch.float32, device=self.device)
        check(lib().ivf_debug_coarse_scores(self._h, _ptr(q), nq, ctypes.byref(opts),
                                            ws.data_ptr(), ws.numel(), _ptr(out), _stream()))
        return out

    def debug_luts(self, queries, probes, nprobe):
        import torch
        q = self._queries(queries)
        nq = q.shape[0]
        pr = probes.to(device=self.device, dtype=torch.int32).contiguous()
        max_nprobe = pr.shape[1]
        npb = self._nprobe(nprobe, nq)
        lut = torch.zeros((nq, max_nprobe, self.m, 16), dtype=torch.uint8, device=self.device)
        lo = torch.zeros((nq, max_nprobe, self.m), dtype=torch.float32, device=self.device)
        delta = torch.zeros((nq, max_nprobe), dtype=torch.float32, device=self.device)
        B = torch.zeros((nq, max_nprobe), dtype=torch.float32, device=self.device)
        check(lib().ivf_debug_luts(self._h, _ptr(q), nq, _ptr(pr), _ptr(npb), max_nprobe,
                                   _ptr(lut), _ptr(lo), _ptr(delta), _ptr(B), _stream()))
        return lut, lo, delta, B

    def debug_batched_luts(self, queries, probes, nprobe):
        """The batched form's tables for caller-given probes: (lut u8
        [nq,max_nprobe,m,16], delta, B [nq,max_nprobe]) device tensors."""
        import torch
        q = self._queries(queries)
        nq = q.shape[0]
        pr = probes.to(device=self.device, dtype=torch.int32).contiguous()
        max_nprobe = pr.shape[1]
        npb = self._nprobe(nprobe, nq)
        ws = self.workspace(nq, max_nprobe, 1, 1, make_opts(form="batched"))
        lut = torch.zeros((nq, max_nprobe, self.m, 16), dtype=torch.uint8, device=self.device)
        delta = torch.zeros((nq, max_nprobe), dtype=torch.float32, device=self.device)
        B = torch.zeros((nq, max_nprobe), dtype=torch.float32, device=self.device)
        check(lib().ivf_debug_batched_luts(self._h, _ptr(q), nq, _ptr(pr), _ptr(npb), max_nprobe,
                                           ws.data_ptr(), ws.numel(), _ptr(lut), _ptr(delta),
                                           _ptr(B), _stream()))
        return lut, delta, B

    def debug_candidates(self, queries, probes, nprobe, rerank: int, opts=None):
        import torch
        q = self._queries(queries)
        nq = q.shape[0]
        pr = probes.to(device=self.device, dtype=torch.int32).contiguous()
        max_nprobe = pr.shape[1]
        npb = self._nprobe(nprobe, nq)
        opts = opts or make_opts()
        ws = self.workspace(nq, max_nprobe, 1, rerank, opts)
        keys = torch.empty((nq, rerank), dtype=torch.int64, device=self.device)
        check(lib().ivf_debug_candidates(self._h, _ptr(q), nq, _ptr(pr), _ptr(npb), max_nprobe,
                                         rerank, ctypes.byref(opts), ws.data_ptr(), ws.numel(),
                                         _ptr(keys), _stream()))
        return keys

    def profile(self, on: bool = True):
        check(lib().ivf_profile_enable(self._h, int(on)))

    def profile_read(self):
        """Summed milliseconds per stage and the number of searches since the last read."""
        ms = (ctypes.c_float * len(STAGES))()
        cnt = ctypes.c_int32()
        check(lib().ivf_profile_read(self._h, ms, ctypes.byref(cnt)))
        return dict(zip(STAGES, list(ms))), cnt.value

    def device_error(self) -> int:
        """Device error mask of the last search's workspace (read and cleared):
        1 = an nprobe out of range, 2 = a bad caller-given probe row."""
        ws = getattr(self, "_last_ws", None)
        if ws is None:
            return 0
        mask = ctypes.c_int32()
        check(lib().ivf_get_device_error(self._h, ws.data_ptr(), ctypes.byref(mask), _stream()))
        return mask.value


def assign_lists(centroids, X, metric: str, coarse: str = "bf16", widen: int = 4,
                 chunk: int = 65536):
    """Nearest list per row of X (device tensors) via ivf_assign; int32 tensor."""
    import torch
    L, d = centroids.shape
    n = X.shape[0]
    chunk = max(1, min(chunk, n))
    nb = lib().ivf_assign_workspace_bytes(L, d, chunk, COARSE[coarse])
    if nb == 0:
        raise IvfError(IVF_ERR_INVALID_ARG, last_error())
    ws = torch.empty(nb, dtype=torch.uint8, device=X.device)
    out = torch.empty(n, dtype=torch.int32, device=X.device)
    check(lib().ivf_assign(_ptr(centroids), L, d, METRIC[metric], _ptr(X), n, chunk,
                           COARSE[coarse], widen, ws.data_ptr(), nb, _ptr(out), _stream()))
    return out


def assign_spill(centroids, X, primary, lam: float = 1.0, chunk: int = 65536):
    """SOAR spill list per row of X (device tensors) via ivf_assign_spill: the
    list l != primary minimising ||x - c_l||^2 + lam <x - c_l, r>^2 / ||r||^2
    with r = x - c_primary (section 4.6.2); int32 tensor."""
    import torch
    L, d = centroids.shape
    n = X.shape[0]
    chunk = max(1, min(chunk, n))
    nb = lib().ivf_assign_spill_workspace_bytes(L, d, chunk)
    if nb == 0:
        raise IvfError(IVF_ERR_INVALID_ARG, last_error())
    ws = torch.empty(nb, dtype=torch.uint8, device=X.device)
    out = torch.empty(n, dtype=torch.int32, device=X.device)
    prim = primary.to(dtype=torch.int32).contiguous()
    check(lib().ivf_assign_spill(_ptr(centroids), L, d, _ptr(X), n, _ptr(prim), float(lam),
                                 chunk, ws.data_ptr(), nb, _ptr(out), _stream()))
    return out


def encode_codes(X, centroids, lists, codebooks):
    """PQ codes [n, m] uint8 of residuals against the lists' mean centroids."""
    import torch
    n, d = X.shape
    m = codebooks.shape[0]
    out = torch.empty((n, m), dtype=torch.uint8, device=X.device)
    check(lib().ivf_encode(_ptr(X), n, d, _ptr(centroids), _ptr(lists), _ptr(codebooks), m,
                           _ptr(out), _stream()))
    return out


def decode_keys(keys):
    """Split candidate keys (int64 view of uint64) into (a float32, id int64) numpy arrays.

    Padding keys (all ones) decode to (+inf, -1).
    """
    import numpy as np
    k = np.asarray(keys).view(np.uint64)
    none = k == np.uint64(0xFFFFFFFFFFFFFFFF)
    o = (k >> np.uint64(32)).astype(np.uint32)
    bits = np.where(o & np.uint32(0x80000000), o & np.uint32(0x7FFFFFFF), ~o).astype(np.uint32)
    a = bits.view(np.float32).copy()
    ids = (k & np.uint64(0xFFFFFFFF)).astype(np.int64)
    a[none] = np.inf
    ids[none] = -1
    return a, ids
