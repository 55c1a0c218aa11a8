// C ABI of the IVF-PQ search path: argument validation, table and
// workspace layout, and the order in which the kernels are enqueued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"
#include "ivf.h"

using namespace ivf;

// Per search a timeline of stage marks (stage, event); the time between two
// consecutive marks is attributed to the first one's stage. RING searches
// are kept between reads.
struct ivf_profile {
  static constexpr int RING = 64;
  static constexpr int MARKS = 32;
  bool on = false;
  int head = 0, count = 0;
  hipEvent_t ev[RING][MARKS] = {};
  int stage[RING][MARKS] = {};
  int nmarks[RING] = {};
  int cur = -1;
};

// Captured searches: one executable graph per set of launch arguments (the
// graph embeds every pointer and size), most recent first, at most 8.
struct ivf_graph_cache {
  struct Entry {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Entry> entries;
  ~ivf_graph_cache() {
    for (auto& e : entries) {
      if (e.exec) (void)hipGraphExecDestroy(e.exec);
      if (e.graph) (void)hipGraphDestroy(e.graph);
    }
  }
};

namespace {

thread_local std::string g_last_error;

ivf_status fail(ivf_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

ivf_status hip_fail(hipError_t e, const char* what) {
  return fail(IVF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define IVF_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

int32_t round_up_i(int64_t x, int64_t a) { return (int32_t)((x + a - 1) / a * a); }

// Workspace of ivf_search_static. The name is a host-side stand-in: kernels
// and copies get the per-device address that hipGetSymbolAddress returns.
static __device__ __align__(256) char scratch[IVF_STATIC_SCRATCH_BYTES];

constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_dev[SCRATCH_DEVICES] = {};

// Device address of the current device's scratch array, looked up once per
// device (each device holds its own copy at its own address).
ivf_status static_scratch(void** out) {
  int dev = -1;
  IVF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_DEVICES)
    return fail(IVF_ERR_DEVICE, "device ordinal beyond the 64 the static scratch tracks");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    IVF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || (uintptr_t)p % 256) return fail(IVF_ERR_INTERNAL, "static scratch address invalid");
    scratch_dev[dev] = p;
  }
  *out = scratch_dev[dev];
  return IVF_OK;
}

constexpr int32_t MAX_LISTS = MAX_SCAN_LISTS;
constexpr int32_t MAX_WIDEN = MAX_LISTS;

// Validate the descriptor and compute the table layout. Returns an empty
// string when valid, else the reason.
std::string plan_tables(const ivf_index_desc* d, ivf_table_layout* lay, int32_t* max_len) {
  if (!d) return "desc is NULL";
  if (d->n < 1 || d->n >= (int64_t)1 << 31) return "n must be in [1, 2^31)";
  if (d->d < 1) return "d must be >= 1";
  if (d->L < 1 || d->L > MAX_LISTS) return "L must be in [1, 16384]";
  if (d->m < 1 || d->m > MAX_M) return "m must be in [1, 256]";
  if (d->d % d->m != 0) return "d must be a multiple of m";
  if (d->metric != IVF_METRIC_L2 && d->metric != IVF_METRIC_IP) return "unknown metric";
  if (d->base_dtype != IVF_DTYPE_F32 && d->base_dtype != IVF_DTYPE_BF16 &&
      d->base_dtype != IVF_DTYPE_U8)
    return "unknown base dtype";
  if (!d->base || !d->centroids || !d->codebooks || !d->codes || !d->list_offsets ||
      !d->list_ids)
    return "a required pointer is NULL";
  const int64_t* off = d->list_offsets;
  if (off[0] != 0) return "list_offsets[0] must be 0";
  int64_t blocks = 0, mx = 0;
  for (int l = 0; l < d->L; ++l) {
    int64_t len = off[l + 1] - off[l];
    if (len < 0) return "list_offsets must be non-decreasing";
    blocks += (len + BLOCK_PTS - 1) / BLOCK_PTS;
    if (len > mx) mx = len;
  }
  if (d->copies < 0 || d->copies > 4) return "copies must be in 0..4";
  const int64_t copies = d->copies > 1 ? d->copies : 1;
  if (copies > 1 && d->n * copies >= ((int64_t)1 << 31) - 1) return "n * copies must be < 2^31 - 1";
  if (off[d->L] > d->n * copies) return copies > 1 ? "list_offsets[L] must be <= n * copies"
                                                   : "list_offsets[L] must be <= n";
  if (blocks * BLOCK_PTS >= ((int64_t)1 << 31)) return "too many list entries (blocks * 64 >= 2^31)";
  if (d->dims) {
    if (d->d_base < d->d) return "d_base must be >= d with dims";
    for (int j = 0; j < d->d; ++j) {
      if (d->dims[j] < 0 || d->dims[j] >= d->d_base) return "dims entries must be in [0, d_base)";
      if (j > 0 && d->dims[j] <= d->dims[j - 1]) return "dims must be strictly ascending";
    }
  } else if (d->d_base != 0 && d->d_base != d->d) {
    return "d_base must be 0 or d without dims";
  }
  std::memset(lay, 0, sizeof(*lay));
  const int32_t words = (d->m + 7) / 8;
  lay->words_per_point = words;
  lay->m_padded = words * 8;
  lay->blocks = (int32_t)blocks;
  lay->L_padded = round_up_i(d->L, TILE_L);
  lay->d_padded = round_up_i(d->d, TILE_D);
  const int32_t dsub = d->d / d->m;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  lay->codes = take((size_t)blocks * words * BLOCK_PTS * 4);
  lay->slot_ids = take((size_t)blocks * BLOCK_PTS * 4);
  lay->block_offsets = take((size_t)(d->L + 1) * 4);
  lay->list_len = take((size_t)d->L * 4);
  lay->centroids = take((size_t)d->L * d->d * 4);
  lay->probe_centroids = take((size_t)d->L * d->d * 4);
  lay->codebooks = take((size_t)lay->m_padded * KSUB * dsub * 4);
  lay->probe_norms = take((size_t)lay->L_padded * 4);
  lay->probe_f32 = take((size_t)lay->L_padded * lay->d_padded * 4);
  lay->probe_bf16 = take((size_t)lay->L_padded * lay->d_padded * 2);
  lay->probe_fp8 = take((size_t)lay->L_padded * lay->d_padded);
  lay->probe_fp8_scale = take((size_t)lay->L_padded * 4);
  lay->dims = take(d->dims ? (size_t)d->d * 4 : 0);
  // List indices by length, longest first: the batched scan serves the work
  // items of long lists first.
  take((size_t)d->L * 4);
  // Build-time scratch: a spilled index's per-point numbering array and flag
  // (else just the flag word), then the copy of the CSR offsets (int64).
  take(copies > 1 ? (size_t)(d->n + 64) * 4 : 64);
  take((size_t)(d->L + 1) * 8);
  lay->total = o;
  if (max_len) *max_len = (int32_t)mx;
  return "";
}

size_t list_off_section(const ivf_index_desc* d, const ivf_table_layout& lay) {
  return lay.total - align_up((size_t)(d->L + 1) * 8);
}

// Numbering scratch of a spilled index: [n] int32, then the flag word; on
// an index without copies only the flag word.
size_t copies_section(const ivf_index_desc* d, const ivf_table_layout& lay) {
  const bool spilled = d->copies > 1;
  return list_off_section(d, lay) - align_up(spilled ? (size_t)(d->n + 64) * 4 : 64);
}

// The longest-first list order: int32 [L], just before the numbering scratch.
size_t list_order_section(const ivf_index_desc* d, const ivf_table_layout& lay) {
  return copies_section(d, lay) - align_up((size_t)d->L * 4);
}

ivf_status check_device() {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n < 1) return fail(IVF_ERR_DEVICE, "no HIP device available");
  int dev = 0;
  IVF_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  IVF_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(IVF_ERR_DEVICE, std::string("device is ") + prop.gcnArchName +
                                    ", this library is built for gfx950");
  return IVF_OK;
}

uint32_t f32_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

ivf_status check_opts(const ivf_search_opts& o) {
  if (o.coarse < IVF_COARSE_EXACT || o.coarse > IVF_COARSE_FP8)
    return fail(IVF_ERR_INVALID_ARG, "opts.coarse out of range");
  // widen * max_nprobe stays below 2^28 (L <= 16384), in range of int32.
  if (o.widen < 1 || o.widen > MAX_WIDEN)
    return fail(IVF_ERR_INVALID_ARG, "opts.widen must be in [1, 16384]");
  if (o.widen_add < 0 || o.widen_add > MAX_LISTS)
    return fail(IVF_ERR_INVALID_ARG, "opts.widen_add must be in [0, 16384]");
  if (o.first_lists < 0 || o.first_lists > 64)
    return fail(IVF_ERR_INVALID_ARG, "opts.first_lists must be in [0, 64]");
  if (o.query_order != 0 && o.query_order != 1)
    return fail(IVF_ERR_INVALID_ARG, "opts.query_order must be 0 or 1");
  if (o.list_order != 0 && o.list_order != 1)
    return fail(IVF_ERR_INVALID_ARG, "opts.list_order must be 0 or 1");
  if (o.form != IVF_FORM_PLAIN && o.form != IVF_FORM_BATCHED)
    return fail(IVF_ERR_INVALID_ARG, "opts.form out of range");
  if (o.use_graph != 0 && o.use_graph != 1)
    return fail(IVF_ERR_INVALID_ARG, "opts.use_graph must be 0 or 1");
  if (o.pool_cap < 0 || o.pool_cap > 16384 || o.pool_cap % 256)
    return fail(IVF_ERR_INVALID_ARG, "opts.pool_cap must be 0 or a multiple of 256 up to 16384");
  if (o.grid < 0 || o.grid > 8) return fail(IVF_ERR_INVALID_ARG, "opts.grid must be in 0..8");
  if (o.rounds < 0 || o.rounds > 8) return fail(IVF_ERR_INVALID_ARG, "opts.rounds must be in 0..8");
  if (o.spill_cap != 0 && (o.spill_cap < 256 || o.spill_cap > 16384 - 256))
    return fail(IVF_ERR_INVALID_ARG, "opts.spill_cap must be 0 or in 256..16128");
  if (o.adaptive != 0 && o.adaptive != 1)
    return fail(IVF_ERR_INVALID_ARG, "opts.adaptive must be 0 or 1");
  if (o.adaptive) {
    if (o.nprobe_init < 1 || o.nprobe_min < 1 || o.reorder_min < 1)
      return fail(IVF_ERR_INVALID_ARG, "opts.nprobe_init, nprobe_min, reorder_min must be >= 1");
    if (!std::isfinite(o.p0) || !std::isfinite(o.p1))
      return fail(IVF_ERR_INVALID_ARG, "opts.p0 and opts.p1 must be finite");
  }
  return IVF_OK;
}

ivf_status check_search(const ivf_index* idx, int32_t nq, int32_t max_nprobe, int32_t k,
                        int32_t rerank) {
  if (!idx) return fail(IVF_ERR_INVALID_ARG, "index is NULL");
  if (nq < 0 || nq > MAX_QUERIES)
    return fail(IVF_ERR_INVALID_ARG, "nq must be in [0, 2^20] per call");
  if (max_nprobe < 1 || max_nprobe > idx->t.L)
    return fail(IVF_ERR_INVALID_ARG, "max_nprobe must be in [1, L]");
  if (rerank < 1 || rerank > MAX_RERANK)
    return fail(IVF_ERR_INVALID_ARG, "rerank must be in [1, 2048]");
  if (k < 1 || k > rerank) return fail(IVF_ERR_INVALID_ARG, "k must be in [1, rerank]");
  if ((int64_t)rerank * idx->t.copies > MAX_RERANK)
    return fail(IVF_ERR_INVALID_ARG, "rerank * copies must be <= 2048 on a spilled index");
  return IVF_OK;
}

ivf_status check_form(const ivf_index* idx, const ivf_search_opts& o) {
  if (o.form == IVF_FORM_BATCHED && idx->t.m > 192)
    return fail(IVF_ERR_UNSUPPORTED, "the batched form supports m <= 192");
  return IVF_OK;
}

}  // namespace

namespace ivf {

Workspace plan_workspace(const Tables& t, int32_t nq, int32_t max_nprobe, int32_t k,
                         int32_t rerank, const ivf_search_opts& o, char* base) {
  (void)k;
  Workspace w;
  std::memset(&w, 0, sizeof(w));
  const int32_t pool = rerank * t.copies;  // scan pool: keys of list entries
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  const size_t nqs = (size_t)(nq > 0 ? nq : 1);
  w.err = (int32_t*)take(16);
  w.order = (int32_t*)take(nqs * 4);
  w.order_bucket = (int32_t*)take(nqs * 4);
  w.order_hist = (int32_t*)take((size_t)2 * ORDER_BUCKETS * 4);
  w.scores = (float*)take(nqs * t.L * 4);
  w.probes = (int32_t*)take(nqs * max_nprobe * 4);
  w.nprobe_eff = (int32_t*)take(nqs * 4);
  w.reorder_eff = (int32_t*)take(nqs * 4);
  if (t.dims) w.qf = (float*)take(nqs * t.d * 4);
  w.bias = (float*)take(nqs * max_nprobe * 4);
  w.cand = (uint64_t*)take(nqs * pool * 8);
  if (t.copies > 1) w.cand_u = (uint64_t*)take(nqs * rerank * 8);
  if (o.coarse != IVF_COARSE_EXACT) {
    const size_t nq_pad = (size_t)round_up_i((int64_t)nqs, TILE_L);
    w.q_lowp = (void*)take(nq_pad * t.d_pad * 4);
    w.q_scale = (float*)take(nq_pad * 4);
  }
  w.pool_cap = o.pool_cap;
  w.grid = o.grid;
  w.first_lists = o.first_lists > 0 ? o.first_lists : 4;
  w.query_order = o.query_order;
  w.list_order = o.list_order;
  if (o.form == IVF_FORM_BATCHED) {
    w.spill_cap = o.spill_cap > 0 ? o.spill_cap : batched_spill_cap(pool, nq);
    w.p1 = (int32_t*)take(nqs * 4);
    w.thr = (uint64_t*)take(nqs * 8);
    w.list_cnt = (int32_t*)take((size_t)t.L * 4);
    w.list_cursor = (int32_t*)take((size_t)t.L * 4);
    w.list_start = (int32_t*)take((size_t)(t.L + 1) * 4);
    w.item_start = (int32_t*)take((size_t)(t.L + 1) * 4);
    w.item_list = (int32_t*)take(nqs * max_nprobe * 4);
    w.pairs = (int32_t*)take(nqs * max_nprobe * 8);
    w.queue = (uint32_t*)take(64);
    w.spill_cnt = (int32_t*)take(nqs * 4);
    w.spill = (uint64_t*)take(nqs * w.spill_cap * 8);
    w.redo = (int32_t*)take(nqs * 4);
    if (t.metric == IVF_METRIC_IP) {
      w.qlut = (uint8_t*)take(nqs * KSUB * t.m_pad);
      w.qlo_sum = (float*)take(nqs * 4);
      w.qdelta = (float*)take(nqs * 4);
    }
  }
  w.total = off;
  return w;
}

}  // namespace ivf

extern "C" {

void ivf_default_opts(ivf_search_opts* o) {
  if (!o) return;
  o->coarse = IVF_COARSE_EXACT;
  o->widen = 2;
  o->widen_add = 0;
  o->first_lists = 0;
  o->query_order = 0;
  o->list_order = 0;
  o->form = IVF_FORM_PLAIN;
  o->use_graph = 0;
  o->pool_cap = 0;
  o->grid = 0;
  o->rounds = 0;
  o->spill_cap = 0;
  o->adaptive = 0;
  o->nprobe_init = 8;
  o->nprobe_min = 1;
  o->reorder_min = 1;
  o->p0 = 0.0f;
  o->p1 = 0.0f;
}

const char* ivf_last_error(void) { return g_last_error.c_str(); }

size_t ivf_tables_bytes(const ivf_index_desc* desc) {
  ivf_table_layout lay;
  std::string why = plan_tables(desc, &lay, nullptr);
  if (!why.empty()) {
    g_last_error = why;
    return 0;
  }
  return lay.total;
}

ivf_status ivf_build_tables(const ivf_index_desc* desc, void* table_mem, size_t table_bytes,
                            void* stream, ivf_index** out) {
  if (!out) return fail(IVF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ivf_table_layout lay;
  int32_t max_len = 0;
  std::string why = plan_tables(desc, &lay, &max_len);
  if (!why.empty()) return fail(IVF_ERR_INVALID_ARG, why);
  if (!table_mem) return fail(IVF_ERR_INVALID_ARG, "table_mem is NULL");
  if ((uintptr_t)table_mem % ALIGN) return fail(IVF_ERR_INVALID_ARG, "table_mem not 256-byte aligned");
  if (table_bytes < lay.total) return fail(IVF_ERR_WORKSPACE, "table_mem smaller than ivf_tables_bytes");
  ivf_status st = check_device();
  if (st != IVF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)table_mem;

  Tables t;
  std::memset(&t, 0, sizeof(t));
  t.n = desc->n;
  t.d = desc->d;
  t.L = desc->L;
  t.m = desc->m;
  t.dsub = desc->d / desc->m;
  t.metric = desc->metric;
  t.base_dtype = desc->base_dtype;
  t.words = lay.words_per_point;
  t.m_pad = lay.m_padded;
  t.blocks = lay.blocks;
  t.L_pad = lay.L_padded;
  t.d_pad = lay.d_padded;
  t.max_list_len = max_len;
  t.d_base = desc->dims ? desc->d_base : desc->d;
  t.copies = desc->copies > 1 ? desc->copies : 1;
  t.dims = desc->dims ? (const int32_t*)(base + lay.dims) : nullptr;
  t.base = desc->base;
  t.codes = (const uint32_t*)(base + lay.codes);
  t.slot_ids = (const int32_t*)(base + lay.slot_ids);
  t.block_off = (const int32_t*)(base + lay.block_offsets);
  t.list_len = (const int32_t*)(base + lay.list_len);
  t.cm = (const float*)(base + lay.centroids);
  t.cp = (const float*)(base + lay.probe_centroids);
  t.codebooks = (const float*)(base + lay.codebooks);
  t.cp_norm2 = (const float*)(base + lay.probe_norms);
  t.cp_f32 = (const float*)(base + lay.probe_f32);
  t.cp_bf16 = (const uint16_t*)(base + lay.probe_bf16);
  t.cp_fp8 = (const uint8_t*)(base + lay.probe_fp8);
  t.cp_fp8_scale = (const float*)(base + lay.probe_fp8_scale);

  std::vector<int32_t> boff(desc->L + 1), llen(desc->L);
  boff[0] = 0;
  for (int l = 0; l < desc->L; ++l) {
    int64_t len = desc->list_offsets[l + 1] - desc->list_offsets[l];
    llen[l] = (int32_t)len;
    boff[l + 1] = boff[l] + (int32_t)((len + BLOCK_PTS - 1) / BLOCK_PTS);
  }
  // Lists by length, longest first (stable: ties keep index order).
  std::vector<int32_t> lorder(desc->L);
  for (int l = 0; l < desc->L; ++l) lorder[l] = l;
  std::stable_sort(lorder.begin(), lorder.end(),
                   [&](int32_t a, int32_t b) { return llen[a] > llen[b]; });
  t.list_order = (const int32_t*)(base + list_order_section(desc, lay));
  IVF_HIP(hipMemcpyAsync((void*)t.list_order, lorder.data(), lorder.size() * 4,
                         hipMemcpyHostToDevice, s));
  int64_t* list_off_dev = (int64_t*)(base + list_off_section(desc, lay));
  const size_t cb_bytes = (size_t)desc->m * KSUB * t.dsub * 4;
  const size_t cb_pad_bytes = (size_t)t.m_pad * KSUB * t.dsub * 4;
  IVF_HIP(hipMemcpyAsync((void*)t.block_off, boff.data(), boff.size() * 4, hipMemcpyHostToDevice, s));
  if (t.dims)
    IVF_HIP(hipMemcpyAsync((void*)t.dims, desc->dims, (size_t)desc->d * 4, hipMemcpyHostToDevice, s));
  IVF_HIP(hipMemcpyAsync((void*)t.list_len, llen.data(), llen.size() * 4, hipMemcpyHostToDevice, s));
  IVF_HIP(hipMemcpyAsync(list_off_dev, desc->list_offsets, (size_t)(desc->L + 1) * 8,
                         hipMemcpyHostToDevice, s));
  const size_t cbytes = (size_t)desc->L * desc->d * 4;
  IVF_HIP(hipMemcpyAsync((void*)t.cm, desc->centroids, cbytes, hipMemcpyDeviceToDevice, s));
  IVF_HIP(hipMemcpyAsync((void*)t.cp, desc->probe_centroids ? desc->probe_centroids : desc->centroids,
                         cbytes, hipMemcpyDeviceToDevice, s));
  IVF_HIP(hipMemsetAsync((void*)t.codebooks, 0, cb_pad_bytes, s));
  IVF_HIP(hipMemcpyAsync((void*)t.codebooks, desc->codebooks, cb_bytes, hipMemcpyDeviceToDevice, s));
  // Flag word: set on the device when a list entry names a point outside
  // [0, n) (the pack kernel then reads no codes for it) or, on a spilled
  // index, a point in more than `copies` lists.
  int32_t* first = (int32_t*)(base + copies_section(desc, lay));
  int32_t* flag = t.copies > 1 ? first + desc->n : first;
  IVF_HIP(launch_fill_u32((uint32_t*)flag, 0u, 1, s));
  IVF_HIP(launch_pack(t, desc->codes, list_off_dev, desc->list_ids, flag, s));
  IVF_HIP(launch_aux_tables(t, s));
  if (t.copies > 1) IVF_HIP(launch_number_copies(t, first, flag, s));
  int32_t bad_entry = 0;
  IVF_HIP(hipMemcpyAsync(&bad_entry, flag, 4, hipMemcpyDeviceToHost, s));
  IVF_HIP(hipStreamSynchronize(s));
  if (bad_entry)
    return fail(IVF_ERR_INVALID_ARG, t.copies > 1
                    ? "a list entry names a point outside [0, n) or one in more than copies lists"
                    : "a list entry names a point outside [0, n)");

  ivf_index* idx = new (std::nothrow) ivf_index;
  if (!idx) return fail(IVF_ERR_INTERNAL, "out of host memory");
  idx->t = t;
  idx->layout = lay;
  idx->table_mem = table_mem;
  idx->prof = nullptr;
  idx->graphs = nullptr;
  *out = idx;
  return IVF_OK;
}

ivf_status ivf_get_table_layout(const ivf_index* idx, ivf_table_layout* out) {
  if (!idx || !out) return fail(IVF_ERR_INVALID_ARG, "NULL argument");
  *out = idx->layout;
  return IVF_OK;
}

void ivf_destroy(ivf_index* idx) {
  if (!idx) return;
  delete idx->graphs;
  if (idx->prof) {
    for (auto& row : idx->prof->ev)
      for (auto& e : row)
        if (e) (void)hipEventDestroy(e);
    delete idx->prof;
  }
  delete idx;
}

ivf_status ivf_profile_enable(ivf_index* idx, int32_t on) {
  if (!idx) return fail(IVF_ERR_INVALID_ARG, "index is NULL");
  if (!idx->prof) {
    idx->prof = new (std::nothrow) ivf_profile;
    if (!idx->prof) return fail(IVF_ERR_INTERNAL, "out of host memory");
  }
  idx->prof->on = on != 0;
  idx->prof->cur = -1;
  return IVF_OK;
}

ivf_status ivf_profile_read(ivf_index* idx, float* ms, int32_t* count) {
  if (!idx || !ms || !count) return fail(IVF_ERR_INVALID_ARG, "NULL argument");
  for (int i = 0; i < IVF_NSTAGES; ++i) ms[i] = 0.0f;
  *count = 0;
  ivf_profile* p = idx->prof;
  if (!p || p->count == 0) return IVF_OK;
  const int first = (p->head - p->count + ivf_profile::RING) % ivf_profile::RING;
  int done = 0;
  for (int c = 0; c < p->count; ++c) {
    const int slot = (first + c) % ivf_profile::RING;
    const int n = p->nmarks[slot];
    if (n < 2 || p->stage[slot][n - 1] != IVF_NSTAGES) continue;  // incomplete
    IVF_HIP(hipEventSynchronize(p->ev[slot][n - 1]));
    for (int k = 0; k + 1 < n; ++k) {
      float t = 0.0f;
      IVF_HIP(hipEventElapsedTime(&t, p->ev[slot][k], p->ev[slot][k + 1]));
      const int st = p->stage[slot][k];
      if (st >= 0 && st < IVF_NSTAGES) ms[st] += t;
    }
    ++done;
  }
  *count = done;
  p->count = 0;
  p->cur = -1;
  return IVF_OK;
}

size_t ivf_search_workspace_bytes(const ivf_index* idx, int32_t nq, int32_t max_nprobe,
                                  int32_t k, int32_t rerank, const ivf_search_opts* opts) {
  ivf_search_opts o;
  ivf_default_opts(&o);
  if (opts) o = *opts;
  if (check_opts(o) != IVF_OK) return 0;
  if (check_search(idx, nq, max_nprobe, k, rerank) != IVF_OK) return 0;
  if (o.spill_cap > 16384 - rerank * idx->t.copies) {
    (void)fail(IVF_ERR_INVALID_ARG, "opts.spill_cap must be at most 16384 - rerank * copies");
    return 0;
  }
  return plan_workspace(idx->t, nq, max_nprobe, k, rerank, o, nullptr).total;
}

}  // extern "C"

namespace {

// Stage marks of the current search (no-ops unless profiling is on).
hipError_t prof_begin(const ivf_index* idx) {
  ivf_profile* p = idx->prof;
  if (!p || !p->on) return hipSuccess;
  const int slot = p->head;
  p->head = (p->head + 1) % ivf_profile::RING;
  if (p->count < ivf_profile::RING) ++p->count;
  p->nmarks[slot] = 0;
  p->cur = slot;
  return hipSuccess;
}

// Time from now on counts for `stage`; IVF_NSTAGES ends the search.
hipError_t prof_mark(const ivf_index* idx, hipStream_t s, int stage) {
  ivf_profile* p = idx->prof;
  if (!p || !p->on || p->cur < 0) return hipSuccess;
  const int slot = p->cur;
  const int k = p->nmarks[slot];
  if (k >= ivf_profile::MARKS) return hipSuccess;
  if (!p->ev[slot][k]) {
    hipError_t e = hipEventCreate(&p->ev[slot][k]);
    if (e != hipSuccess) return e;
  }
  p->stage[slot][k] = stage;
  p->nmarks[slot] = k + 1;
  hipError_t e = hipEventRecord(p->ev[slot][k], s);
  if (stage == IVF_NSTAGES) p->cur = -1;  // this search is complete
  return e;
}

// Shared front part of every search entry: validation and workspace carving.
ivf_status begin_search(const ivf_index* idx, int32_t nq, int32_t max_nprobe, int32_t k,
                        int32_t rerank, const ivf_search_opts* opts, void* workspace,
                        size_t workspace_bytes, ivf_search_opts* o, Workspace* w) {
  // `opts` may point at *o: read it before *o is written.
  ivf_search_opts req;
  ivf_default_opts(&req);
  if (opts) req = *opts;
  *o = req;
  ivf_status st = check_opts(*o);
  if (st != IVF_OK) return st;
  st = check_search(idx, nq, max_nprobe, k, rerank);
  if (st != IVF_OK) return st;
  if (idx->prof) idx->prof->cur = -1;  // only entries that call prof_begin are timed
  if (o->spill_cap > 16384 - rerank * idx->t.copies)
    return fail(IVF_ERR_INVALID_ARG, "opts.spill_cap must be at most 16384 - rerank * copies");
  st = check_form(idx, *o);
  if (st != IVF_OK) return st;
  Workspace need = plan_workspace(idx->t, nq, max_nprobe, k, rerank, *o, nullptr);
  if (nq > 0 && !workspace) return fail(IVF_ERR_INVALID_ARG, "workspace is NULL");
  if ((uintptr_t)workspace % ALIGN) return fail(IVF_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (workspace_bytes < need.total) return fail(IVF_ERR_WORKSPACE, "workspace too small");
  *w = plan_workspace(idx->t, nq, max_nprobe, k, rerank, *o, (char*)workspace);
  return IVF_OK;
}

ivf_status run_scan_and_rerank(const ivf_index* idx, const float* Q, const float* Qr, int32_t nq,
                               int32_t max_nprobe, int32_t k, int32_t rerank,
                               const ivf_search_opts& o, const Workspace& w, int64_t* out_ids,
                               float* out_dist, hipStream_t s) {
  const Tables& t = idx->t;
  // The scan keeps `pool` keys of list entries; on a spilled index they are
  // reduced to `rerank` distinct points before the re-rank.
  const int32_t pool = rerank * t.copies;
  IVF_HIP(prof_mark(idx, s, IVF_STAGE_PREP));
  if (!scan_owns_bias(t, max_nprobe)) IVF_HIP(launch_bias(t, Q, nq, max_nprobe, w, s));
  if (o.form == IVF_FORM_BATCHED) {
    // Rounds over probe ranks [b_r, b_{r+1}) with b = 0, 4, 16, 64, ...:
    // each round's merge publishes a tighter threshold for the next.
    const int rounds = o.rounds > 0 ? o.rounds : 1;
    IVF_HIP(launch_batched_first(t, Q, nq, max_nprobe, pool, w, s));
    int lo = 0;
    for (int r = 0; r < rounds; ++r) {
      const int hi = r + 1 == rounds ? max_nprobe : (lo == 0 ? 4 : lo * 4);
      if (r > 0) IVF_HIP(prof_mark(idx, s, IVF_STAGE_PREP));
      IVF_HIP(launch_batched_pairs(t, nq, max_nprobe, lo, hi, w, s));
      IVF_HIP(prof_mark(idx, s, IVF_STAGE_SCAN));
      IVF_HIP(launch_batched_main(t, Q, nq, max_nprobe, pool, w, s));
      IVF_HIP(prof_mark(idx, s, IVF_STAGE_MERGE));
      IVF_HIP(launch_batched_merge(t, nq, pool, w, s));
      lo = hi;
      if (lo >= max_nprobe) break;
    }
    IVF_HIP(launch_batched_redo(t, Q, nq, max_nprobe, pool, w, s));
  } else {
    IVF_HIP(prof_mark(idx, s, IVF_STAGE_SCAN));
    IVF_HIP(launch_scan_plain(t, Q, nq, max_nprobe, pool, w, s));
  }
  if (t.copies > 1) {
    IVF_HIP(prof_mark(idx, s, IVF_STAGE_MERGE));
    IVF_HIP(launch_dedup_pool(t, nq, rerank, w, s));
  }
  IVF_HIP(prof_mark(idx, s, IVF_STAGE_RERANK));
  if (out_ids)
    IVF_HIP(launch_rerank(t, Qr, nq, k, rerank, t.copies > 1 ? w.cand_u : w.cand,
                          o.adaptive ? w.reorder_eff : nullptr, w, out_ids, out_dist, s));
  IVF_HIP(prof_mark(idx, s, IVF_NSTAGES));
  return IVF_OK;
}

// The queries of the search steps: the kept components of a filtered index
// (gathered into the workspace), else the caller's queries.
ivf_status search_queries(const ivf_index* idx, const float* queries, int32_t nq,
                          const Workspace& w, hipStream_t s, const float** out) {
  *out = queries;
  if (!idx->t.dims) return IVF_OK;
  IVF_HIP(launch_gather_queries(idx->t, queries, nq, w.qf, s));
  *out = w.qf;
  return IVF_OK;
}

ivf_status run_coarse(const ivf_index* idx, const float* Q, int32_t nq, const int32_t* nprobe,
                      int32_t max_nprobe, int32_t k, int32_t rerank, const ivf_search_opts& o,
                      const Workspace& w, hipStream_t s) {
  const Tables& t = idx->t;
  const AdaptiveArgs ad{o.adaptive, o.nprobe_init, o.nprobe_min, o.reorder_min, k, rerank,
                        o.p0, o.p1};
  IVF_HIP(prof_mark(idx, s, IVF_STAGE_COARSE));
  if (o.coarse == IVF_COARSE_EXACT) {
    IVF_HIP(launch_coarse_exact(t, Q, nq, w.scores, s));
    IVF_HIP(prof_mark(idx, s, IVF_STAGE_SELECT));
    IVF_HIP(launch_select_probes(t, Q, nq, nprobe, max_nprobe, 1, 0, false, w, s, ad));
  } else {
    IVF_HIP(launch_coarse_mfma(t, Q, nq, o.coarse, w, s));
    IVF_HIP(prof_mark(idx, s, IVF_STAGE_SELECT));
    IVF_HIP(launch_select_probes(t, Q, nq, nprobe, max_nprobe, o.widen, o.widen_add, true, w,
                                 s, ad));
  }
  return IVF_OK;
}

}  // namespace

extern "C" {

ivf_status ivf_search(const ivf_index* idx, const float* queries, int32_t nq,
                      const int32_t* nprobe, int32_t max_nprobe, int32_t k, int32_t rerank,
                      const ivf_search_opts* opts, void* workspace, size_t workspace_bytes,
                      int64_t* out_ids, float* out_dist, void* stream) {
  ivf_search_opts o;
  Workspace w;
  ivf_status st = begin_search(idx, nq, max_nprobe, k, rerank, opts, workspace, workspace_bytes,
                               &o, &w);
  if (st != IVF_OK) return st;
  if (nq == 0) return IVF_OK;
  if (!queries || !nprobe || !out_ids || !out_dist)
    return fail(IVF_ERR_INVALID_ARG, "a required pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (o.use_graph) {
    if (!s) return fail(IVF_ERR_INVALID_ARG, "graph capture needs a non-default stream");
    std::vector<uint64_t> key = {(uint64_t)nq, (uint64_t)max_nprobe, (uint64_t)k,
                                 (uint64_t)rerank, (uint64_t)o.coarse, (uint64_t)o.widen,
                                 (uint64_t)o.widen_add, (uint64_t)o.first_lists,
                                 (uint64_t)o.query_order, (uint64_t)o.list_order,
                                 (uint64_t)o.form, (uint64_t)o.pool_cap, (uint64_t)o.grid,
                                 (uint64_t)o.rounds, (uint64_t)o.spill_cap,
                                 (uint64_t)o.adaptive, (uint64_t)o.nprobe_init,
                                 (uint64_t)o.nprobe_min, (uint64_t)o.reorder_min,
                                 (uint64_t)f32_bits(o.p0), (uint64_t)f32_bits(o.p1),
                                 (uint64_t)(uintptr_t)queries,
                                 (uint64_t)(uintptr_t)nprobe, (uint64_t)(uintptr_t)workspace,
                                 (uint64_t)(uintptr_t)out_ids, (uint64_t)(uintptr_t)out_dist};
    ivf_index* mi = const_cast<ivf_index*>(idx);
    if (!mi->graphs) {
      mi->graphs = new (std::nothrow) ivf_graph_cache;
      if (!mi->graphs) return fail(IVF_ERR_INTERNAL, "out of host memory");
    }
    auto& ents = mi->graphs->entries;
    for (size_t i = 0; i < ents.size(); ++i) {
      if (ents[i].key == key) {
        IVF_HIP(hipGraphLaunch(ents[i].exec, s));
        return IVF_OK;
      }
    }
    ivf_graph_cache::Entry e;
    e.key = key;
    IVF_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    ivf_status cst = IVF_OK;
    const float* Qs = queries;
    if (launch_fill_u32((uint32_t*)w.err, 0u, 4, s) != hipSuccess) cst = IVF_ERR_DEVICE;
    if (cst == IVF_OK) cst = search_queries(idx, queries, nq, w, s, &Qs);
    if (cst == IVF_OK) cst = run_coarse(idx, Qs, nq, nprobe, max_nprobe, k, rerank, o, w, s);
    if (cst == IVF_OK)
      cst = run_scan_and_rerank(idx, Qs, queries, nq, max_nprobe, k, rerank, o, w, out_ids,
                                out_dist, s);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(s, &g);
    if (cst != IVF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return cst;
    }
    if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
    e.graph = g;
    hipError_t ie = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(ie, "hipGraphInstantiate");
    }
    if (ents.size() >= 8) {
      (void)hipGraphExecDestroy(ents.back().exec);
      (void)hipGraphDestroy(ents.back().graph);
      ents.pop_back();
    }
    ents.insert(ents.begin(), e);
    IVF_HIP(hipGraphLaunch(ents.front().exec, s));
    return IVF_OK;
  }
  IVF_HIP(prof_begin(idx));
  IVF_HIP(launch_fill_u32((uint32_t*)w.err, 0u, 4, s));
  const float* Qs = queries;
  st = search_queries(idx, queries, nq, w, s, &Qs);
  if (st != IVF_OK) return st;
  st = run_coarse(idx, Qs, nq, nprobe, max_nprobe, k, rerank, o, w, s);
  if (st != IVF_OK) return st;
  return run_scan_and_rerank(idx, Qs, queries, nq, max_nprobe, k, rerank, o, w, out_ids, out_dist,
                             s);
}

ivf_status ivf_search_static(const ivf_index* idx, const float* queries, int32_t nq,
                             const int32_t* nprobe, int32_t max_nprobe, int32_t k, int32_t rerank,
                             const ivf_search_opts* opts, int64_t* out_ids, float* out_dist,
                             void* stream) {
  ivf_search_opts o;
  ivf_default_opts(&o);
  if (opts) o = *opts;
  ivf_status st = check_opts(o);
  if (st != IVF_OK) return st;
  st = check_search(idx, nq, max_nprobe, k, rerank);
  if (st != IVF_OK) return st;
  if (o.use_graph) return fail(IVF_ERR_INVALID_ARG, "ivf_search_static needs opts.use_graph == 0");
  const int32_t pool = rerank * idx->t.copies;
  if (o.spill_cap > 16384 - pool)
    return fail(IVF_ERR_INVALID_ARG, "opts.spill_cap must be at most 16384 - rerank * copies");
  const size_t cap = IVF_STATIC_SCRATCH_BYTES;
  if (o.form == IVF_FORM_BATCHED && o.spill_cap == 0) {
    // The largest survivor capacity (from the automatic one down to 256
    // keys, in steps of 256) whose workspace fits the scratch.
    int32_t c = batched_spill_cap(pool, nq);
    if (c > 16384 - 256) c = 16384 - 256;  // the range an explicit spill_cap takes
    ivf_search_opts t = o;
    for (;;) {
      t.spill_cap = c;
      if (plan_workspace(idx->t, nq, max_nprobe, k, rerank, t, nullptr).total <= cap || c <= 256)
        break;
      c = c - 256 > 256 ? (c - 1) / 256 * 256 : 256;
    }
    o.spill_cap = c;
  }
  const size_t need = plan_workspace(idx->t, nq, max_nprobe, k, rerank, o, nullptr).total;
  if (need > cap)
    return fail(IVF_ERR_WORKSPACE, "request needs " + std::to_string(need) +
                                       " bytes of workspace; the static scratch holds " +
                                       std::to_string(cap) + " (split the batch)");
  if (nq == 0) return IVF_OK;
  void* ws = nullptr;
  st = static_scratch(&ws);
  if (st != IVF_OK) return st;
  return ivf_search(idx, queries, nq, nprobe, max_nprobe, k, rerank, &o, ws, cap, out_ids,
                    out_dist, stream);
}

ivf_status ivf_search_with_probes(const ivf_index* idx, const float* queries, int32_t nq,
                                  const int32_t* probes, const int32_t* nprobe,
                                  int32_t max_nprobe, int32_t k, int32_t rerank,
                                  const ivf_search_opts* opts, void* workspace,
                                  size_t workspace_bytes, int64_t* out_ids, float* out_dist,
                                  void* stream) {
  ivf_search_opts o;
  Workspace w;
  ivf_status st = begin_search(idx, nq, max_nprobe, k, rerank, opts, workspace, workspace_bytes,
                               &o, &w);
  if (st != IVF_OK) return st;
  if (o.adaptive)
    return fail(IVF_ERR_INVALID_ARG, "opts.adaptive needs the coarse step (use ivf_search)");
  if (nq == 0) return IVF_OK;
  if (!queries || !probes || !nprobe || !out_ids || !out_dist)
    return fail(IVF_ERR_INVALID_ARG, "a required pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  IVF_HIP(prof_begin(idx));
  IVF_HIP(launch_fill_u32((uint32_t*)w.err, 0u, 4, s));
  IVF_HIP(launch_copy_probes(probes, nprobe, nq, max_nprobe, idx->t.L, w, s));
  const float* Qs = queries;
  st = search_queries(idx, queries, nq, w, s, &Qs);
  if (st != IVF_OK) return st;
  return run_scan_and_rerank(idx, Qs, queries, nq, max_nprobe, k, rerank, o, w, out_ids, out_dist,
                             s);
}

ivf_status ivf_debug_probes(const ivf_index* idx, const float* queries, int32_t nq,
                            const int32_t* nprobe, int32_t max_nprobe,
                            const ivf_search_opts* opts, void* workspace, size_t workspace_bytes,
                            int32_t* out_probes, void* stream) {
  ivf_search_opts o;
  Workspace w;
  ivf_status st = begin_search(idx, nq, max_nprobe, 1, 1, opts, workspace, workspace_bytes, &o, &w);
  if (st != IVF_OK) return st;
  if (nq == 0) return IVF_OK;
  if (!queries || !nprobe || !out_probes) return fail(IVF_ERR_INVALID_ARG, "a required pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  IVF_HIP(launch_fill_u32((uint32_t*)w.err, 0u, 4, s));
  const float* Qs = queries;
  st = search_queries(idx, queries, nq, w, s, &Qs);
  if (st != IVF_OK) return st;
  st = run_coarse(idx, Qs, nq, nprobe, max_nprobe, 1, 1, o, w, s);
  if (st != IVF_OK) return st;
  IVF_HIP(hipMemcpyAsync(out_probes, w.probes, (size_t)nq * max_nprobe * 4,
                         hipMemcpyDeviceToDevice, s));
  return IVF_OK;
}

ivf_status ivf_debug_adaptive(const ivf_index* idx, const float* queries, int32_t nq,
                              const int32_t* nprobe, int32_t max_nprobe, int32_t k,
                              int32_t rerank, const ivf_search_opts* opts, void* workspace,
                              size_t workspace_bytes, int32_t* out_nprobe,
                              int32_t* out_reorder, void* stream) {
  ivf_search_opts o;
  Workspace w;
  ivf_status st = begin_search(idx, nq, max_nprobe, k, rerank, opts, workspace, workspace_bytes,
                               &o, &w);
  if (st != IVF_OK) return st;
  if (!o.adaptive) return fail(IVF_ERR_INVALID_ARG, "opts.adaptive must be 1");
  if (nq == 0) return IVF_OK;
  if (!queries || !nprobe || !out_nprobe || !out_reorder)
    return fail(IVF_ERR_INVALID_ARG, "a required pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  IVF_HIP(launch_fill_u32((uint32_t*)w.err, 0u, 4, s));
  const float* Qs = queries;
  st = search_queries(idx, queries, nq, w, s, &Qs);
  if (st != IVF_OK) return st;
  st = run_coarse(idx, Qs, nq, nprobe, max_nprobe, k, rerank, o, w, s);
  if (st != IVF_OK) return st;
  IVF_HIP(hipMemcpyAsync(out_nprobe, w.nprobe_eff, (size_t)nq * 4, hipMemcpyDeviceToDevice, s));
  IVF_HIP(hipMemcpyAsync(out_reorder, w.reorder_eff, (size_t)nq * 4, hipMemcpyDeviceToDevice, s));
  return IVF_OK;
}

ivf_status ivf_debug_coarse_scores(const ivf_index* idx, const float* queries, int32_t nq,
                                   const ivf_search_opts* opts, void* workspace,
                                   size_t workspace_bytes, float* out_scores, void* stream) {
  ivf_search_opts o;
  Workspace w;
  ivf_status st = begin_search(idx, nq, 1, 1, 1, opts, workspace, workspace_bytes, &o, &w);
  if (st != IVF_OK) return st;
  if (o.coarse == IVF_COARSE_EXACT) return fail(IVF_ERR_INVALID_ARG, "opts.coarse must be an MFMA form");
  if (nq == 0) return IVF_OK;
  if (!queries || !out_scores) return fail(IVF_ERR_INVALID_ARG, "a required pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  const float* Qs = queries;
  st = search_queries(idx, queries, nq, w, s, &Qs);
  if (st != IVF_OK) return st;
  IVF_HIP(launch_coarse_mfma(idx->t, Qs, nq, o.coarse, w, s));
  IVF_HIP(hipMemcpyAsync(out_scores, w.scores, (size_t)nq * idx->t.L * 4, hipMemcpyDeviceToDevice, s));
  return IVF_OK;
}

ivf_status ivf_debug_luts(const ivf_index* idx, const float* queries, int32_t nq,
                          const int32_t* probes, const int32_t* nprobe, int32_t max_nprobe,
                          uint8_t* out_lut, float* out_lo, float* out_delta, float* out_B,
                          void* stream) {
  if (!idx) return fail(IVF_ERR_INVALID_ARG, "index is NULL");
  if (nq < 0 || nq > MAX_QUERIES)
    return fail(IVF_ERR_INVALID_ARG, "nq must be in [0, 2^20] per call");
  if (max_nprobe < 1 || max_nprobe > idx->t.L)
    return fail(IVF_ERR_INVALID_ARG, "max_nprobe must be in [1, L]");
  if (nq == 0) return IVF_OK;
  if (!queries || !probes || !nprobe || !out_lut || !out_lo || !out_delta || !out_B)
    return fail(IVF_ERR_INVALID_ARG, "a required pointer is NULL");
  IVF_HIP(launch_debug_luts(idx->t, queries, nq, probes, nprobe, max_nprobe, out_lut, out_lo,
                            out_delta, out_B, (hipStream_t)stream));
  return IVF_OK;
}

ivf_status ivf_debug_batched_luts(const ivf_index* idx, const float* queries, int32_t nq,
                                  const int32_t* probes, const int32_t* nprobe,
                                  int32_t max_nprobe, void* workspace, size_t workspace_bytes,
                                  uint8_t* out_lut, float* out_delta, float* out_B,
                                  void* stream) {
  ivf_search_opts req, o;
  ivf_default_opts(&req);
  req.form = IVF_FORM_BATCHED;
  Workspace w;
  ivf_status st =
      begin_search(idx, nq, max_nprobe, 1, 1, &req, workspace, workspace_bytes, &o, &w);
  if (st != IVF_OK) return st;
  if (!w.qlut && idx->t.metric == IVF_METRIC_IP)
    return fail(IVF_ERR_INTERNAL, "batched workspace plan has no per-query tables");
  if (nq == 0) return IVF_OK;
  if (!queries || !probes || !nprobe || !out_lut || !out_delta || !out_B)
    return fail(IVF_ERR_INVALID_ARG, "a required pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  IVF_HIP(launch_fill_u32((uint32_t*)w.err, 0u, 4, s));
  IVF_HIP(launch_copy_probes(probes, nprobe, nq, max_nprobe, idx->t.L, w, s));
  const float* Qs = queries;
  st = search_queries(idx, queries, nq, w, s, &Qs);
  if (st != IVF_OK) return st;
  IVF_HIP(launch_bias(idx->t, Qs, nq, max_nprobe, w, s));
  IVF_HIP(launch_debug_batched_luts(idx->t, Qs, nq, max_nprobe, w, out_lut, out_delta, out_B, s));
  return IVF_OK;
}

ivf_status ivf_debug_candidates(const ivf_index* idx, const float* queries, int32_t nq,
                                const int32_t* probes, const int32_t* nprobe,
                                int32_t max_nprobe, int32_t rerank, const ivf_search_opts* opts,
                                void* workspace, size_t workspace_bytes, uint64_t* out_keys,
                                void* stream) {
  ivf_search_opts o;
  Workspace w;
  ivf_status st = begin_search(idx, nq, max_nprobe, 1, rerank, opts, workspace, workspace_bytes,
                               &o, &w);
  if (st != IVF_OK) return st;
  if (o.adaptive)
    return fail(IVF_ERR_INVALID_ARG, "opts.adaptive needs the coarse step (use ivf_search)");
  if (nq == 0) return IVF_OK;
  if (!queries || !probes || !nprobe || !out_keys)
    return fail(IVF_ERR_INVALID_ARG, "a required pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  IVF_HIP(launch_fill_u32((uint32_t*)w.err, 0u, 4, s));
  IVF_HIP(launch_copy_probes(probes, nprobe, nq, max_nprobe, idx->t.L, w, s));
  const float* Qs = queries;
  st = search_queries(idx, queries, nq, w, s, &Qs);
  if (st != IVF_OK) return st;
  st = run_scan_and_rerank(idx, Qs, queries, nq, max_nprobe, 1, rerank, o, w, nullptr, nullptr, s);
  if (st != IVF_OK) return st;
  uint64_t* pool = idx->t.copies > 1 ? w.cand_u : w.cand;
  IVF_HIP(launch_sort_rows(pool, nq, rerank, s));
  IVF_HIP(hipMemcpyAsync(out_keys, pool, (size_t)nq * rerank * 8, hipMemcpyDeviceToDevice, s));
  return IVF_OK;
}

}  // extern "C"

namespace {

// Workspace of ivf_assign: centroid operand tables, then per-chunk buffers.
struct AssignPlan {
  Tables t;
  Workspace w;
  int32_t* ones;
  size_t total;
};

AssignPlan plan_assign(int32_t L, int32_t d, int32_t metric, int32_t chunk, int32_t coarse,
                       const float* centroids, char* base) {
  AssignPlan a;
  std::memset(&a, 0, sizeof(a));
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  Tables& t = a.t;
  t.d = d;
  t.d_base = d;
  t.copies = 1;
  t.L = L;
  t.m = 1;
  t.dsub = d;
  t.metric = metric;
  t.L_pad = round_up_i(L, TILE_L);
  t.d_pad = round_up_i(d, TILE_D);
  t.cp = centroids;
  t.cm = centroids;
  t.cp_norm2 = (const float*)take((size_t)t.L_pad * 4);
  t.cp_f32 = (const float*)take((size_t)t.L_pad * t.d_pad * 4);
  t.cp_bf16 = (const uint16_t*)take((size_t)t.L_pad * t.d_pad * 2);
  t.cp_fp8 = (const uint8_t*)take((size_t)t.L_pad * t.d_pad);
  t.cp_fp8_scale = (const float*)take((size_t)t.L_pad * 4);
  Workspace& w = a.w;
  const size_t cp = (size_t)round_up_i(chunk, TILE_L);
  w.err = (int32_t*)take(16);
  w.scores = (float*)take((size_t)chunk * L * 4);
  w.nprobe_eff = (int32_t*)take((size_t)chunk * 4);
  a.ones = (int32_t*)take((size_t)chunk * 4);
  if (coarse != IVF_COARSE_EXACT) {
    w.q_lowp = (void*)take(cp * t.d_pad * 4);
    w.q_scale = (float*)take(cp * 4);
  }
  a.total = off;
  return a;
}

}  // namespace

extern "C" {

size_t ivf_assign_workspace_bytes(int32_t L, int32_t d, int32_t chunk, int32_t coarse) {
  if (L < 1 || L > 16384 || d < 1 || chunk < 1 || chunk > (1 << 20) || coarse < 0 ||
      coarse > IVF_COARSE_FP8) {
    g_last_error = "invalid assign sizes";
    return 0;
  }
  return plan_assign(L, d, IVF_METRIC_L2, chunk, coarse, nullptr, nullptr).total;
}

ivf_status ivf_assign(const float* centroids, int32_t L, int32_t d, int32_t metric,
                      const float* X, int64_t n, int32_t chunk, int32_t coarse, int32_t widen,
                      void* workspace, size_t workspace_bytes, int32_t* out_list, void* stream) {
  if (L < 1 || L > 16384 || d < 1 || n < 0 || chunk < 1 || chunk > (1 << 20))
    return fail(IVF_ERR_INVALID_ARG, "invalid assign sizes");
  if (metric != IVF_METRIC_L2 && metric != IVF_METRIC_IP) return fail(IVF_ERR_INVALID_ARG, "unknown metric");
  if (coarse < IVF_COARSE_EXACT || coarse > IVF_COARSE_FP8 || widen < 1 || widen > MAX_WIDEN)
    return fail(IVF_ERR_INVALID_ARG, "invalid coarse form or widen (1..16384)");
  if (n == 0) return IVF_OK;
  if (!centroids || !X || !out_list || !workspace) return fail(IVF_ERR_INVALID_ARG, "a required pointer is NULL");
  if ((uintptr_t)workspace % ALIGN) return fail(IVF_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  AssignPlan a = plan_assign(L, d, metric, chunk, coarse, centroids, (char*)workspace);
  if (workspace_bytes < a.total) return fail(IVF_ERR_WORKSPACE, "workspace too small");
  ivf_status st = check_device();
  if (st != IVF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  IVF_HIP(launch_aux_tables(a.t, s));
  IVF_HIP(launch_fill_u32((uint32_t*)a.ones, 1u, (size_t)chunk, s));
  IVF_HIP(launch_fill_u32((uint32_t*)a.w.err, 0u, 4, s));
  for (int64_t r0 = 0; r0 < n; r0 += chunk) {
    const int32_t rows = (int32_t)((n - r0) < chunk ? (n - r0) : chunk);
    const float* Xc = X + r0 * d;
    Workspace w = a.w;
    w.probes = out_list + r0;  // max_nprobe = 1: one list per row
    if (coarse == IVF_COARSE_EXACT) {
      IVF_HIP(launch_coarse_exact(a.t, Xc, rows, w.scores, s));
      IVF_HIP(launch_select_probes(a.t, Xc, rows, a.ones, 1, 1, 0, false, w, s));
    } else {
      IVF_HIP(launch_coarse_mfma(a.t, Xc, rows, coarse, w, s));
      IVF_HIP(launch_select_probes(a.t, Xc, rows, a.ones, 1, widen, 0, true, w, s));
    }
  }
  return IVF_OK;
}

size_t ivf_assign_spill_workspace_bytes(int32_t L, int32_t d, int32_t chunk) {
  if (L < 2 || L > 16384 || d < 1 || chunk < 1 || chunk > (1 << 20)) {
    g_last_error = "invalid spill-assign sizes";
    return 0;
  }
  return plan_assign(L, d, IVF_METRIC_L2, chunk, IVF_COARSE_EXACT, nullptr, nullptr).total;
}

ivf_status ivf_assign_spill(const float* centroids, int32_t L, int32_t d, const float* X,
                            int64_t n, const int32_t* primary, float lam, int32_t chunk,
                            void* workspace, size_t workspace_bytes, int32_t* out_list,
                            void* stream) {
  if (L < 2 || L > 16384 || d < 1 || n < 0 || chunk < 1 || chunk > (1 << 20))
    return fail(IVF_ERR_INVALID_ARG, "invalid spill-assign sizes");
  if (!std::isfinite(lam) || lam < 0.0f) return fail(IVF_ERR_INVALID_ARG, "lam must be finite and >= 0");
  if (n == 0) return IVF_OK;
  if (!centroids || !X || !primary || !out_list || !workspace)
    return fail(IVF_ERR_INVALID_ARG, "a required pointer is NULL");
  if ((uintptr_t)workspace % ALIGN) return fail(IVF_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  // The exact-coarse assign layout: scores [chunk][L] hold the losses, the
  // top-1 selection over them picks the spill list.
  AssignPlan a = plan_assign(L, d, IVF_METRIC_L2, chunk, IVF_COARSE_EXACT, centroids,
                             (char*)workspace);
  if (workspace_bytes < a.total) return fail(IVF_ERR_WORKSPACE, "workspace too small");
  ivf_status st = check_device();
  if (st != IVF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  IVF_HIP(launch_fill_u32((uint32_t*)a.ones, 1u, (size_t)chunk, s));
  IVF_HIP(launch_fill_u32((uint32_t*)a.w.err, 0u, 4, s));
  for (int64_t r0 = 0; r0 < n; r0 += chunk) {
    const int32_t rows = (int32_t)((n - r0) < chunk ? (n - r0) : chunk);
    Workspace w = a.w;
    w.probes = out_list + r0;
    IVF_HIP(launch_spill_loss(X + r0 * d, rows, d, centroids, L, primary + r0, lam, w.scores, s));
    IVF_HIP(launch_select_probes(a.t, X + r0 * d, rows, a.ones, 1, 1, 0, false, w, s));
    IVF_HIP(launch_spill_fix(primary + r0, rows, L, out_list + r0, s));
  }
  return IVF_OK;
}

ivf_status ivf_encode(const float* X, int64_t n, int32_t d, const float* centroids,
                      const int32_t* lists, const float* codebooks, int32_t m,
                      uint8_t* out_codes, void* stream) {
  if (n < 0 || d < 1 || m < 1 || m > MAX_M || d % m != 0)
    return fail(IVF_ERR_INVALID_ARG, "invalid encode sizes");
  if (n == 0) return IVF_OK;
  if (!X || !centroids || !lists || !codebooks || !out_codes)
    return fail(IVF_ERR_INVALID_ARG, "a required pointer is NULL");
  ivf_status st = check_device();
  if (st != IVF_OK) return st;
  IVF_HIP(launch_encode(X, n, d, m, centroids, lists, codebooks, out_codes, (hipStream_t)stream));
  return IVF_OK;
}

ivf_status ivf_get_device_error(const ivf_index* idx, void* workspace, int32_t* out_mask,
                                void* stream) {
  if (out_mask) *out_mask = 0;
  if (!idx || !workspace || !out_mask) return fail(IVF_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  int32_t v[4] = {0, 0, 0, 0};
  // The error word is the first 16 bytes of every workspace layout.
  IVF_HIP(hipMemcpyAsync(v, workspace, 16, hipMemcpyDeviceToHost, s));
  IVF_HIP(hipStreamSynchronize(s));
  IVF_HIP(launch_fill_u32((uint32_t*)workspace, 0u, 4, s));
  *out_mask = v[0];
  return IVF_OK;
}

}  // extern "C"
