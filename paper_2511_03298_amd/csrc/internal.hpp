// Host-side structures shared by the ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ivf.h"

namespace ivf {

constexpr int KSUB = 16;          // codewords per subspace (4-bit codes)
constexpr int BLOCK_PTS = 64;     // points per packed block (one wavefront)
constexpr int MAX_M = 256;
constexpr int MAX_RERANK = 2048;
constexpr int MAX_QUERIES = 1 << 20;  // queries per search call
constexpr int MAX_L = 1 << 20;
constexpr int TILE_L = 64;        // low-precision centroid tables: L padded to this
constexpr int TILE_D = 64;        // ... and d padded to this
constexpr size_t ALIGN = 256;
constexpr int ORDER_BUCKETS = 1024;  // scan-length buckets of the longest-first query order
constexpr int MAX_SCAN_LISTS = 16384;  // lists of an index that can be searched

inline size_t align_up(size_t x, size_t a = ALIGN) { return (x + a - 1) / a * a; }

// Device view of a built index (pointers into caller-owned table memory).
struct Tables {
  int64_t n;
  int32_t d, L, m, dsub, metric, base_dtype;
  int32_t words;      // 32-bit code words per point = m_pad / 8
  int32_t m_pad;      // m rounded up to a multiple of 8
  int32_t blocks;     // total 64-point blocks
  int32_t L_pad, d_pad;
  int32_t max_list_len;
  int32_t d_base;               // row width of base / queries (>= d)
  int32_t copies;               // most lists one point lies in (spilled index: >= 2)
  const int32_t* dims;          // [d] kept base columns, or nullptr
  const void* base;
  const uint32_t* codes;        // [blocks][words][64]
  const int32_t* slot_ids;      // [blocks][64]
  const int32_t* block_off;     // [L+1]
  const int32_t* list_len;      // [L]
  const int32_t* list_order;    // [L] list indices by length, longest first (ties by index)
  const float* cm;              // [L][d]
  const float* cp;              // [L][d]
  const float* codebooks;       // [m_pad][16][dsub]
  const float* cp_norm2;        // [L_pad]
  const float* cp_f32;          // [L_pad][d_pad]
  const uint16_t* cp_bf16;      // [L_pad][d_pad]
  const uint8_t* cp_fp8;        // [L_pad][d_pad]
  const float* cp_fp8_scale;    // [L_pad]
};

}  // namespace ivf

struct ivf_profile;      // per-stage event ring, see abi.cpp
struct ivf_graph_cache;  // captured searches, see abi.cpp

struct ivf_index {
  ivf::Tables t;
  ivf_table_layout layout;
  void* table_mem;
  ivf_profile* prof;
  ivf_graph_cache* graphs;
};

namespace ivf {

// ---- workspace for one search -------------------------------------------
struct Workspace {
  float* scores;        // [nq][L] coarse scores (exact or approximate)
  int32_t* probes;      // [nq][max_nprobe]
  int32_t* nprobe_eff;  // [nq]; -1 marks an invalid request
  int32_t* reorder_eff; // [nq] re-rank size (adaptive form; else rerank)
  float* qf;            // [nq][d] kept query components (filtered index only)
  float* bias;          // [nq][max_nprobe] per-(q,list) constant (IP), else unused
  uint64_t* cand;       // [nq][rerank * copies] scan pool (keys of list entries)
  uint64_t* cand_u;     // [nq][rerank] one key per point (spilled index only)
  int32_t* err;         // [4] device error word
  int32_t* order;       // [nq] launch order of the per-query scans, longest first
  int32_t* order_bucket;  // [nq] scan-length bucket of each query
  int32_t* order_hist;  // [2 * ORDER_BUCKETS] bucket counts, then bucket cursors
  // batched form
  int32_t* p1;          // [nq] first probe slot of phase 2
  uint64_t* thr;        // [nq] phase-1 threshold keys
  int32_t* list_cnt;    // [L] phase-2 pairs per list
  int32_t* list_cursor; // [L]
  int32_t* list_start;  // [L+1]
  int32_t* item_start;  // [L+1]
  int32_t* item_list;   // [nq*max_nprobe] list of each work item
  int32_t* pairs;       // [nq*max_nprobe][2] (query, probe slot) grouped by list
  uint32_t* queue;      // [1] work-queue counter
  int32_t* spill_cnt;   // [nq] survivors per query
  uint64_t* spill;      // [nq][spill_cap] survivors
  int32_t* redo;        // [nq] 1 = survivors overflowed, recompute
  uint8_t* qlut;        // IP: [nq][16][m_pad] per-query u8 tables (code-major)
  float* qlo_sum;       // IP: [nq] pairwise sum of the subspace minima
  float* qdelta;        // IP: [nq] quantisation step
  void* q_lowp;         // [nq_pad][d_pad] queries converted for MFMA coarse
  float* q_scale;       // [nq_pad]
  size_t total;
  int32_t spill_cap;
  int32_t pool_cap;  // plain scan candidate buffer beyond R (0 = auto)
  int32_t grid;      // batched workgroups per CU (0 = auto)
  int32_t first_lists;  // batched first-list pass: lists scanned at least (>= 1)
  int32_t query_order;  // 0: per-query scans longest first; 1: query index order
  int32_t list_order;   // 0: batched work items of the longest lists first; 1: list order
};

int32_t batched_spill_cap(int32_t rerank, int32_t nq);

Workspace plan_workspace(const Tables& t, int32_t nq, int32_t max_nprobe, int32_t k,
                         int32_t rerank, const ivf_search_opts& o, char* base);

// ---- launchers (each enqueues on `s`, returns hipSuccess or an error) ----
// flag[0] is set to 1 when a list entry names a point outside [0, n).
hipError_t launch_pack(const Tables& t, const uint8_t* codes, const int64_t* list_off_dev,
                       const int32_t* list_ids, int32_t* flag, hipStream_t s);
// Spilled index: slot values id * copies + c (see tables.hip); first [n] and
// flag [1] are scratch, flag[0] = 1 when a point lies in too many lists.
hipError_t launch_number_copies(const Tables& t, int32_t* first, int32_t* flag, hipStream_t s);
hipError_t launch_aux_tables(const Tables& t, hipStream_t s);

hipError_t launch_coarse_exact(const Tables& t, const float* Q, int32_t nq, float* scores,
                               hipStream_t s);
hipError_t launch_coarse_mfma(const Tables& t, const float* Q, int32_t nq, int coarse,
                              const Workspace& w, hipStream_t s);
// Select per query the min(L, nprobe[q]*widen + widen_add) best lists of
// `scores` and, when the scores are approximate (`rescore`), re-score them
// canonically and keep the nprobe[q] best. Writes probes / nprobe_eff; with `ad.on`, the
// adaptive probe count and re-rank size of Eq. 2 (reorder_eff).
struct AdaptiveArgs {
  int32_t on, nprobe_init, nprobe_min, reorder_min, k, R;
  float p0, p1;
};
hipError_t launch_select_probes(const Tables& t, const float* Q, int32_t nq,
                                const int32_t* nprobe, int32_t max_nprobe, int32_t widen,
                                int32_t widen_add, bool rescore, const Workspace& w, hipStream_t s,
                                const AdaptiveArgs& ad = AdaptiveArgs{});
hipError_t launch_copy_probes(const int32_t* probes, const int32_t* nprobe, int32_t nq,
                              int32_t max_nprobe, int32_t L, const Workspace& w,
                              hipStream_t s);
hipError_t launch_gather_queries(const Tables& t, const float* Q, int32_t nq, float* qf,
                                 hipStream_t s);
hipError_t launch_bias(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                       const Workspace& w, hipStream_t s);
// Inner product with probe rows of at most 1024 slots: the scan kernel (plain
// form, first-list pass) computes the list constants itself, so the search
// needs no launch_bias.
inline bool scan_owns_bias(const Tables& t, int32_t max_nprobe) {
  return t.metric == IVF_METRIC_IP && max_nprobe <= 1024;
}
hipError_t launch_scan_plain(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                             int32_t rerank, const Workspace& w, hipStream_t s);
// Batched form: first-list pass (pool + threshold per query), then per
// round: work list for probe ranks [lo, hi), persistent list-major scan,
// merge (new pool and threshold); finally the plain recompute of queries
// whose survivors overflowed.
hipError_t launch_batched_first(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                                int32_t rerank, const Workspace& w, hipStream_t s);
hipError_t launch_batched_pairs(const Tables& t, int32_t nq, int32_t max_nprobe, int32_t lo,
                                int32_t hi, const Workspace& w, hipStream_t s);
hipError_t launch_batched_main(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                               int32_t rerank, const Workspace& w, hipStream_t s);
hipError_t launch_batched_merge(const Tables& t, int32_t nq, int32_t rerank, const Workspace& w,
                                hipStream_t s);
hipError_t launch_batched_redo(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                               int32_t rerank, const Workspace& w, hipStream_t s);
hipError_t launch_debug_luts(const Tables& t, const float* Q, int32_t nq, const int32_t* probes,
                             const int32_t* nprobe, int32_t max_nprobe, uint8_t* out_lut, float* out_lo, float* out_delta, float* out_B,
                             hipStream_t s);
// Batched form's tables per (q, p < nprobe_eff[q]) of w.probes, from the
// builders the batched scan uses: out_lut [nq][max_nprobe][m][16] u8,
// out_delta / out_B [nq][max_nprobe]. Needs w.bias for inner product.
hipError_t launch_debug_batched_luts(const Tables& t, const float* Q, int32_t nq,
                                     int32_t max_nprobe, const Workspace& w, uint8_t* out_lut,
                                     float* out_delta, float* out_B, hipStream_t s);
// pool: [nq][rerank] keys with point ids in their low 32 bits; reorder:
// per-query re-rank sizes (<= rerank) or nullptr for all of them.
hipError_t launch_rerank(const Tables& t, const float* Q, int32_t nq, int32_t k, int32_t rerank,
                         const uint64_t* pool, const int32_t* reorder,
                         const Workspace& w, int64_t* out_ids, float* out_dist, hipStream_t s);
// Spilled index: from the [nq][rerank * copies] entry keys of w.cand, each
// point once at its smallest key, the rerank smallest into w.cand_u.
hipError_t launch_dedup_pool(const Tables& t, int32_t nq, int32_t rerank, const Workspace& w,
                             hipStream_t s);
// SOAR spill loss of rows X [rows][d] against every list (canonical FP32;
// +inf for the row's primary list) into loss [rows][L].
hipError_t launch_spill_loss(const float* X, int32_t rows, int32_t d, const float* C, int32_t L,
                             const int32_t* primary, float lam, float* loss, hipStream_t s);
hipError_t launch_spill_fix(const int32_t* primary, int32_t rows, int32_t L, int32_t* out,
                            hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_sort_rows(uint64_t* cand, int32_t nq, int32_t R, hipStream_t s);
hipError_t launch_encode(const float* X, int64_t n, int32_t d, int32_t m, const float* cm,
                         const int32_t* lists, const float* codebooks, uint8_t* codes,
                         hipStream_t s);

}  // namespace ivf
