/*
 * ivf.h -- C ABI of the MI355X (gfx950) IVF-PQ search path.
 *
 * The library answers the k-nearest-neighbour problem of the paper's
 * introduction (the k points of X closest to a query under a metric)
 * approximately, with the partition-based pipeline of section 4.1 and the
 * search procedure of Alg. 2 (static nprobe / reorder, brute-force branch of
 * Alg. 3):
 *   1. coarse scores of every query against the list centroids and the
 *      nprobe nearest lists (TopNClusters);
 *   2. per probed list a lookup table of Eq. (1) on the residual query,
 *      quantised to 8-bit entries (sections 2.4, 2.5, 4.5);
 *   3. the ADC scan of the probed lists' 4-bit codes;
 *   4. the `reorder` (= rerank) best candidates per query (UpdateNNPool);
 *   5. exact FP32 re-ranking of those candidates and the top k.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers unless marked "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     every call only enqueues work on it and returns, unless noted.
 *   - The library never allocates device memory. Table memory and search
 *     workspace are sized by the *_bytes queries and owned by the caller
 *     (ivf_search_static instead uses a fixed array of the code object).
 *   - Host-side validation happens before anything is enqueued: on a non-OK
 *     status nothing was written and ivf_last_error() describes the problem.
 *     No exception crosses this boundary and the library never aborts.
 *   - Sharing: searches never write the table memory, so searches of one
 *     index may be in flight on several streams at once, each with its own
 *     workspace (a workspace serves one search at a time). The host handle is
 *     not locked: the graph cache (use_graph) and the profiling ring live in
 *     it, so calls on one index from several host threads must be serialised
 *     by the caller, and ivf_destroy must follow the last of them.
 *   - Distances: IVF_METRIC_L2 returns squared Euclidean distances, ascending;
 *     IVF_METRIC_IP returns inner products, descending. Ties are broken by
 *     the smaller id at every selection step.
 */
#ifndef IVFPQ_IVF_H
#define IVFPQ_IVF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ivf_index ivf_index; /* opaque host handle */

typedef enum {
  IVF_OK = 0,
  IVF_ERR_INVALID_ARG = 1, /* bad size, pointer, enum or combination       */
  IVF_ERR_DEVICE = 2,      /* no usable gfx950 device, or a HIP call failed */
  IVF_ERR_WORKSPACE = 3,   /* table memory or workspace too small          */
  IVF_ERR_UNSUPPORTED = 4, /* valid request the library does not implement */
  IVF_ERR_INTERNAL = 5
} ivf_status;

typedef enum { IVF_METRIC_L2 = 0, IVF_METRIC_IP = 1 } ivf_metric;
/* Raw-row storage for the re-rank. BF16 and U8 (byte vectors such as SIFT /
 * BIGANN) are widened to FP32 exactly; the distances are then FP32 sums. */
typedef enum { IVF_DTYPE_F32 = 0, IVF_DTYPE_BF16 = 1, IVF_DTYPE_U8 = 2 } ivf_dtype;

/* A trained IVF + residual-PQ index (Alg. 1 outputs), K = 16 codewords per
 * subspace (4-bit codes). Sizes: 1 <= d, 1 <= m <= 256, d % m == 0,
 * 1 <= L, 1 <= n < 2^31. */
typedef struct {
  int64_t n;                      /* number of base vectors                        */
  int32_t d;                      /* dimension                                     */
  int32_t L;                      /* number of inverted lists                      */
  int32_t m;                      /* PQ subspaces, d' = d / m                      */
  int32_t metric;                 /* ivf_metric                                    */
  int32_t base_dtype;             /* ivf_dtype of `base`                           */
  const void* base;               /* [n,d] row-major raw rows for the re-rank.
                                     Referenced, not copied: must outlive searches */
  const float* centroids;         /* [L,d] arithmetic-mean centroids: the residual
                                     origin (section 4.6.1). Copied.              */
  const float* probe_centroids;   /* [L,d] centroids used to select lists, or NULL
                                     (= centroids). For IP pass the normalised
                                     centroids (section 4.6.1). Copied.           */
  const float* codebooks;         /* [m,16,d'] PQ codewords of the residuals.
                                     Copied.                                      */
  const uint8_t* codes;           /* one 4-bit code (0..15) per byte: [n,m], row =
                                     point id; with copies >= 2 [list_offsets[L],m],
                                     row = list entry (the residual to that entry's
                                     list). Consumed: packed into the tables.     */
  const int64_t* list_offsets;    /* HOST [L+1] CSR offsets into list_ids,
                                     non-decreasing, list_offsets[0] == 0 and
                                     list_offsets[L] <= n * copies (rows in no
                                     list are never returned).                    */
  const int32_t* list_ids;        /* [list_offsets[L]] point ids (rows of base)
                                     grouped by list, ascending within a list; a
                                     point lies in at most `copies` lists.
                                     Consumed.                                    */
  int32_t d_base;                 /* row width of `base` and of the queries the
                                     searches take: d, or 0 (= d) when dims is
                                     NULL; >= d otherwise                          */
  const int32_t* dims;            /* HOST [d] or NULL. Component filtration
                                     (section 4.3, Alg. 1/2): the index (centroids,
                                     codebooks, codes) lives in the base columns
                                     dims[0..d), strictly ascending, < d_base.
                                     Steps 1-4 use those components of each query,
                                     the re-rank the full d_base-wide query and
                                     rows. Copied.                                 */
  int32_t copies;                 /* Spilled assignment (section 4.6.2, SOAR): the
                                     most lists one point lies in, 1..4 (0 = 1).
                                     With copies >= 2 a point scanned in several
                                     probed lists enters the candidate pool once,
                                     at the smallest of its approximate distances;
                                     n * copies < 2^31 and rerank * copies <= 2048.
                                     ivf_build_tables fails with
                                     IVF_ERR_INVALID_ARG when a point lies in more
                                     lists.                                       */
} ivf_index_desc;

/* Coarse-scoring precision (step 1). IVF_COARSE_EXACT scores every list with
 * the canonical FP32 formula on the vector ALUs. The MFMA forms compute an
 * approximate score matrix (FP32, BF16, or FP8 e4m3 with per-row scales, all
 * with FP32 accumulation), keep the widen*nprobe + widen_add best lists,
 * re-score those with the canonical FP32 formula and keep the nprobe best. */
typedef enum {
  IVF_COARSE_EXACT = 0,
  IVF_COARSE_F32 = 1,
  IVF_COARSE_BF16 = 2,
  IVF_COARSE_FP8 = 3
} ivf_coarse;

/* Scan schedule (steps 2-4). PLAIN: one workgroup per query walks its probed
 * lists in coarse order. BATCHED: persistent workgroups pull (query, list
 * chunk) items from a device work queue. Both give identical results. */
typedef enum { IVF_FORM_PLAIN = 0, IVF_FORM_BATCHED = 1 } ivf_form;

typedef struct {
  int32_t coarse;    /* ivf_coarse                                              */
  int32_t widen;     /* 1..16384; MFMA coarse forms keep min(L, widen*nprobe
                        + widen_add) lists before the canonical re-score
                        (ignored by IVF_COARSE_EXACT)                         */
  int32_t form;      /* ivf_form                                                */
  int32_t use_graph; /* 1 = capture the whole search into a hipGraph on first
                        use with these exact arguments (sizes, options and
                        every pointer) and replay it afterwards; needs a
                        non-default stream. Up to 8 graphs are cached per
                        index; per-stage profiling does not see replays.     */
  int32_t pool_cap;  /* plain scan (and the batched form's first-list pass):
                        candidate buffer beyond R, in keys, multiple of 256,
                        256..16384; 0 = auto. Larger = fewer pool reductions,
                        more LDS per workgroup                                */
  int32_t grid;      /* BATCHED: persistent workgroups per compute unit, 0..8;
                        0 = auto (from the kernel's LDS footprint)            */
  int32_t rounds;    /* BATCHED: list-major rounds over probe ranks [0,4),
                        [4,16), [16,64), ... (the last takes the rest), each
                        ending with a merge that tightens the per-query
                        threshold; 1..8, 0 = auto (1)                         */
  int32_t spill_cap; /* BATCHED: survivor keys kept per query and round; a
                        query with more is recomputed by the plain scan.
                        0 = auto (a 2 GiB buffer for the batch, at most
                        16384 - rerank), else 256..16384 - rerank            */
  /* Adaptive probing depth and re-rank size (section 4.2, Eq. 2), computed
   * on the device after step 1 (ivf_search only). The paper's trained
   * easy/hard classifier is replaced by a closed form of its centroid-
   * distance feature: with the coarse scores s_1 <= s_2 <= ... of the query,
   * e = s (L2) or 1 + s (IP), p = e_1 / e_K clamped to [0, 1] (1 when
   * e_K <= 0), K = min(nprobe_init, nprobe[q]). Then, in FP32,
   * g = max(p - p0, 0) * (p + p1) and
   *   nprobe_q  = min(nprobe[q], n_min + floor((nprobe[q] - n_min) * g)),
   *               n_min = clamp(nprobe_min, 1, nprobe[q]);
   *   reorder_q = min(rerank,   r_min + floor((rerank - r_min) * g)),
   *               r_min = clamp(reorder_min, k, rerank).
   * The candidate pool still keeps the rerank best keys; the re-rank uses
   * the reorder_q best of them (the set a pool of that size would hold). */
  int32_t adaptive;    /* 0 or 1                                              */
  int32_t nprobe_init; /* K >= 1                                              */
  int32_t nprobe_min;  /* >= 1                                                */
  int32_t reorder_min; /* >= 1                                                */
  float p0, p1;        /* finite                                              */
  int32_t widen_add;   /* 0..16384: MFMA coarse forms keep min(L, widen*nprobe
                          + widen_add) lists for the canonical re-score (an
                          additive margin: the approximate scores only misorder
                          lists near the cut)                                  */
  int32_t first_lists; /* BATCHED: the first-list pass, whose pool's largest
                          key is the first threshold of the rounds, scans each
                          query's nearest lists in coarse order: at least
                          first_lists of them, and on until it has seen
                          rerank*copies points. 1..64, 0 = auto (4). More
                          lists: a tighter first threshold (fewer survivors to
                          merge) for more per-query scanning.                 */
  int32_t query_order; /* launch order of the one-workgroup-per-query scans
                          (plain form, first-list pass): 0 = longest scan
                          first (queries bucketed by the points they will
                          visit), 1 = query index order. Results are the same;
                          longest-first ends the grid evenly when scan lengths
                          vary across queries.                                 */
  int32_t list_order;  /* BATCHED: order of the work items on the queue: 0 =
                          longest list first, 1 = list index order. Results
                          are the same.                                        */
} ivf_search_opts;

/* Entry points without a passage of the paper behind them are marked
 * "Infrastructure": sizing, layout inspection, error reporting and
 * profiling that any caller of the path above needs. */

/* Defaults: EXACT coarse, widen 2, PLAIN form, no graph, auto pool and grid.
 * Infrastructure. */
void ivf_default_opts(ivf_search_opts* opts);

/* Bytes of device memory ivf_build_tables needs for this index; 0 if the
 * descriptor is invalid (see ivf_last_error). Host only, no device work.
 * Infrastructure. */
size_t ivf_tables_bytes(const ivf_index_desc* desc);

/* Lay out the index in `table_mem` (>= ivf_tables_bytes, 256-byte aligned):
 * packed 4-bit code blocks per list (step 3 operand), slot ids, centroid
 * copies and low-precision centroid tables. Synchronises `stream` before it
 * returns, so the descriptor's arrays may be freed afterwards (except base).
 * A list_ids entry outside [0, n) (or, with copies >= 2, a point in more
 * lists) is found on the device and reported as IVF_ERR_INVALID_ARG.
 * On success *out receives a host handle that references table_mem. */
ivf_status ivf_build_tables(const ivf_index_desc* desc, void* table_mem,
                            size_t table_bytes, void* stream, ivf_index** out);

/* Bytes of workspace one ivf_search call with these sizes needs; 0 if the
 * arguments are invalid. max_nprobe bounds every nprobe[q]. Every search
 * entry point takes 0 <= nq <= 2^20 queries per call (larger batches are
 * split by the caller), as the assignment calls take at most 2^20 rows.
 * Infrastructure. */
size_t ivf_search_workspace_bytes(const ivf_index* idx, int32_t nq,
                                  int32_t max_nprobe, int32_t k,
                                  int32_t rerank, const ivf_search_opts* opts);

/* Search nq queries (Alg. 2 with static parameters). On a spilled index
 * (copies >= 2) the scan keeps the rerank * copies best (distance, copy)
 * keys, which hold the rerank best distinct points, and the pool keeps each
 * of those once at its best copy before the re-rank.
 *   queries  [nq,d] FP32 row-major.
 *   nprobe   [nq] int32, each in 1..max_nprobe (max_nprobe <= L). A value out
 *            of range sets the device error word (ivf_get_device_error) and
 *            that query's row is written as ids -1, distances NaN.
 *   k        1..rerank; rerank (reorder) 1..2048 candidates re-ranked exactly.
 *   out_ids  [nq,k] int64 point ids, -1 when fewer than k candidates exist.
 *   out_dist [nq,k] FP32; padding is +inf (L2) or -inf (IP).
 * opts NULL = defaults. The workspace must hold ivf_search_workspace_bytes. */
ivf_status ivf_search(const ivf_index* idx, const float* queries, int32_t nq,
                      const int32_t* nprobe, int32_t max_nprobe, int32_t k,
                      int32_t rerank, const ivf_search_opts* opts,
                      void* workspace, size_t workspace_bytes,
                      int64_t* out_ids, float* out_dist, void* stream);

/* Steps 2-5 on caller-given probe sets: probes [nq,max_nprobe] int32 list
 * indices in visiting order, nprobe [nq] how many of each row are used. The
 * first nprobe[q] entries of a row must be distinct lists in [0, L) (the
 * probe set of Alg. 2 is a set of clusters); a row that breaks this sets
 * bit 2 of the device error word and is answered as an invalid nprobe is
 * (ids -1, distances NaN). Same outputs and workspace as ivf_search. */
ivf_status ivf_search_with_probes(const ivf_index* idx, const float* queries,
                                  int32_t nq, const int32_t* probes,
                                  const int32_t* nprobe, int32_t max_nprobe,
                                  int32_t k, int32_t rerank,
                                  const ivf_search_opts* opts, void* workspace,
                                  size_t workspace_bytes, int64_t* out_ids,
                                  float* out_dist, void* stream);

/* Bytes of the library's static scratch array (one per device). */
#define IVF_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* ivf_search without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, hosts that
 * forbid hipMalloc). The workspace is a file-scope device array of
 * IVF_STATIC_SCRATCH_BYTES in the library's code object: every device holds
 * its own copy from the first call on it until the process ends, and this
 * call neither allocates nor frees device memory. Same arguments (minus the
 * workspace), outputs and validation as ivf_search, with these limits:
 *   - a request whose workspace (ivf_search_workspace_bytes) exceeds
 *     IVF_STATIC_SCRATCH_BYTES fails with IVF_ERR_WORKSPACE before any work
 *     is enqueued: split the batch. With the BATCHED form and spill_cap 0 the
 *     survivor capacity is the largest one (at most the automatic one,
 *     at least 256 keys) that fits; results do not depend on it;
 *   - opts->use_graph must be 0 (the caller may capture the call itself);
 *   - the scratch is shared by every call on one device and keeps the last
 *     call's contents (each search clears what it needs): calls that overlap
 *     on one device, on different streams or host threads, race. Serialise
 *     them, e.g. on one stream.
 * The device is the current one (hipGetDevice), which must be the device of
 * idx's table memory. */
ivf_status ivf_search_static(const ivf_index* idx, const float* queries,
                             int32_t nq, const int32_t* nprobe,
                             int32_t max_nprobe, int32_t k, int32_t rerank,
                             const ivf_search_opts* opts, int64_t* out_ids,
                             float* out_dist, void* stream);

/* Step 1 only: out_probes [nq,max_nprobe] int32 list indices ordered by
 * (canonical score, list index); entries past the query's probe count
 * (nprobe[q], or the adaptive choice with opts->adaptive) are -1. */
ivf_status ivf_debug_probes(const ivf_index* idx, const float* queries,
                            int32_t nq, const int32_t* nprobe,
                            int32_t max_nprobe, const ivf_search_opts* opts,
                            void* workspace, size_t workspace_bytes,
                            int32_t* out_probes, void* stream);

/* Adaptive choice only (opts->adaptive = 1, section 4.2): per query the
 * probe count and re-rank size ivf_search would use with these arguments,
 * out_nprobe [nq] and out_reorder [nq] int32 (device); -1 for an invalid
 * nprobe[q]. The workspace is sized by ivf_search_workspace_bytes for the
 * same (nq, max_nprobe, k, rerank, opts). */
ivf_status ivf_debug_adaptive(const ivf_index* idx, const float* queries, int32_t nq,
                              const int32_t* nprobe, int32_t max_nprobe, int32_t k,
                              int32_t rerank, const ivf_search_opts* opts, void* workspace,
                              size_t workspace_bytes, int32_t* out_nprobe,
                              int32_t* out_reorder, void* stream);

/* The approximate coarse score matrix of an MFMA form (opts->coarse != EXACT):
 * out_scores [nq,L] FP32, |c_l|^2 - 2<q,c_l> (L2) or -<q,c_l> (IP) computed
 * from the operands in that precision with FP32 accumulation. */
ivf_status ivf_debug_coarse_scores(const ivf_index* idx, const float* queries,
                                   int32_t nq, const ivf_search_opts* opts,
                                   void* workspace, size_t workspace_bytes,
                                   float* out_scores, void* stream);

/* Step 2 only, for every (q, p < nprobe[q]) of caller-given probes:
 *   out_lut   [nq,max_nprobe,m,16] uint8 quantised table,
 *   out_lo    [nq,max_nprobe,m] FP32 per-subspace offsets,
 *   out_delta [nq,max_nprobe] FP32 scale, out_B [nq,max_nprobe] FP32 constant,
 * so that the ADC value of codes c is B + delta * sum_j lut[j][c_j].
 * Entries with p >= nprobe[q] are left untouched. */
ivf_status ivf_debug_luts(const ivf_index* idx, const float* queries,
                          int32_t nq, const int32_t* probes,
                          const int32_t* nprobe, int32_t max_nprobe,
                          uint8_t* out_lut, float* out_lo, float* out_delta,
                          float* out_B, void* stream);

/* Step 2 as the BATCHED form computes it (its own table builders: the scan
 * kernel's per-item builder for L2, the per-query table plus list bias for
 * IP), for every (q, p < nprobe[q]) of caller-given probes (rows as in
 * ivf_search_with_probes): out_lut [nq,max_nprobe,m,16] uint8,
 * out_delta and out_B [nq,max_nprobe] FP32; entries with p >= nprobe[q]
 * are left untouched. The workspace is sized by ivf_search_workspace_bytes
 * for (nq, max_nprobe, 1, 1) with opts.form = IVF_FORM_BATCHED (m <= 192).
 * Same quantities as ivf_debug_luts (sections 2.4, 2.5, 4.5.1). */
ivf_status ivf_debug_batched_luts(const ivf_index* idx, const float* queries,
                                  int32_t nq, const int32_t* probes,
                                  const int32_t* nprobe, int32_t max_nprobe,
                                  void* workspace, size_t workspace_bytes,
                                  uint8_t* out_lut, float* out_delta, float* out_B,
                                  void* stream);

/* Steps 2-4 on caller-given probes: out_keys [nq,rerank] uint64 candidate
 * keys in ascending order, key = (ord(a) << 32) | id, where a is the FP32
 * ADC value and ord maps float order onto unsigned order (sign bit set:
 * all bits inverted; else sign bit set). Padding is UINT64_MAX. On a
 * spilled index each point appears once, at its smallest a. */
ivf_status ivf_debug_candidates(const ivf_index* idx, const float* queries,
                                int32_t nq, const int32_t* probes,
                                const int32_t* nprobe, int32_t max_nprobe,
                                int32_t rerank, const ivf_search_opts* opts,
                                void* workspace, size_t workspace_bytes,
                                uint64_t* out_keys, void* stream);

/* Byte offsets of the table sections inside table_mem (for inspection):
 * codes: uint32 [blocks][words][64], word w of a point holds the 4-bit codes
 * of subspaces 8w..8w+7 in bits 4s..4s+3 (padding subspaces are 0);
 * slot_ids: int32 [blocks][64] point id per slot, -1 for padding (spilled
 * index: id * copies + c, c numbering one point's entries in slot order);
 * block_offsets: int32 [L+1] first block of each list; dims: int32 [d] kept
 * base columns of a filtered index (an empty section without filtration). */
typedef struct {
  size_t codes, slot_ids, block_offsets, list_len, centroids, probe_centroids,
      codebooks, probe_norms, probe_f32, probe_bf16, probe_fp8, probe_fp8_scale, dims, total;
  int32_t words_per_point, m_padded, blocks, L_padded, d_padded, reserved;
} ivf_table_layout;

/* Infrastructure. */
ivf_status ivf_get_table_layout(const ivf_index* idx, ivf_table_layout* out);

/* Reads and clears the device error word kept in `workspace` (synchronises
 * `stream`) into *out_mask (host): 0 when no device-side violation was
 * recorded since the last read, else a bit mask: 1 = an nprobe[q] out of
 * range; 2 = a caller-given probe row (ivf_search_with_probes,
 * ivf_debug_candidates) with a list index outside [0, L) or a list named
 * twice. Returns IVF_ERR_INVALID_ARG for a NULL argument, IVF_ERR_DEVICE when
 * a HIP call fails (*out_mask is then 0). Infrastructure: no passage of the
 * paper defines it. */
ivf_status ivf_get_device_error(const ivf_index* idx, void* workspace,
                                int32_t* out_mask, void* stream);

/* Per-stage timing of ivf_search / ivf_search_with_probes (infrastructure).
 * While enabled,
 * every search records HIP events on its stream around its stages
 * (IVF_STAGE_*): coarse scoring, probe selection, scan preparation (IP
 * biases; batched form: first-list pass and each round's work-list build),
 * the scan kernel itself (batched: every round's), the merges (batched
 * form; a spilled index's per-point pool reduction), the re-rank. ivf_profile_read waits for the last recorded event and
 * returns, per stage, the summed milliseconds and the number of completed
 * searches since the previous read (then resets). At most 64 searches are
 * kept between reads (older ones are dropped). Graph replays
 * (opts.use_graph) are not profiled. */
enum { IVF_STAGE_COARSE = 0, IVF_STAGE_SELECT = 1, IVF_STAGE_PREP = 2,
       IVF_STAGE_SCAN = 3, IVF_STAGE_MERGE = 4, IVF_STAGE_RERANK = 5,
       IVF_NSTAGES = 6 };
ivf_status ivf_profile_enable(ivf_index* idx, int32_t on);
ivf_status ivf_profile_read(ivf_index* idx, float* ms /* [IVF_NSTAGES] */,
                            int32_t* count);

/* ---- Index construction on the GPU (Alg. 1) ----------------------------- */

/* Workspace of ivf_assign for `chunk` rows per pass (1..2^20).
 * Infrastructure. */
size_t ivf_assign_workspace_bytes(int32_t L, int32_t d, int32_t chunk,
                                  int32_t coarse);

/* Nearest list of every row of X [n,d] (FP32, device): out_list[n] int32 =
 * the list with the smallest (canonical FP32 coarse score, list index)
 * against centroids [L,d] (device; the probe centroids: normalised for IP),
 * i.e. the top-1 of search step 1. coarse/widen as in ivf_search_opts: the
 * MFMA forms pre-select `widen` lists per row from the approximate scores,
 * then re-score canonically (exact when the canonical best is among them).
 * Rows are processed `chunk` at a time. Errors as for ivf_search. */
ivf_status ivf_assign(const float* centroids, int32_t L, int32_t d,
                      int32_t metric, const float* X, int64_t n, int32_t chunk,
                      int32_t coarse, int32_t widen, void* workspace,
                      size_t workspace_bytes, int32_t* out_list, void* stream);

/* PQ codes of residuals (Alg. 1 Quantize): out_codes [n,m] uint8,
 * code_j(x) = argmin_i sum_u (r_{j d'+u} - codebooks[j,i,u])^2 with
 * r = x - centroids[lists[x]] (each component rounded once), the sum
 * sequential in u in FP32, ties to the smallest i. All arrays device:
 * X [n,d], centroids [L,d] (mean centroids), lists [n], codebooks [m,16,d/m]. */
ivf_status ivf_encode(const float* X, int64_t n, int32_t d,
                      const float* centroids, const int32_t* lists,
                      const float* codebooks, int32_t m, uint8_t* out_codes,
                      void* stream);

/* Spill lists of SOAR (section 4.6.2 integrates it; the loss is SOAR's):
 * for every row x of X [n,d] with primary list p = primary[x] and residual
 * r = x - c_p, out_list[x] = the list l != p with the smallest
 *   loss(l) = sum_t (x_t - c_lt)^2 + lam * (sum_t r_t (x_t - c_lt))^2 / sum_t r_t^2
 * (the second term is dropped when r = 0), ties to the smaller l. Canonical
 * FP32: every component difference rounded once, the three sums sequential
 * in t, no fused multiply-add, then pp = proj * proj, loss = dist +
 * lam * (pp / rr). All arrays device: centroids [L,d] (the mean centroids,
 * the residual origin), primary [n] int32 in [0, L) (a row whose primary is
 * out of range gets out_list -1), out_list [n] int32.
 * L >= 2, lam finite and >= 0. Rows are processed `chunk` at a time
 * (workspace: ivf_assign_spill_workspace_bytes). */
size_t ivf_assign_spill_workspace_bytes(int32_t L, int32_t d, int32_t chunk);
ivf_status ivf_assign_spill(const float* centroids, int32_t L, int32_t d,
                            const float* X, int64_t n, const int32_t* primary,
                            float lam, int32_t chunk, void* workspace,
                            size_t workspace_bytes, int32_t* out_list,
                            void* stream);

/* Frees the host handle only; table_mem stays the caller's. Infrastructure. */
void ivf_destroy(ivf_index* idx);

/* Message for the last non-OK status on this thread ("" if none).
 * Infrastructure. */
const char* ivf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IVFPQ_IVF_H */
