// Batched form of steps 2-4: list-major, persistent, work-queue scheduled.
//
// The candidate pool of a query is the exact set of its R smallest keys
// (ord(a) << 32 | id) over every point of its probed lists, as in the plain
// form; only the schedule differs:
//   phase 1  per query, the plain scan of its first probed lists until at
//            least R points are seen: pool P1 and threshold thr = R-th key
//            (no key above thr can enter the final pool);
//   rounds   the remaining (query, list) pairs, restricted to a range of
//            probe ranks per round, are grouped by list into work items of
//            up to 16 queries (the longest lists' items first); persistent
//            workgroups pull items from an atomic counter, build the
//            queries' tables, stream the list's code blocks once, and append
//            every key <= thr of its query to a per-query survivor buffer;
//   merge    after each round, per query, the R smallest keys of the pool and
//            its survivors become the new pool and its R-th key the new thr,
//            so later rounds keep fewer survivors. A query whose buffer
//            overflowed is recomputed by the plain scan at the end.
//
// Table layout for the scan: entry (query g, subspace j, code c) is a u16 at
// ((j*2 + g/8)*16 + c)*8 + g%8. The 16 rows of one (j, half) span 256 bytes,
// every LDS bank once, so lanes reading any codes of the same subspace never
// conflict; one 16-byte read returns 8 queries' entries, summed with packed
// 16-bit adds (sums are at most 255*256 < 2^16).
#include "common.hpp"
#include "internal.hpp"

namespace ivf {

// Queries per work item: 16 (two 8-query halves of the table), or 8 when the
// 16-query table would leave room for only one workgroup per CU (m_pad > 96).
template <int W>
constexpr int item_queries() { return W * 8 > 96 ? 8 : 16; }
inline int item_queries_rt(int W) { return W * 8 > 96 ? 8 : 16; }

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// One three-input add and one byte extract per instruction, kept as written
// (the compiler would otherwise rebalance the sums into more instructions).
__device__ __forceinline__ uint32_t add3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ uint32_t bfe8(uint32_t x, int shift) {
  uint32_t r;
  asm("v_bfe_u32 %0, %1, %2, 8" : "=v"(r) : "v"(x), "i"(shift));
  return r;
}

// ---------------------------------------------------------------------------
// Work list: (query, probe slot) pairs of one round grouped by list. A pair
// belongs to the round [lo, hi) when p1[q] <= p < nprobe_eff[q], lo <= p < hi
// and the query has not overflowed.
// ---------------------------------------------------------------------------

struct RoundSel {
  const int32_t* nprobe_eff;
  const int32_t* p1;
  const int32_t* redo;
  int32_t lo, hi;
  __device__ __forceinline__ bool operator()(int q, int p) const {
    return p >= lo && p < hi && p >= p1[q] && p < nprobe_eff[q] && redo[q] == 0;
  }
};

constexpr int PAIR_CHUNK = 4096;  // (query, probe) entries per workgroup

// Per-list counts of phase-2 pairs: a workgroup histograms its chunk in LDS
// and adds each non-zero bin to the global count once (lists probed by many
// queries would otherwise serialise on global atomics).
__global__ void __launch_bounds__(256) pairs_count_kernel(int32_t nq, int32_t max_nprobe, int32_t L,
                                                          const int32_t* __restrict__ probes,
                                                          RoundSel sel,
                                                          int32_t* __restrict__ cnt) {
  extern __shared__ int32_t hist[];  // [L]
  for (int l = threadIdx.x; l < L; l += blockDim.x) hist[l] = 0;
  __syncthreads();
  const int64_t n = (int64_t)nq * max_nprobe;
  const int64_t b = (int64_t)blockIdx.x * PAIR_CHUNK;
  for (int64_t i = b + threadIdx.x; i < b + PAIR_CHUNK && i < n; i += blockDim.x) {
    const int q = (int)(i / max_nprobe), p = (int)(i % max_nprobe);
    if (sel(q, p)) atomicAdd(&hist[probes[i]], 1);
  }
  __syncthreads();
  for (int l = threadIdx.x; l < L; l += blockDim.x)
    if (hist[l]) atomicAdd(&cnt[l], hist[l]);
}

// Exclusive scans of per-list pair counts and item counts (one workgroup)
// over the lists in `order` (the index's lists longest first, so that the
// persistent workgroups take the long items first and the grid ends on short
// ones), or in index order when it is null; the items of one list are
// consecutive. Thread t owns the lists at positions [t*per, t*per + per),
// per <= 16 (L <= 16384): their list indices and counts are loaded together
// before the scan.
constexpr int SCAN_PER = MAX_SCAN_LISTS / 1024;
__global__ void __launch_bounds__(1024) pairs_scan_kernel(int32_t L, int32_t BG,
                                                         const int32_t* __restrict__ order,
                                                         const int32_t* __restrict__ cnt,
                                                         int32_t* __restrict__ list_start,
                                                         int32_t* __restrict__ item_start,
                                                         int32_t* __restrict__ cursor,
                                                         int32_t* __restrict__ item_list) {
  __shared__ int32_t sp[1024], si[1024];
  const int tid = threadIdx.x;
  const int per = (L + 1023) / 1024;
  const int b = tid * per, e = min(L, b + per);
  int32_t lid[SCAN_PER], c[SCAN_PER];
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    const int i = b + k;
    lid[k] = k < per && i < e ? (order ? order[i] : i) : -1;
  }
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) c[k] = lid[k] >= 0 ? cnt[lid[k]] : 0;
  int32_t ps = 0, is = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    ps += c[k];
    is += (c[k] + BG - 1) / BG;
  }
  sp[tid] = ps;
  si[tid] = is;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int32_t a = tid >= off ? sp[tid - off] : 0, d = tid >= off ? si[tid - off] : 0;
    __syncthreads();
    sp[tid] += a;
    si[tid] += d;
    __syncthreads();
  }
  int32_t pacc = sp[tid] - ps, iacc = si[tid] - is;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    if (lid[k] < 0) continue;
    const int l = lid[k];
    list_start[l] = pacc;
    item_start[l] = iacc;
    cursor[l] = 0;
    const int ni = (c[k] + BG - 1) / BG;
    for (int i = 0; i < ni; ++i) item_list[iacc + i] = l;
    pacc += c[k];
    iacc += ni;
  }
  if (tid == 1023) {
    list_start[L] = sp[1023];
    item_start[L] = si[1023];
  }
}

// Scatter the pairs to their list's range: a workgroup reserves, per list,
// one range for its whole chunk, then places entries with LDS atomics.
__global__ void __launch_bounds__(256) pairs_fill_kernel(int32_t nq, int32_t max_nprobe, int32_t L,
                                                         const int32_t* __restrict__ probes,
                                                         RoundSel sel,
                                                         const int32_t* __restrict__ list_start,
                                                         int32_t* __restrict__ cursor,
                                                         int32_t* __restrict__ pairs) {
  extern __shared__ int32_t hist[];  // [L]: counts, then base positions
  for (int l = threadIdx.x; l < L; l += blockDim.x) hist[l] = 0;
  __syncthreads();
  const int64_t n = (int64_t)nq * max_nprobe;
  const int64_t b = (int64_t)blockIdx.x * PAIR_CHUNK;
  for (int64_t i = b + threadIdx.x; i < b + PAIR_CHUNK && i < n; i += blockDim.x) {
    const int q = (int)(i / max_nprobe), p = (int)(i % max_nprobe);
    if (sel(q, p)) atomicAdd(&hist[probes[i]], 1);
  }
  __syncthreads();
  for (int l = threadIdx.x; l < L; l += blockDim.x)
    if (hist[l]) hist[l] = list_start[l] + atomicAdd(&cursor[l], hist[l]);
  __syncthreads();
  for (int64_t i = b + threadIdx.x; i < b + PAIR_CHUNK && i < n; i += blockDim.x) {
    const int q = (int)(i / max_nprobe), p = (int)(i % max_nprobe);
    if (sel(q, p)) {
      const int pos = atomicAdd(&hist[probes[i]], 1);
      pairs[2 * pos] = q;
      pairs[2 * pos + 1] = p;
    }
  }
}

// ---------------------------------------------------------------------------
// Wave-level table build of one (query, list), the canonical arithmetic of the
// plain form. Operands come from LDS: rq = the residual q - c_l (L2, each
// component rounded once) or q itself (IP), and the codebooks. Lane ln covers
// entries e = ln + 64 r (subspace j = 4r + ln/16, code ln%16). Pass 1 finds
// the per-subspace minima (kept in LDS) and the largest range; pass 2
// recomputes the same entries and writes the quantised u16 table into the
// interleaved layout.
// ---------------------------------------------------------------------------

__device__ __forceinline__ float lut_entry(const Tables& t, const float* rq, const float* cb_s,
                                           int j, int code) {
  const int ds = t.dsub;
  const float* cb = cb_s + ((size_t)j * KSUB + code) * ds;
  const float* r = rq + j * ds;
  float acc = 0.0f;
  if (t.metric == IVF_METRIC_L2) {
    for (int u = 0; u < ds; ++u) {
      const float df = r[u] - cb[u];
      acc = acc + df * df;
    }
    return acc;
  }
  for (int u = 0; u < ds; ++u) acc = acc + r[u] * cb[u];
  return plus_zero(-acc);
}

// Destination of a built table: the interleaved u16 scan layout (slot g of
// the item) or, for inner product, the per-query table in global memory
// (code-major: entry (j, c) at c*m_pad + j).
struct ItemStore {
  uint16_t* lut16;
  int g;
  int halves;  // 8-query halves of the item table (1 or 2)
  __device__ __forceinline__ void operator()(int j, int code, uint32_t v) const {
    lut16[((j * halves + (g >> 3)) * 16 + code) * 8 + (g & 7)] = (uint16_t)v;
  }
};

template <int W, class Store>
__device__ __forceinline__ void wave_build_lut(const Tables& t, const float* rq, const float* cb_s,
                                               float bias, const Store& store, float* lo_s,
                                               float* outB, float* outDelta) {
  constexpr int MP = W * 8;  // padded subspaces
  const int ln = lane_id();
  const int code = ln & 15;
  if constexpr (MP <= 64) {
    // Up to 16 entries per lane: keep them in registers, one pass.
    constexpr int NR = MP / 4;
    float T[NR];
    float mx = 0.0f;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int j = 4 * r + (ln >> 4);
      T[r] = j < t.m ? lut_entry(t, rq, cb_s, j, code) : 0.0f;
      float v = T[r];
      for (int s = 1; s < 16; s <<= 1) v = fminf(v, __shfl_xor(v, s));
      if (code == 0 && j < t.m) lo_s[j] = v;
      T[r] = T[r] - v;  // entry minus its subspace minimum (rounded once)
      mx = fmaxf(mx, T[r]);
    }
    for (int s = 1; s < IVF_WAVE; s <<= 1) mx = fmaxf(mx, __shfl_xor(mx, s));
    const float rng = mx;
    const bool live = rng > 0.0f;
    const float sc = live ? 255.0f / rng : 0.0f;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int j = 4 * r + (ln >> 4);
      uint32_t v = 0;
      if (live && j < t.m) v = (uint32_t)fminf(rintf(T[r] * sc), 255.0f);
      store(j, code, v);
    }
    const float ls = wave_pairwise_sum(lo_s, t.m);
    if (ln == 0) {
      *outB = ls + bias;
      *outDelta = live ? rng / 255.0f : 0.0f;
    }
    return;
  }
  const int nr = (t.m + 3) / 4;
  float mx = 0.0f;
#pragma unroll 1
  for (int r = 0; r < nr; ++r) {
    const int j = 4 * r + (ln >> 4);
    const float T = j < t.m ? lut_entry(t, rq, cb_s, j, code) : 0.0f;
    float v = T;
    for (int s = 1; s < 16; s <<= 1) v = fminf(v, __shfl_xor(v, s));
    if (code == 0 && j < t.m) lo_s[j] = v;
    mx = fmaxf(mx, T - v);
  }
  for (int s = 1; s < IVF_WAVE; s <<= 1) mx = fmaxf(mx, __shfl_xor(mx, s));
  const float rng = mx;
  const bool live = rng > 0.0f;
  const float sc = live ? 255.0f / rng : 0.0f;
#pragma unroll 1
  for (int r = 0; r < MP / 4; ++r) {
    const int j = 4 * r + (ln >> 4);
    uint32_t v = 0;
    if (live && j < t.m)
      v = (uint32_t)fminf(rintf((lut_entry(t, rq, cb_s, j, code) - lo_s[j]) * sc), 255.0f);
    store(j, code, v);
  }
  const float ls = wave_pairwise_sum(lo_s, t.m);
  if (ln == 0) {
    *outB = ls + bias;
    *outDelta = live ? rng / 255.0f : 0.0f;
  }
}

// L2 table of one (query, list) with one lane per subspace (m_pad <= 64):
// the 16 entries of subspace j stay in lane j's registers, so its minimum is
// local and a single cross-lane max gives the range. Lane j visits the codes
// in the rotated order (k + j) mod 16, which spreads every store into the
// interleaved table over 16 LDS banks (and every codebook read over 64).
// Same canonical arithmetic as lut_entry: r_u = q_u - c_u rounded once,
// T = sum_u (r_u - B_u)^2 sequentially in u. cbT: codebooks transposed in
// LDS, entry (j, code, u) at (code*d' + u)*m_pad + j.
template <int W>
__device__ __forceinline__ void wave_build_lut_lanes(const Tables& t, const float* qg,
                                                     const float* cl, const float* cbT, int g,
                                                     uint16_t* lut16, float* outB,
                                                     float* outDelta) {
  constexpr int MP = W * 8;
  static_assert(MP <= IVF_WAVE, "one lane per subspace");
  const int j = lane_id();
  const int ds = t.dsub;
  const bool has = j < t.m;
  float T[KSUB];
#pragma unroll
  for (int k = 0; k < KSUB; ++k) T[k] = 0.0f;
  float lo = 0.0f, mx = 0.0f;
  if (has) {
    for (int u = 0; u < ds; ++u) {
      const float r = qg[j * ds + u] - cl[j * ds + u];
#pragma unroll
      for (int k = 0; k < KSUB; ++k) {
        const int code = (k + j) & 15;
        const float df = r - cbT[(code * ds + u) * MP + j];
        T[k] = T[k] + df * df;
      }
    }
    lo = T[0];
#pragma unroll
    for (int k = 1; k < KSUB; ++k) lo = fminf(lo, T[k]);
#pragma unroll
    for (int k = 0; k < KSUB; ++k) {
      T[k] = T[k] - lo;  // entry minus its subspace minimum (rounded once)
      mx = fmaxf(mx, T[k]);
    }
  }
  for (int s = 1; s < IVF_WAVE; s <<= 1) mx = fmaxf(mx, __shfl_xor(mx, s));
  const float rng = mx;
  const bool live = rng > 0.0f;
  const float sc = live ? 255.0f / rng : 0.0f;
  if (j < MP) {
#pragma unroll
    for (int k = 0; k < KSUB; ++k) {
      const int code = (k + j) & 15;
      uint32_t v = 0;
      if (live && has) v = (uint32_t)fminf(rintf(T[k] * sc), 255.0f);
      lut16[((j * 2 + (g >> 3)) * 16 + code) * 8 + (g & 7)] = (uint16_t)v;  // 16-query items
    }
  }
  // Pairwise sum of lo_j over j < m (zeros beyond): the butterfly pairs the
  // same operands in every lane, so lane 0 holds the canonical tree sum.
  const int width = (int)pow2_ceil((uint32_t)t.m);
  float x = has ? lo : 0.0f;
  for (int s = 1; s < width; s <<= 1) x = x + __shfl_xor(x, s);
  const float ls = __shfl(x, 0);
  if (j == 0) {
    *outB = ls + 0.0f;
    *outDelta = live ? rng / 255.0f : 0.0f;
  }
}

// The same build for 64 < m_pad <= 128 with two subspaces per lane (j and
// j + 64) and the item's half count as a parameter. The pairwise sum of lo
// is the canonical tree over 128 leaves: its top level adds the halves
// 0..63 and 64..127, each the butterfly of one lane-resident value.
template <int W, int HALVES>
__device__ __forceinline__ void wave_build_lut_lanes2(const Tables& t, const float* qg,
                                                      const float* cl, const float* cbT, int g,
                                                      uint16_t* lut16, float* outB,
                                                      float* outDelta) {
  constexpr int MP = W * 8;
  static_assert(MP > IVF_WAVE && MP <= 2 * IVF_WAVE, "two subspaces per lane");
  const int ln = lane_id();
  const int ds = t.dsub;
  float T[2][KSUB];
  float lo[2] = {0.0f, 0.0f};
  float mx = 0.0f;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = ln + IVF_WAVE * h;
#pragma unroll
    for (int k = 0; k < KSUB; ++k) T[h][k] = 0.0f;
    if (j < t.m) {
      for (int u = 0; u < ds; ++u) {
        const float r = qg[j * ds + u] - cl[j * ds + u];
#pragma unroll
        for (int k = 0; k < KSUB; ++k) {
          const int code = (k + j) & 15;
          const float df = r - cbT[(code * ds + u) * MP + j];
          T[h][k] = T[h][k] + df * df;
        }
      }
      float v = T[h][0];
#pragma unroll
      for (int k = 1; k < KSUB; ++k) v = fminf(v, T[h][k]);
      lo[h] = v;
#pragma unroll
      for (int k = 0; k < KSUB; ++k) {
        T[h][k] = T[h][k] - v;  // entry minus its subspace minimum (rounded once)
        mx = fmaxf(mx, T[h][k]);
      }
    }
  }
  for (int s = 1; s < IVF_WAVE; s <<= 1) mx = fmaxf(mx, __shfl_xor(mx, s));
  const float rng = mx;
  const bool live = rng > 0.0f;
  const float sc = live ? 255.0f / rng : 0.0f;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = ln + IVF_WAVE * h;
    if (j < MP) {
#pragma unroll
      for (int k = 0; k < KSUB; ++k) {
        const int code = (k + j) & 15;
        uint32_t v = 0;
        if (live && j < t.m) v = (uint32_t)fminf(rintf(T[h][k] * sc), 255.0f);
        lut16[((j * HALVES + (g >> 3)) * 16 + code) * 8 + (g & 7)] = (uint16_t)v;
      }
    }
  }
  float x0 = lo[0], x1 = lo[1];
  for (int s = 1; s < IVF_WAVE; s <<= 1) {
    x0 = x0 + __shfl_xor(x0, s);
    x1 = x1 + __shfl_xor(x1, s);
  }
  const float ls = __shfl(x0, 0) + __shfl(x1, 0);
  if (ln == 0) {
    *outB = ls + 0.0f;
    *outDelta = live ? rng / 255.0f : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// Phase 2: persistent list-major scan.
// ---------------------------------------------------------------------------

// Per-workgroup LDS of the scan kernel. The per-wave subspace minima are
// needed only by the generic L2 builder (wave_build_lut).
template <int W, int BG, bool NEED_LO>
struct BatchShared {
  uint16_t lut16[W * 8 * (BG / 8) * 16 * 8];
  float lo[NEED_LO ? IVF_NWAVES : 1][NEED_LO ? W * 8 : 1];
  float B[BG], delta[BG];
  uint64_t thr[BG];
  // Per query pair k (queries 2k, 2k+1 in the low, high half): 1 + the
  // largest S whose value can still pass, 0 if none can (S < 2^16 always).
  uint32_t slim[BG / 2];
  int32_t qid[BG], slot[BG];
  int32_t item, next, l, nqi;
};

// Codebooks are staged in LDS when they fit beside the tables.
template <int W>
constexpr bool cb_in_lds() { return W <= 16; }
// L2 tables are built with one lane per subspace (two when m_pad > 64) when
// m_pad <= 128.
template <int W>
constexpr bool lane_build() { return W * 8 <= 2 * IVF_WAVE; }

// PER_QUERY (inner product): the tables come from the first-list pass (one
// per query, published by the plain kernel) and are only copied per item; otherwise (L2) each item builds its residual tables.
// Three workgroups per CU (12 waves) fit the LDS of every shape; the register
// budget is set to match (the unrolled word loop would otherwise hoist
// most of its table reads and leave room for one).
template <int W, bool PER_QUERY, int BG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
batched_scan_kernel(
    Tables t, const float* __restrict__ Q, int32_t max_nprobe, const float* __restrict__ bias,
    const uint64_t* __restrict__ thr, const int32_t* __restrict__ list_start,
    const int32_t* __restrict__ list_cnt,
    const int32_t* __restrict__ item_start, const int32_t* __restrict__ item_list,
    const int32_t* __restrict__ pairs, uint32_t* __restrict__ queue,
    int32_t* __restrict__ spill_cnt, uint64_t* __restrict__ spill, int32_t cap,
    const uint32_t* __restrict__ qlut, const float* __restrict__ qlo_sum,
    const float* __restrict__ qdelta) {
  constexpr bool per_query = PER_QUERY;
  constexpr bool need_lo = !per_query && !lane_build<W>();
  __shared__ BatchShared<W, BG, need_lo> sh;
  constexpr int HALVES = BG / 8;
  extern __shared__ __align__(16) unsigned char dyn[];
  // L2 only: per-wave residual operand and (when they fit) the codebooks.
  float* rq_all = reinterpret_cast<float*>(dyn);         // [4][d] per-wave query operand
  float* cb_s = rq_all + IVF_NWAVES * t.d;               // [m*16*d'] (when staged)
  const float* cb = cb_in_lds<W>() ? cb_s : t.codebooks;
  float* rq = rq_all + wave_index() * t.d;
  const int tid = threadIdx.x, wave = tid / IVF_WAVE, ln = lane_id();
  const int n_items = item_start[t.L];
  float* cbT = reinterpret_cast<float*>(dyn);  // lane builder: [16*d'][m_pad]
  if constexpr (!per_query && lane_build<W>()) {
    constexpr int MP = W * 8;
    const int per = KSUB * t.dsub;  // floats per subspace
    for (int i = tid; i < t.m * per; i += blockDim.x) {
      const int j = i / per, cu = i % per;  // cu = code * d' + u
      cbT[cu * MP + j] = t.codebooks[i];
    }
  } else if constexpr (cb_in_lds<W>() && !per_query) {
    for (int i = tid; i < t.m * KSUB * t.dsub; i += blockDim.x) cb_s[i] = t.codebooks[i];
  }
  if (tid == 0) sh.next = (int32_t)atomicAdd(queue, 1u);
  __syncthreads();
  for (;;) {
    const int item = sh.next;
    if (item >= n_items) break;  // uniform: every wave leaves together
    if (tid < BG) {
      const int l = item_list[item];
      const int first = (item - item_start[l]) * BG;
      const int nqi = min(BG, list_cnt[l] - first);
      const bool v = tid < nqi;
      const int pi = list_start[l] + first + tid;
      const int q = v ? pairs[2 * pi] : -1;
      sh.qid[tid] = q;
      sh.slot[tid] = v ? pairs[2 * pi + 1] : 0;
      sh.thr[tid] = v ? thr[q] : 0ull;
      if (tid == 0) {
        sh.l = l;
        sh.nqi = nqi;
      }
    }
    __syncthreads();
    if (tid == 0) sh.next = (int32_t)atomicAdd(queue, 1u);  // overlaps this item
    const int l = sh.l, nqi = sh.nqi;
    const int n_l = t.list_len[l];
    const int blk0 = t.block_off[l];
    const int nblk = (n_l + BLOCK_PTS - 1) / BLOCK_PTS;
    // Each wave's first code block is requested now; its latency overlaps
    // the table set-up below.
    uint32_t nx[W];
    uint32_t nid = 0;
    if (wave < nblk) {
      const uint32_t* cw = t.codes + (size_t)(blk0 + wave) * W * BLOCK_PTS + ln;
#pragma unroll
      for (int w = 0; w < W; ++w) nx[w] = cw[w * BLOCK_PTS];
      nid = (uint32_t)t.slot_ids[(size_t)(blk0 + wave) * BLOCK_PTS + ln];
    }
    if constexpr (per_query) {
      // Copy the queries' tables into the interleaved layout. Lane (c, pp)
      // of task (subspaces 4jg..4jg+3, half h) moves code c of queries
      // g0 = 8h + 2pp and g0 + 1: each store is one u32 holding both u16
      // entries, and the 64 lanes of a store hit 64 distinct banks.
      constexpr int MP = W * 8;
      const int c = ln >> 2, pp = ln & 3;
#pragma unroll 1
      for (int task = wave; task < MP / 4 * HALVES; task += IVF_NWAVES) {
        const int jg = task / HALVES, h = task % HALVES;
        const int g0 = 8 * h + 2 * pp;
        const uint32_t a0 = g0 < nqi ? qlut[((size_t)sh.qid[g0] * KSUB + c) * (MP / 4) + jg] : 0u;
        const uint32_t a1 =
            g0 + 1 < nqi ? qlut[((size_t)sh.qid[g0 + 1] * KSUB + c) * (MP / 4) + jg] : 0u;
        uint32_t* dst = reinterpret_cast<uint32_t*>(sh.lut16);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int j = 4 * jg + jj;
          const uint32_t v = ((a0 >> (8 * jj)) & 0xffu) | (((a1 >> (8 * jj)) & 0xffu) << 16);
          dst[(((j * HALVES + h) * 16 + c) * 8 + (g0 & 7)) >> 1] = v;
        }
      }
      if (tid < nqi) {
        const int q = sh.qid[tid];
        sh.B[tid] = qlo_sum[q] + bias[(size_t)q * max_nprobe + sh.slot[tid]];
        sh.delta[tid] = qdelta[q];
      }
    }
    // L2 tables: wave w builds queries w, w+4, w+8, w+12; absent queries get
    // an all-zero table and no passing S.
#pragma unroll 1
    for (int g = wave; g < BG && !per_query; g += IVF_NWAVES) {
      if (g < nqi) {
        const float* qg = Q + (size_t)sh.qid[g] * t.d;
        const float* c = t.cm + (size_t)l * t.d;
        if constexpr (lane_build<W>() && W * 8 <= IVF_WAVE) {
          static_assert(BG == 16, "the one-lane builder writes 16-query items");
          wave_build_lut_lanes<W>(t, qg, c, cbT, g, sh.lut16, &sh.B[g], &sh.delta[g]);
        } else if constexpr (lane_build<W>()) {
          wave_build_lut_lanes2<W, HALVES>(t, qg, c, cbT, g, sh.lut16, &sh.B[g], &sh.delta[g]);
        } else {
          for (int i = ln; i < t.d; i += IVF_WAVE) rq[i] = qg[i] - c[i];
          wave_build_lut<W>(t, rq, cb, 0.0f, ItemStore{sh.lut16, g, HALVES},
                            sh.lo[need_lo ? wave : 0], &sh.B[g], &sh.delta[g]);
        }
      } else {
        for (int e = ln; e < W * 8 * 16; e += IVF_WAVE)
          sh.lut16[(((e >> 4) * HALVES + (g >> 3)) * 16 + (e & 15)) * 8 + (g & 7)] = 0;
      }
    }
    __syncthreads();
    // Per query, the largest integer sum S whose value a(S) = B + delta*S can
    // still be <= the threshold's value part; a(S) is non-decreasing in S, so
    // a point with a larger S cannot pass and needs no key.
    if (tid < BG) {
      const int g = tid;
      uint32_t smax = 0xffffffffu;  // no S passes
      if (g < nqi) {
        const uint32_t othr = (uint32_t)(sh.thr[g] >> 32);
        const float Bg = sh.B[g], dg = sh.delta[g];
        int lo = -1, hi = 65536;  // f(lo) passes (or lo = -1), f(hi) fails
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (f2ord(plus_zero(Bg + dg * (float)mid)) <= othr) lo = mid; else hi = mid;
        }
        smax = lo < 0 ? 0xffffffffu : (uint32_t)lo;
      }
      // 1 + smax in the query's u16 half (0: none). Sums are at most
      // 255 * 192 < 65534, so clamping smax to 65534 changes no outcome.
      const uint32_t lim = smax == 0xffffffffu ? 0u : (smax < 65534u ? smax : 65534u) + 1u;
      const uint32_t other = __shfl_xor(lim, 1);
      if ((g & 1) == 0) sh.slim[g >> 1] = lim | (other << 16);
    }
    __syncthreads();
    // Code words stay in registers: the current block in `cur`, the wave's
    // next block in flight into `nx` (when there is none the current block is
    // requested again and not used; a branch would make the compiler wait
    // for the loads before the lookups). The block's slot ids travel with
    // its words, so a block with candidates does not wait for them.
    const unsigned char* lutb = reinterpret_cast<const unsigned char*>(sh.lut16);
#pragma unroll 1
    for (int bi = wave; bi < nblk; bi += IVF_NWAVES) {
      const int blk = blk0 + bi;
      uint32_t cur[W];
#pragma unroll
      for (int w = 0; w < W; ++w) cur[w] = nx[w];
      const uint32_t cur_id = nid;
      {
        const int nb = bi + IVF_NWAVES < nblk ? blk + IVF_NWAVES : blk;
        const uint32_t* cw = t.codes + (size_t)nb * W * BLOCK_PTS + ln;
#pragma unroll
        for (int w = 0; w < W; ++w) nx[w] = cw[w * BLOCK_PTS];
        nid = (uint32_t)t.slot_ids[(size_t)nb * BLOCK_PTS + ln];
      }
      // acc[k] holds the sums of queries 2k (low half) and 2k+1 (high half).
      // Plain 32-bit adds are exact on the packed pairs: a half never exceeds
      // 255 * 192 < 2^16, so no carry crosses into the high half, and two
      // subspaces fold into one three-input add.
      constexpr int NACC = BG / 2;
      constexpr uint32_t SUBB = HALVES * 256;  // bytes of one subspace's rows
      uint32_t acc[NACC];
#pragma unroll
      for (int k = 0; k < NACC; ++k) acc[k] = 0u;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        // Byte k of ev / od: the code of subspace 8w + 2k / 8w + 2k + 1,
        // times 16 (the byte offset of its row within the subspace).
        const uint32_t ev = (cur[w] << 4) & 0xf0f0f0f0u;
        const uint32_t od = cur[w] & 0xf0f0f0f0u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const unsigned char* r0 = lutb + bfe8(ev, 8 * k) + (uint32_t)(w * 8 + 2 * k) * SUBB;
          const unsigned char* r1 = lutb + bfe8(od, 8 * k) + (uint32_t)(w * 8 + 2 * k + 1) * SUBB;
#pragma unroll
          for (int h = 0; h < HALVES; ++h) {
            const uint4 a = *reinterpret_cast<const uint4*>(r0 + 256 * h);
            const uint4 b = *reinterpret_cast<const uint4*>(r1 + 256 * h);
            acc[4 * h + 0] = add3(acc[4 * h + 0], a.x, b.x);
            acc[4 * h + 1] = add3(acc[4 * h + 1], a.y, b.y);
            acc[4 * h + 2] = add3(acc[4 * h + 2], a.z, b.z);
            acc[4 * h + 3] = add3(acc[4 * h + 3], a.w, b.w);
          }
        }
        // One word's table reads and adds stay together: without this fence
        // the scheduler hoists later words' reads and runs out of registers.
        // The other resident waves hide each word's LDS latency.
        __builtin_amdgcn_sched_barrier(0);
      }
      const bool valid = bi * BLOCK_PTS + ln < n_l;
      // Pre-check in the integer domain: per half, the saturating difference
      // (1 + smax) - S is non-zero exactly when S <= smax (absent queries
      // have 1 + smax = 0).
      uint32_t hit = 0;
#pragma unroll
      for (int k = 0; k < NACC; ++k)
        hit |= __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(
                                                __builtin_bit_cast(u16x2, sh.slim[k]),
                                                __builtin_bit_cast(u16x2, acc[k])));
      if (__ballot(valid && hit != 0) == 0) continue;  // the common case: nothing passes
      uint32_t cand = 0;
#pragma unroll
      for (int g = 0; g < BG; ++g) {
        const uint32_t S = (acc[g >> 1] >> (16 * (g & 1))) & 0xffffu;
        const uint32_t lim = (sh.slim[g >> 1] >> (16 * (g & 1))) & 0xffffu;
        cand |= S < lim ? (1u << g) : 0u;
      }
      if (!valid) cand = 0;
      // Rare path: exact keys for the candidate (point, query) pairs.
      const uint32_t id = cand ? cur_id : 0u;
      // Which candidates pass on the full key; lane g collects query g's count.
      uint32_t passbits = 0, count = 0;
#pragma unroll
      for (int g = 0; g < BG; ++g) {
        const bool c = (cand >> g) & 1u;
        if (__ballot(c) == 0) continue;
        const uint32_t S = (acc[g >> 1] >> (16 * (g & 1))) & 0xffffu;
        const uint64_t key = make_key(plus_zero(sh.B[g] + sh.delta[g] * (float)S), id);
        const bool pass = c && key <= sh.thr[g];
        passbits |= pass ? 1u << g : 0u;
        const uint32_t n = (uint32_t)__popcll(__ballot(pass));
        count = ln == g ? n : count;
      }
      // One reservation per query with survivors, all issued together.
      uint32_t base = 0;
      if (ln < BG && count) base = (uint32_t)atomicAdd(&spill_cnt[sh.qid[ln]], (int)count);
#pragma unroll
      for (int g = 0; g < BG; ++g) {
        const bool pass = (passbits >> g) & 1u;
        const uint64_t mask = __ballot(pass);
        if (mask == 0) continue;
        const uint32_t pos = (uint32_t)__shfl((int)base, g) + lanes_below(mask);
        if (pass && pos < (uint32_t)cap) {
          const uint32_t S = (acc[g >> 1] >> (16 * (g & 1))) & 0xffffu;
          spill[(size_t)sh.qid[g] * cap + pos] =
              make_key(plus_zero(sh.B[g] + sh.delta[g] * (float)S), id);
        }
      }
    }
    __syncthreads();  // the tables are rebuilt for the next item
  }
}

// ---------------------------------------------------------------------------
// Merge after a round: pool plus survivors -> the R smallest keys, and their
// largest as the next round's threshold. The pool is full whenever survivors
// exist (the first pass stops only after R points, or at the last list), and
// keys are unique, so exactly R keys remain.
// ---------------------------------------------------------------------------

// Grid-stride over queries: a launch with a large LDS footprint runs one
// workgroup per CU and skips the queries another launch takes.
__global__ void __launch_bounds__(256) merge_kernel(int32_t nq, int32_t R, int32_t cap,
                                                    int32_t ns_lo, int32_t ns_hi,
                                                    const int32_t* __restrict__ nprobe_eff,
                                                    const int32_t* __restrict__ spill_cnt,
                                                    const uint64_t* __restrict__ spill,
                                                    uint64_t* __restrict__ cand,
                                                    uint64_t* __restrict__ thr,
                                                    int32_t* __restrict__ redo) {
  extern __shared__ __align__(16) unsigned char dyn[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(dyn);  // [pow2(R + ns_hi)]
  __shared__ SelectScratch sc;
  __shared__ uint32_t cnt;
  __shared__ unsigned long long maxkey;
  const int tid = threadIdx.x;
  for (int q = blockIdx.x; q < nq; q += gridDim.x) {  // q is uniform: barriers are safe
    const int ns = spill_cnt[q];
    if (nprobe_eff[q] < 0 || redo[q] != 0 || ns <= ns_lo) continue;
    if (ns > cap) {
      if (tid == 0) redo[q] = 1;  // recomputed at the end; skipped from now on
      continue;
    }
    if (ns > ns_hi) continue;  // a later launch with more LDS takes it
    if (tid == 0) cnt = 0;
    __syncthreads();
    for (int i = tid; i < R; i += blockDim.x) {
      const uint64_t k = cand[(size_t)q * R + i];
      wave_append(k != KEY_NONE, k, keys, &cnt);
    }
    __syncthreads();
    uint32_t n = cnt;
    for (int i = tid; i < ns; i += blockDim.x) keys[n + i] = spill[(size_t)q * cap + i];
    __syncthreads();
    n += (uint32_t)ns;
    if (n > (uint32_t)R) {
      KeyUnion u{keys, n, nullptr, 0};
      const uint64_t kth = block_kth(u, (uint32_t)R, &sc);
      n = block_compact_le(keys, n, kth, &cnt);
      if (n > (uint32_t)R) n = (uint32_t)R;
    }
    for (int i = tid; i < R; i += blockDim.x)
      cand[(size_t)q * R + i] = (uint32_t)i < n ? keys[i] : KEY_NONE;
    if (n == (uint32_t)R) {
      // Its largest key, the R-th smallest so far, bounds every key that can
      // still enter the pool (block_kth may return a looser bound).
      if (tid == 0) maxkey = 0;
      __syncthreads();
      uint64_t mk = 0;
      for (uint32_t i = tid; i < n; i += blockDim.x) mk = keys[i] > mk ? keys[i] : mk;
      for (int off = 1; off < IVF_WAVE; off <<= 1) {
        const uint64_t o = __shfl_xor(mk, off);
        mk = o > mk ? o : mk;
      }
      if (lane_id() == 0) atomicMax(&maxkey, (unsigned long long)mk);
      __syncthreads();
      if (tid == 0) thr[q] = maxkey;
    }
    __syncthreads();  // LDS is reused by the next query
  }
}

// ---------------------------------------------------------------------------

hipError_t launch_scan_plain_ex(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                                int32_t rerank, const Workspace& w, int32_t* p1_out,
                                uint64_t* thr_out, const int32_t* only, hipStream_t s);

// Survivor capacity per query: as many keys as the merge can hold in LDS
// beside the pool (MERGE_KEYS in all), within SPILL_BUDGET bytes for the batch.
constexpr int32_t MERGE_KEYS = 16384;  // 128 KiB of LDS
constexpr int64_t SPILL_BUDGET = 2ll << 30;

int32_t batched_spill_cap(int32_t R, int32_t nq) {
  int64_t c = SPILL_BUDGET / (8 * (int64_t)(nq > 0 ? nq : 1));
  if (c > MERGE_KEYS - R) c = MERGE_KEYS - R;
  if (c < 1024) c = 1024;
  return (int32_t)c;
}

// The first merge launch takes queries with up to this many survivors, with
// a small LDS footprint (many workgroups per CU); a second one the rest.
static int32_t merge_small_ns(int32_t R, int32_t cap) {
  const int32_t keys = (int32_t)pow2_ceil((uint32_t)(R + 2048));
  const int32_t n = keys - R;
  return n < cap ? n : cap;
}

hipError_t launch_batched_first(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                                int32_t R, const Workspace& w, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  hipError_t e;
  if ((e = launch_fill_u32((uint32_t*)w.redo, 0u, (size_t)nq, s)) != hipSuccess) return e;
  // First lists per query -> pool, threshold, first probe rank of the rounds
  // and, for inner product, the per-query tables of the list-major scan.
  return launch_scan_plain_ex(t, Q, nq, max_nprobe, R, w, w.p1, w.thr, nullptr, s);
}

hipError_t launch_batched_pairs(const Tables& t, int32_t nq, int32_t max_nprobe, int32_t lo,
                                int32_t hi, const Workspace& w, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  hipError_t e;
  if ((e = launch_fill_u32((uint32_t*)w.list_cnt, 0u, (size_t)t.L, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32((uint32_t*)w.spill_cnt, 0u, (size_t)nq, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(w.queue, 0u, 1, s)) != hipSuccess) return e;
  const RoundSel sel{w.nprobe_eff, w.p1, w.redo, lo, hi};
  const int64_t np_total = (int64_t)nq * max_nprobe;
  const unsigned g1 = (unsigned)((np_total + PAIR_CHUNK - 1) / PAIR_CHUNK);
  const size_t hist_lds = (size_t)t.L * 4;
  hipLaunchKernelGGL(pairs_count_kernel, dim3(g1), dim3(256), hist_lds, s, nq, max_nprobe, t.L,
                     w.probes, sel, w.list_cnt);
  hipLaunchKernelGGL(pairs_scan_kernel, dim3(1), dim3(1024), 0, s, t.L, item_queries_rt(t.words),
                     w.list_order == 0 ? t.list_order : nullptr, w.list_cnt, w.list_start,
                     w.item_start, w.list_cursor, w.item_list);
  hipLaunchKernelGGL(pairs_fill_kernel, dim3(g1), dim3(256), hist_lds, s, nq, max_nprobe, t.L,
                     w.probes, sel, w.list_start, w.list_cursor, w.pairs);
  return hipGetLastError();
}

template <int W>
static hipError_t launch_main_w(const Tables& t, const float* Q, int32_t max_nprobe,
                                const Workspace& w, hipStream_t s) {
  constexpr int BG = item_queries<W>();
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t lds = t.metric == IVF_METRIC_IP ? 0
                     : lane_build<W>()
                         ? (size_t)W * 8 * KSUB * t.dsub * 4
                         : (size_t)IVF_NWAVES * t.d * 4 +
                               (cb_in_lds<W>() ? (size_t)t.m * KSUB * t.dsub * 4 : 0);
  const dim3 block(256);
  const uint32_t* qlut = reinterpret_cast<const uint32_t*>(w.qlut);
  auto launch = [&](auto kernel) -> hipError_t {
    // Persistent grid: as many workgroups per CU as registers and LDS allow
    // (at most 6), unless the caller fixed it.
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, lds) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (per_cu > 6) per_cu = 6;
    if (w.grid > 0) per_cu = w.grid;
    hipLaunchKernelGGL(kernel, dim3(cus * per_cu), block, lds, s, t, Q, max_nprobe, w.bias,
                       w.thr, w.list_start, w.list_cnt, w.item_start, w.item_list, w.pairs,
                       w.queue,
                       w.spill_cnt, w.spill, w.spill_cap, qlut, w.qlo_sum, w.qdelta);
    return hipGetLastError();
  };
  if (t.metric == IVF_METRIC_IP) return launch(batched_scan_kernel<W, true, BG>);
  return launch(batched_scan_kernel<W, false, BG>);
}

hipError_t launch_batched_main(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                               int32_t R, const Workspace& w, hipStream_t s) {
  (void)R;
  if (nq == 0) return hipSuccess;
  switch (t.words) {
#define X(N) \
  case N: return launch_main_w<N>(t, Q, max_nprobe, w, s);
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
    X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24)
#undef X
    default: return hipErrorNotSupported;
  }
}

hipError_t launch_batched_merge(const Tables& t, int32_t nq, int32_t R, const Workspace& w,
                                hipStream_t s) {
  (void)t;
  if (nq == 0) return hipSuccess;
  const int32_t cap = w.spill_cap, small = merge_small_ns(R, cap);
  size_t lds = (size_t)pow2_ceil((uint32_t)(R + small)) * 8;
  hipLaunchKernelGGL(merge_kernel, dim3(nq), dim3(256), lds, s, nq, R, cap, 0, small,
                     w.nprobe_eff, w.spill_cnt, w.spill, w.cand, w.thr, w.redo);
  if (cap > small) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    lds = (size_t)pow2_ceil((uint32_t)(R + cap)) * 8;
    const int grid = nq < cus ? nq : cus;
    hipLaunchKernelGGL(merge_kernel, dim3(grid), dim3(256), lds, s, nq, R, cap, small, cap,
                       w.nprobe_eff, w.spill_cnt, w.spill, w.cand, w.thr, w.redo);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Parity export of the batched form's tables. Per (query, probe slot) the
// table the scan would use, as u8 [m][16] with its scale delta and constant
// B: for L2 the scan kernel's own per-item builder for this W (the query in
// slot 0 of an item, one wave), for inner product the per-query table the
// first-list pass publishes, with B = its pairwise sum of the minima + the
// list bias.
// ---------------------------------------------------------------------------

template <int W>
__global__ void __launch_bounds__(IVF_WAVE) batched_lut_export_kernel(
    Tables t, const float* __restrict__ Q, int32_t max_nprobe, const int32_t* __restrict__ probes,
    const int32_t* __restrict__ nprobe_eff, const float* __restrict__ bias,
    const uint8_t* __restrict__ qlut, const float* __restrict__ qlo_sum,
    const float* __restrict__ qdelta, uint8_t* __restrict__ out_lut, float* __restrict__ out_delta,
    float* __restrict__ out_B) {
  constexpr int HALVES = item_queries<W>() / 8;
  constexpr int MP = W * 8;
  __shared__ uint16_t lut16[MP * HALVES * 16 * 8];
  __shared__ float lo[MP];
  __shared__ float sB, sD;
  extern __shared__ __align__(16) unsigned char dyn[];
  const int q = blockIdx.x, p = blockIdx.y;
  const size_t qp = (size_t)q * max_nprobe + p;
  if (p >= nprobe_eff[q]) return;  // uniform over the wave
  const int ln = threadIdx.x;
  uint8_t* out = out_lut + qp * t.m * KSUB;
  if (t.metric == IVF_METRIC_IP) {
    for (int e = ln; e < t.m * KSUB; e += IVF_WAVE)
      out[e] = qlut[((size_t)q * KSUB + (e & 15)) * t.m_pad + (e >> 4)];
    if (ln == 0) {
      out_delta[qp] = qdelta[q];
      out_B[qp] = qlo_sum[q] + bias[qp];
    }
    return;
  }
  const int l = probes[qp];
  const float* qg = Q + (size_t)q * t.d;
  const float* c = t.cm + (size_t)l * t.d;
  if constexpr (lane_build<W>()) {
    float* cbT = reinterpret_cast<float*>(dyn);  // [16*d'][m_pad], as in the scan kernel
    const int per = KSUB * t.dsub;
    for (int i = ln; i < t.m * per; i += IVF_WAVE) cbT[(i % per) * MP + i / per] = t.codebooks[i];
    __syncthreads();
    if constexpr (MP <= IVF_WAVE)
      wave_build_lut_lanes<W>(t, qg, c, cbT, 0, lut16, &sB, &sD);
    else
      wave_build_lut_lanes2<W, HALVES>(t, qg, c, cbT, 0, lut16, &sB, &sD);
  } else {
    float* rq = reinterpret_cast<float*>(dyn);  // [d] residual query
    float* cb_s = rq + t.d;                     // [m*16*d'] when staged
    for (int i = ln; i < t.d; i += IVF_WAVE) rq[i] = qg[i] - c[i];
    if constexpr (cb_in_lds<W>())
      for (int i = ln; i < t.m * KSUB * t.dsub; i += IVF_WAVE) cb_s[i] = t.codebooks[i];
    __syncthreads();
    wave_build_lut<W>(t, rq, cb_in_lds<W>() ? cb_s : t.codebooks, 0.0f,
                      ItemStore{lut16, 0, HALVES}, lo, &sB, &sD);
  }
  __syncthreads();
  for (int e = ln; e < t.m * KSUB; e += IVF_WAVE)
    out[e] = (uint8_t)lut16[(((e >> 4) * HALVES) * 16 + (e & 15)) * 8];
  if (ln == 0) {
    out_delta[qp] = sD;
    out_B[qp] = sB;
  }
}

template <int W>
static hipError_t launch_lut_export_w(const Tables& t, const float* Q, int32_t nq,
                                      int32_t max_nprobe, const Workspace& w, uint8_t* out_lut,
                                      float* out_delta, float* out_B, hipStream_t s) {
  if (t.metric == IVF_METRIC_IP) {
    // The per-query tables come from the first-list pass, as in the search.
    hipError_t e = launch_scan_plain_ex(t, Q, nq, max_nprobe, 1, w, w.p1, w.thr, nullptr, s);
    if (e != hipSuccess) return e;
  }
  const size_t lds = t.metric == IVF_METRIC_IP ? 0
                     : lane_build<W>()     ? (size_t)W * 8 * KSUB * t.dsub * 4
                                           : (size_t)t.d * 4 +
                                   (cb_in_lds<W>() ? (size_t)t.m * KSUB * t.dsub * 4 : 0);
  hipLaunchKernelGGL(batched_lut_export_kernel<W>, dim3(nq, max_nprobe), dim3(IVF_WAVE), lds, s, t,
                     Q, max_nprobe, w.probes, w.nprobe_eff, w.bias, w.qlut, w.qlo_sum, w.qdelta,
                     out_lut, out_delta, out_B);
  return hipGetLastError();
}

hipError_t launch_debug_batched_luts(const Tables& t, const float* Q, int32_t nq,
                                     int32_t max_nprobe, const Workspace& w, uint8_t* out_lut,
                                     float* out_delta, float* out_B, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  switch (t.words) {
#define X(N) \
  case N: return launch_lut_export_w<N>(t, Q, nq, max_nprobe, w, out_lut, out_delta, out_B, s);
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
    X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24)
#undef X
    default: return hipErrorNotSupported;
  }
}

// Queries whose survivors overflowed in any round: the plain scan again.
hipError_t launch_batched_redo(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                               int32_t R, const Workspace& w, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  return launch_scan_plain_ex(t, Q, nq, max_nprobe, R, w, nullptr, nullptr, w.redo, s);
}

}  // namespace ivf
