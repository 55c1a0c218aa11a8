// Steps 2-4 of the search: lookup table of Eq. (1) per (query, probed list),
// its 8-bit quantisation, the ADC scan of the list's 4-bit codes and the
// candidate pool of the `reorder` best (approximate value, id) keys
// (Alg. 3, brute-force branch: CalculatePQDistances + UpdateNNPool).
//
// Canonical arithmetic (compiled without FP contraction), identical to the
// CPU reference definition:
//   L2   T[j,i] = sum_u (r_{j d'+u} - B[j,i,u])^2, r = q - cm_l, sequential in u
//   IP   T[j,i] = -sum_u q_{j d'+u} B[j,i,u];   bias_l = -<q, cm_l> (sequential)
//   lo_j = min_i T[j,i];  rng = max_j max_i (T[j,i] - lo_j)
//   s = 255 / rng;  delta = rng / 255  (correctly rounded divisions)
//   lut[j,i] = min(255, rint((T[j,i] - lo_j) * s))   (0 everywhere if rng == 0)
//   B = pairwise_sum_j(lo_j) + bias_l
//   a(x) = B + delta * float(sum_j lut[j, code_j(x)])
// The pool keeps the R smallest keys (ord(a) << 32 | id).
#include "common.hpp"
#include "internal.hpp"

namespace ivf {

struct LutState {
  float delta;
  float lo_sum;   // pairwise sum of lo_j
  uint32_t rng_bits;
  uint32_t pad;
};

// Float table of one (query, list) pair (L2) or of the query (IP).
__device__ __forceinline__ void lut_float(const Tables& t, const float* qv, int l, float* Tf) {
  const int ne = t.m * KSUB;
  const int ds = t.dsub;
  if (t.metric == IVF_METRIC_L2) {
    const float* c = t.cm + (size_t)l * t.d;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      const int j = e >> 4;
      const float* cb = t.codebooks + (size_t)e * ds;
      float acc = 0.0f;
      for (int u = 0; u < ds; ++u) {
        float r = qv[j * ds + u] - c[j * ds + u];
        float df = r - cb[u];
        acc = acc + df * df;
      }
      Tf[e] = acc;
    }
  } else {
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      const int j = e >> 4;
      const float* cb = t.codebooks + (size_t)e * ds;
      float acc = 0.0f;
      for (int u = 0; u < ds; ++u) acc = acc + qv[j * ds + u] * cb[u];
      Tf[e] = plus_zero(-acc);
    }
  }
}

// Quantise Tf into lut8 (m_pad*16 bytes), lo[0..m), and publish delta and
// the pairwise sum of lo in `st`. All threads; ends with a barrier.
__device__ __forceinline__ void lut_quantize(const Tables& t, const float* Tf, float* lo,
                                             uint8_t* lut8, LutState* st) {
  const int m = t.m;
  if (threadIdx.x == 0) st->rng_bits = 0u;
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const float* row = Tf + j * KSUB;
    float mn = row[0];
    for (int i = 1; i < KSUB; ++i) mn = fminf(mn, row[i]);
    float mx = 0.0f;
    for (int i = 0; i < KSUB; ++i) mx = fmaxf(mx, row[i] - mn);
    lo[j] = mn;
    atomicMax(&st->rng_bits, __float_as_uint(mx));  // mx >= 0: bit order = value order
  }
  __syncthreads();
  const float rng = __uint_as_float(st->rng_bits);
  const bool live = rng > 0.0f;
  const float s = live ? 255.0f / rng : 0.0f;
  const int ne = t.m_pad * KSUB;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const int j = e >> 4;
    uint8_t v = 0;
    if (live && j < m) {
      float x = rintf((Tf[e] - lo[j]) * s);
      v = (uint8_t)fminf(x, 255.0f);
    }
    lut8[e] = v;
  }
  if (threadIdx.x < IVF_WAVE) {
    float ls = wave_pairwise_sum(lo, m);
    if (threadIdx.x == 0) {
      st->lo_sum = ls;
      st->delta = live ? rng / 255.0f : 0.0f;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Plain form: one workgroup per query, lists visited in coarse order.
// ---------------------------------------------------------------------------

template <int W>
struct ScanShared {
  uint8_t lut8[W * 8 * KSUB];
  float lo[W * 8];
  LutState st;
  SelectScratch sc;
  unsigned long long maxkey;
  uint32_t total;
  uint32_t cnt;
};

// Code words of one 64-point block: word w of this lane's point.
template <int W>
__device__ __forceinline__ void load_words(const Tables& t, int blk, uint32_t (&words)[W]) {
  const uint32_t* cw = t.codes + (size_t)blk * W * BLOCK_PTS + lane_id();
#pragma unroll
  for (int w = 0; w < W; ++w) words[w] = cw[w * BLOCK_PTS];
}

template <int W>
__global__ void __launch_bounds__(256) scan_plain_kernel(Tables t, const float* __restrict__ Q,
                                                         int32_t nq, int32_t max_nprobe,
                                                         int32_t R, int32_t cap,
                                                         const int32_t* __restrict__ probes,
                                                         const int32_t* __restrict__ nprobe_eff,
                                                         float* __restrict__ bias,
                                                         uint64_t* __restrict__ cand,
                                                         int32_t* __restrict__ p1_out,
                                                         uint64_t* __restrict__ thr_out,
                                                         const int32_t* __restrict__ only,
                                                         int32_t first_lists,
                                                         uint8_t* __restrict__ qlut_out,
                                                         float* __restrict__ qlo_out,
                                                         float* __restrict__ qdelta_out,
                                                         const int32_t* __restrict__ order,
                                                         int32_t own_bias) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ ScanShared<W> sh;
  // `order`: the launch order of the queries (longest scan first), or the
  // identity when null.
  const int q = order ? order[blockIdx.x] : blockIdx.x;
  const int tid = threadIdx.x;
  const int wave = tid / IVF_WAVE;
  uint64_t* keys = reinterpret_cast<uint64_t*>(dyn);            // [R + cap]
  float* Tf = reinterpret_cast<float*>(keys + R + cap);          // [m_pad*16]
  float* qv = Tf + t.m_pad * KSUB;                               // [d]
  float* sbias = qv + t.d;                                       // [max_nprobe] (own_bias)
  // `only`: recompute just the flagged queries. `p1_out`: the batched form's
  // first-list pass: stop after the first first_lists lists, or later, once
  // the lists scanned hold at least R points, and publish where phase 2
  // starts and the R-th smallest key (the rounds' first threshold).
  if (only && only[q] == 0) return;
  const int np = nprobe_eff[q];

  // Software pipeline: each wave holds the code words of the next block it
  // will scan (the first one before any table is built, then one ahead,
  // reaching into the next probed list), so global loads overlap the table
  // build, the lookups and the pool maintenance.
  const int32_t* qprobes = probes + (size_t)q * max_nprobe;
  uint32_t nx[W];
  bool have = false;
  if (np > 0) {
    const int l0 = qprobes[0];
    if (wave < (t.list_len[l0] + BLOCK_PTS - 1) / BLOCK_PTS) {
      load_words<W>(t, t.block_off[l0] + wave, nx);
      have = true;
    }
  }
  for (int i = tid; i < t.d; i += blockDim.x) qv[i] = Q[(size_t)q * t.d + i];
  if (tid == 0) sh.total = 0;
  __syncthreads();
  // `own_bias` (inner product): the list constants -<q, cm_l> of every probe
  // slot are computed here, one thread per slot, kept in LDS for this scan
  // and published for the batched scan's work items. The table build below
  // ends with barriers before any list is scanned.
  if (own_bias) {
    for (int p = tid; p < np; p += blockDim.x) {
      const float b = ip_list_bias(t.cm + (size_t)qprobes[p] * t.d, qv, t.d);
      sbias[p] = b;
      bias[(size_t)q * max_nprobe + p] = b;
    }
  }

  uint64_t thr = KEY_NONE;
  const uint32_t limit = (uint32_t)(R + cap - IVF_BLOCK);
  const bool ip = t.metric == IVF_METRIC_IP;
  if (ip && np > 0) {
    lut_float(t, qv, 0, Tf);
    __syncthreads();
    lut_quantize(t, Tf, sh.lo, sh.lut8, &sh.st);
    if (qlut_out) {
      // First-list pass of the batched form: publish the query's table for
      // the list-major scan (code-major: entry (j, c) at c * m_pad + j).
      uint8_t* dst = qlut_out + (size_t)q * KSUB * t.m_pad;
      for (int e = tid; e < t.m_pad * KSUB; e += blockDim.x)
        dst[e] = sh.lut8[(e % t.m_pad) * KSUB + e / t.m_pad];
      if (tid == 0) {
        qlo_out[q] = sh.st.lo_sum;
        qdelta_out[q] = sh.st.delta;
      }
    }
  }
  const int lane = lane_id();
  int seen = 0, p_end = np;
  for (int p = 0; p < np; ++p) {
    if (p1_out && seen >= R && p >= first_lists) {
      p_end = p;
      break;
    }
    const int l = qprobes[p];
    const int l_next = p + 1 < np ? qprobes[p + 1] : -1;
    const int nblk_next = l_next >= 0 ? (t.list_len[l_next] + BLOCK_PTS - 1) / BLOCK_PTS : 0;
    const int blk0_next = l_next >= 0 ? t.block_off[l_next] : 0;
    float b = 0.0f;
    if (!ip) {
      lut_float(t, qv, l, Tf);
      __syncthreads();
      lut_quantize(t, Tf, sh.lo, sh.lut8, &sh.st);
    } else {
      b = own_bias ? sbias[p] : bias[(size_t)q * max_nprobe + p];
    }
    const float B = sh.st.lo_sum + b;
    const float delta = sh.st.delta;
    const int n_l = t.list_len[l];
    seen += n_l;
    const int blk0 = t.block_off[l];
    const int nblk = (n_l + BLOCK_PTS - 1) / BLOCK_PTS;
    for (int b0 = 0; b0 < nblk; b0 += IVF_NWAVES) {
      const int bi = b0 + wave;
      if (bi < nblk) {
        if (!have) load_words<W>(t, blk0 + bi, nx);
        uint32_t cur[W];
#pragma unroll
        for (int w = 0; w < W; ++w) cur[w] = nx[w];
        // Request the wave's next block now, without branching (a branch
        // makes the compiler wait for these loads before the lookups); when
        // there is none, the current block is read again and not used.
        const bool more = bi + IVF_NWAVES < nblk;
        have = more || wave < nblk_next;
        load_words<W>(t, more ? blk0 + bi + IVF_NWAVES
                              : (wave < nblk_next ? blk0_next + wave : blk0 + bi), nx);
        uint32_t S = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const uint32_t x = cur[w];
#pragma unroll
          for (int s8 = 0; s8 < 8; ++s8)
            S += sh.lut8[(w * 8 + s8) * KSUB + ((x >> (4 * s8)) & 15u)];
        }
        const bool valid = bi * BLOCK_PTS + lane < n_l;
        const float a = plus_zero(B + delta * (float)S);
        const uint32_t oa = f2ord(a);
        const bool maybe = valid && oa <= (uint32_t)(thr >> 32);
        const uint32_t id = maybe ? (uint32_t)t.slot_ids[(size_t)(blk0 + bi) * BLOCK_PTS + lane] : 0u;
        const uint64_t key = ((uint64_t)oa << 32) | id;
        wave_append(maybe && key <= thr, key, keys, &sh.total);
      }
      __syncthreads();
      const uint32_t total = sh.total;
      if (total > limit) {
        KeyUnion u{keys, total, nullptr, 0};
        thr = block_kth(u, (uint32_t)R, &sh.sc);
        const uint32_t kept = block_compact_le(keys, total, thr, &sh.cnt);
        if (tid == 0) sh.total = kept < (uint32_t)R ? kept : (uint32_t)R;
        __syncthreads();
      }
    }
    __syncthreads();  // the table is rebuilt for the next list
  }
  uint32_t total = sh.total;
  if (total > (uint32_t)R) {
    KeyUnion u{keys, total, nullptr, 0};
    thr = block_kth(u, (uint32_t)R, &sh.sc);
    total = block_compact_le(keys, total, thr, &sh.cnt);
    if (total > (uint32_t)R) total = (uint32_t)R;
  }
  if (p1_out) {
    // First-list pass of the batched form: the pool unsorted (the merge
    // sorts) and its largest key, the exact R-th smallest, as threshold.
    if (tid == 0) sh.maxkey = 0;
    __syncthreads();
    uint64_t mk = 0;
    for (uint32_t i = tid; i < total; i += blockDim.x) mk = keys[i] > mk ? keys[i] : mk;
    if (mk) atomicMax(&sh.maxkey, (unsigned long long)mk);
    for (int i = tid; i < R; i += blockDim.x)
      cand[(size_t)q * R + i] = (uint32_t)i < total ? keys[i] : KEY_NONE;
    __syncthreads();
    if (tid == 0) {
      p1_out[q] = np > 0 ? p_end : 0;
      thr_out[q] = total >= (uint32_t)R ? (uint64_t)sh.maxkey : KEY_NONE;
    }
    return;
  }
  // The pool in any order (the re-rank orders its own results; the parity
  // export sorts it).
  for (int i = tid; i < R; i += blockDim.x)
    cand[(size_t)q * R + i] = (uint32_t)i < total ? keys[i] : KEY_NONE;
}

// Ascending order of every query's candidate keys (parity export only).
__global__ void __launch_bounds__(256) sort_rows_kernel(uint64_t* __restrict__ cand, int32_t R) {
  extern __shared__ __align__(16) unsigned char dyn[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(dyn);
  const int q = blockIdx.x;
  const uint32_t n2 = pow2_ceil((uint32_t)R);
  for (uint32_t i = threadIdx.x; i < n2; i += blockDim.x)
    keys[i] = i < (uint32_t)R ? cand[(size_t)q * R + i] : KEY_NONE;
  block_bitonic_sort(keys, n2);
  for (int i = threadIdx.x; i < R; i += blockDim.x) cand[(size_t)q * R + i] = keys[i];
}

hipError_t launch_sort_rows(uint64_t* cand, int32_t nq, int32_t R, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(sort_rows_kernel, dim3(nq), dim3(256), (size_t)pow2_ceil((uint32_t)R) * 8, s,
                     cand, R);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Longest-first launch order of the per-query scans. A query's scan length
// is the number of list entries it will visit (for the batched form's
// first-list pass, up to its stop rule); queries are bucketed by it on a log
// scale, 32 buckets per octave, and a counting sort over the buckets gives
// the workgroup order. Long scans then start first and the grid ends with
// short ones. Only the schedule changes: each query's pool is the same.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int order_bucket(uint64_t len) {
  const uint32_t w = len > 0xffffffffull ? 0xffffffffu : (uint32_t)len;
  if (w == 0) return ORDER_BUCKETS - 1;
  const int e = 31 - __clz((int)w);
  const uint32_t f = e >= 5 ? (w >> (e - 5)) & 31u : (w << (5 - e)) & 31u;
  return ORDER_BUCKETS - 1 - (e * 32 + (int)f);  // e * 32 + f <= 1023
}

// One thread per query: the points of the lists its scan will visit (for
// the first-list pass, up to its stop rule).
__global__ void __launch_bounds__(256) order_count_kernel(Tables t, int32_t nq, int32_t max_nprobe,
                                                          const int32_t* __restrict__ probes,
                                                          const int32_t* __restrict__ nprobe_eff,
                                                          int32_t first_lists, int32_t R,
                                                          int32_t* __restrict__ bucket,
                                                          int32_t* __restrict__ hist) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const int np = nprobe_eff[q];
  const int32_t* qprobes = probes + (size_t)q * max_nprobe;
  uint64_t seen = 0;
  for (int p = 0; p < np; ++p) {
    if (first_lists > 0 && seen >= (uint64_t)R && p >= first_lists) break;
    seen += (uint32_t)t.list_len[qprobes[p]];
  }
  const int b = order_bucket(seen);
  bucket[q] = b;
  atomicAdd(&hist[b], 1);
}

// Each workgroup scans the bucket counts in LDS, then places its queries:
// position = start of the bucket + a global per-bucket cursor.
__global__ void __launch_bounds__(256) order_place_kernel(int32_t nq,
                                                          const int32_t* __restrict__ bucket,
                                                          const int32_t* __restrict__ hist,
                                                          int32_t* __restrict__ cursor,
                                                          int32_t* __restrict__ order) {
  constexpr int PER = ORDER_BUCKETS / 256;
  __shared__ int32_t part[256];
  __shared__ int32_t start[ORDER_BUCKETS];
  const int tid = threadIdx.x;
  int32_t c[PER], sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    c[i] = hist[tid * PER + i];
    sum += c[i];
  }
  part[tid] = sum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int32_t a = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += a;
    __syncthreads();
  }
  int32_t acc = part[tid] - sum;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    start[tid * PER + i] = acc;
    acc += c[i];
  }
  __syncthreads();
  const int q = blockIdx.x * blockDim.x + tid;
  if (q < nq) {
    const int b = bucket[q];
    order[start[b] + atomicAdd(&cursor[b], 1)] = q;
  }
}

static hipError_t launch_scan_order(const Tables& t, int32_t nq, int32_t max_nprobe,
                                    int32_t first_lists, int32_t R, const Workspace& w,
                                    hipStream_t s) {
  hipError_t e = launch_fill_u32((uint32_t*)w.order_hist, 0u, (size_t)2 * ORDER_BUCKETS, s);
  if (e != hipSuccess) return e;
  const unsigned g = (unsigned)((nq + 255) / 256);
  hipLaunchKernelGGL(order_count_kernel, dim3(g), dim3(256), 0, s, t, nq, max_nprobe, w.probes,
                     w.nprobe_eff, first_lists, R, w.order_bucket, w.order_hist);
  hipLaunchKernelGGL(order_place_kernel, dim3(g), dim3(256), 0, s, nq, w.order_bucket,
                     w.order_hist, w.order_hist + ORDER_BUCKETS, w.order);
  return hipGetLastError();
}

// Candidate-buffer slack beyond R (keys): the requested size (default 1024),
// at least one round of one block per wave.
inline int32_t scan_cap(int32_t R, int32_t requested) {
  (void)R;
  int32_t cap = requested > 0 ? requested : 1024;
  if (cap < IVF_BLOCK) cap = IVF_BLOCK;
  return cap;
}

template <int W>
static hipError_t launch_scan_plain_w(const Tables& t, const float* Q, int32_t nq,
                                      int32_t max_nprobe, int32_t R, const Workspace& w,
                                      int32_t* p1_out, uint64_t* thr_out, const int32_t* only,
                                      hipStream_t s) {
  const int32_t cap = scan_cap(R, w.pool_cap);
  // Inner product: the kernel computes the list constants itself unless it
  // only recomputes flagged queries (their constants are in place already).
  const bool own_bias = scan_owns_bias(t, max_nprobe) && !only;
  size_t lds = (size_t)(R + cap) * 8 + (size_t)t.m_pad * KSUB * 4 + (size_t)t.d * 4 +
               (own_bias ? (size_t)max_nprobe * 4 : 0);
  const bool pub = p1_out && t.metric == IVF_METRIC_IP;
  const int32_t first_lists = w.first_lists > 0 ? w.first_lists : 1;
  // A recompute of flagged queries (`only`) keeps the identity order.
  const bool ordered = !only && w.order && w.query_order == 0;
  if (ordered) {
    const hipError_t e = launch_scan_order(t, nq, max_nprobe, p1_out ? first_lists : 0, R, w, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(scan_plain_kernel<W>, dim3(nq), dim3(256), lds, s, t, Q, nq, max_nprobe, R,
                     cap, w.probes, w.nprobe_eff, w.bias, w.cand, p1_out, thr_out, only,
                     first_lists, pub ? w.qlut : nullptr, pub ? w.qlo_sum : nullptr,
                     pub ? w.qdelta : nullptr, ordered ? w.order : nullptr, own_bias ? 1 : 0);
  return hipGetLastError();
}

#define IVF_W_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) \
  X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

hipError_t launch_scan_plain_ex(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                                int32_t rerank, const Workspace& w, int32_t* p1_out,
                                uint64_t* thr_out, const int32_t* only, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  switch (t.words) {
#define X(N) \
  case N:    \
    return launch_scan_plain_w<N>(t, Q, nq, max_nprobe, rerank, w, p1_out, thr_out, only, s);
    IVF_W_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_scan_plain(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                             int32_t rerank, const Workspace& w, hipStream_t s) {
  return launch_scan_plain_ex(t, Q, nq, max_nprobe, rerank, w, nullptr, nullptr, nullptr, s);
}

// ---------------------------------------------------------------------------
// Parity export of step 2: the quantised table of each (query, probed list).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) debug_lut_kernel(Tables t, const float* __restrict__ Q,
                                                        int32_t max_nprobe,
                                                        const int32_t* __restrict__ probes,
                                                        const int32_t* __restrict__ nprobe,
                                                        uint8_t* out_lut, float* out_lo,
                                                        float* out_delta, float* out_B) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ uint8_t lut8[MAX_M * KSUB];
  __shared__ float lo[MAX_M];
  __shared__ LutState st;
  const int q = blockIdx.x, p = blockIdx.y;
  const size_t qp = (size_t)q * max_nprobe + p;
  if (p >= nprobe[q] || probes[qp] < 0 || probes[qp] >= t.L) return;
  float* Tf = reinterpret_cast<float*>(dyn);
  float* qv = Tf + t.m_pad * KSUB;
  // Filtered index: the kept components of the d_base-wide query.
  for (int i = threadIdx.x; i < t.d; i += blockDim.x)
    qv[i] = Q[(size_t)q * t.d_base + (t.dims ? t.dims[i] : i)];
  __syncthreads();
  const int l = probes[qp];
  lut_float(t, qv, l, Tf);
  __syncthreads();
  lut_quantize(t, Tf, lo, lut8, &st);
  float b = 0.0f;
  if (t.metric == IVF_METRIC_IP) {  // -<q, cm_l>, sequential over t
    const float* c = t.cm + (size_t)l * t.d;
    for (int k = 0; k < t.d; ++k) b = b + qv[k] * c[k];
    b = plus_zero(-b);
  }
  for (int e = threadIdx.x; e < t.m * KSUB; e += blockDim.x) out_lut[qp * t.m * KSUB + e] = lut8[e];
  for (int j = threadIdx.x; j < t.m; j += blockDim.x) out_lo[qp * t.m + j] = lo[j];
  if (threadIdx.x == 0) {
    out_delta[qp] = st.delta;
    out_B[qp] = st.lo_sum + b;
  }
}

hipError_t launch_debug_luts(const Tables& t, const float* Q, int32_t nq, const int32_t* probes,
                             const int32_t* nprobe, int32_t max_nprobe, uint8_t* out_lut, float* out_lo, float* out_delta, float* out_B,
                             hipStream_t s) {
  if (nq == 0) return hipSuccess;
  size_t lds = (size_t)t.m_pad * KSUB * 4 + (size_t)t.d * 4;
  hipLaunchKernelGGL(debug_lut_kernel, dim3(nq, max_nprobe), dim3(256), lds, s, t, Q, max_nprobe,
                     probes, nprobe, out_lut, out_lo, out_delta, out_B);
  return hipGetLastError();
}

}  // namespace ivf
