// Step 1 of the search (Alg. 2, TopNClusters): coarse scores of every query
// against the list centroids, and the nprobe nearest lists per query.
//
// The canonical score, which fixes the probe sets bit for bit, is
//   L2: s = sum_t (q_t - c_t)^2      IP: s = -sum_t q_t c_t
// summed sequentially over t in FP32 with every product and sum rounded on
// its own (this file is compiled without FP contraction). Smaller is nearer;
// ties go to the smaller list index.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"
#include "rank_sort.hpp"

namespace ivf {

constexpr int CQ = 32;   // queries per tile
constexpr int CL = 64;   // lists per tile
constexpr int CD = 32;   // dimensions staged per step

// One workgroup per (32-query x 64-list) tile; each thread owns 2 queries x
// 4 lists and walks t in order, so every score is the canonical seq-sum.
__global__ void __launch_bounds__(256) coarse_exact_kernel(Tables t, const float* __restrict__ Q,
                                                           int32_t nq, float* __restrict__ S) {
  __shared__ float qs[CQ][CD + 1];
  __shared__ float cs[CL][CD + 1];
  const int tid = threadIdx.x;
  const int l0 = blockIdx.x * CL, q0 = blockIdx.y * CQ;
  const int tq = (tid / 16) * 2;   // 0..30
  const int tl = (tid % 16);       // lists tl, tl+16, tl+32, tl+48
  const bool ip = t.metric == IVF_METRIC_IP;
  float acc[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  for (int d0 = 0; d0 < t.d; d0 += CD) {
    const int dn = min(CD, t.d - d0);
    __syncthreads();
    for (int e = tid; e < CQ * CD; e += 256) {
      int r = e / CD, c = e % CD;
      int q = q0 + r;
      qs[r][c] = (q < nq && c < dn) ? Q[(size_t)q * t.d + d0 + c] : 0.0f;
    }
    for (int e = tid; e < CL * CD; e += 256) {
      int r = e / CD, c = e % CD;
      int l = l0 + r;
      cs[r][c] = (l < t.L && c < dn) ? t.cp[(size_t)l * t.d + d0 + c] : 0.0f;
    }
    __syncthreads();
    for (int c = 0; c < dn; ++c) {
      float qv0 = qs[tq][c], qv1 = qs[tq + 1][c];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float cv = cs[tl + 16 * j][c];
        if (ip) {
          acc[0][j] = acc[0][j] + qv0 * cv;
          acc[1][j] = acc[1][j] + qv1 * cv;
        } else {
          float d0v = qv0 - cv, d1v = qv1 - cv;
          acc[0][j] = acc[0][j] + d0v * d0v;
          acc[1][j] = acc[1][j] + d1v * d1v;
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    int q = q0 + tq + i;
    if (q >= nq) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int l = l0 + tl + 16 * j;
      if (l < t.L) S[(size_t)q * t.L + l] = ip ? plus_zero(-acc[i][j]) : acc[i][j];
    }
  }
}

hipError_t launch_coarse_exact(const Tables& t, const float* Q, int32_t nq, float* scores,
                               hipStream_t s) {
  dim3 grid((t.L + CL - 1) / CL, (nq + CQ - 1) / CQ);
  hipLaunchKernelGGL(coarse_exact_kernel, grid, dim3(256), 0, s, t, Q, nq, scores);
  return hipGetLastError();
}

// Sequential FP32 sum over t = 0..d-1 of q_t c_t (IP) or (q_t - c_t)^2
// (L2), one thread. Rows are fetched in 16-byte vectors when d is a multiple
// of 4, 16 vectors (64 floats) requested before any is used, since the rows
// come from the caches with long latency; the accumulation order is the
// same in both paths.
template <bool IP>
__device__ __forceinline__ float seq_row_sum(const float* q, const float* c, int d) {
  float acc = 0.0f;
  int i = 0;
  if ((d & 3) == 0) {
    constexpr int NV = 16;
    const float4* c4 = reinterpret_cast<const float4*>(c);
    for (; i < d; i += 4 * NV) {
      float4 v[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k)
        v[k] = i + 4 * k < d ? c4[(i >> 2) + k] : make_float4(0, 0, 0, 0);
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const float cv[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int ii = i + 4 * k + e;
          if (ii < d) {
            if (IP) {
              acc = acc + q[ii] * cv[e];
            } else {
              const float df = q[ii] - cv[e];
              acc = acc + df * df;
            }
          }
        }
      }
    }
  } else {
    for (; i < d; ++i) {
      if (IP) {
        acc = acc + q[i] * c[i];
      } else {
        const float df = q[i] - c[i];
        acc = acc + df * df;
      }
    }
  }
  return acc;
}

// Canonical score of one (query, list) pair against the probe centroid.
__device__ __forceinline__ float canonical_score(const Tables& t, const float* q, int l) {
  const float* c = t.cp + (size_t)l * t.d;
  if (t.metric == IVF_METRIC_IP) return plus_zero(-seq_row_sum<true>(q, c, t.d));
  return seq_row_sum<false>(q, c, t.d);
}

// Eq. 2 (section 4.2) in FP32, in the order written: the adaptive count
// between v_min (clamped to [1, v_max]) and v_max for hardness p.
__device__ __forceinline__ int32_t eq2_count(float p, int32_t vmin, int32_t vmax, float p0,
                                             float p1) {
  vmin = vmin < 1 ? 1 : (vmin > vmax ? vmax : vmin);
  const float relu = fmaxf(p - p0, 0.0f);
  const float g = relu * (p + p1);
  const float span = (float)(vmax - vmin);
  const float x = fminf(span * g, span + 1.0f);  // caps the conversion only
  const int32_t v = vmin + (int32_t)floorf(x);
  return v < vmax ? v : vmax;
}

// The `want` smallest (ord(score), list) keys of one score row, held NK per
// thread in registers (list = tid + 256 i), written to keys[0..want) in no
// particular order. The want-th smallest ord is found by 4-bit radix passes
// from the top. Each thread counts its keys per digit in 8-bit fields (four
// u32, digit d in byte d % 4 of word d / 4); the fields are then spread to
// 16-bit ones and summed over the wave by a transposing butterfly (every
// exchange hands half of the remaining counters to the partner lane, so 10
// exchanges instead of 48), and across the four waves by 16 lanes of wave
// 0, which also scan them and pick the digit: no LDS atomic serialises on a
// popular digit. The passes stop as soon as the chosen digit holds exactly
// the keys still needed (then every key whose top bits are at most the
// prefix is taken); after all eight, keys equal to the want-th ord are taken
// in ascending list order, each one's rank among them counted with ballots.
// All threads; ends with a barrier. Needs want <= the number of keys (ord
// 0xffffffff marks a missing key; finite scores never map to it).
template <int NK>
__device__ void row_select(const uint32_t (&o)[NK], int want, uint64_t* keys, uint32_t* cnt) {
  static_assert(NK <= 64, "per-thread digit counts must fit 8 bits, wave sums 16 bits");
  // wsum[wave][v]: 16-bit wave sums; word 2k holds digits 4k (low half) and
  // 4k + 2 (high half), word 2k + 1 digits 4k + 1 and 4k + 3.
  __shared__ uint32_t wsum[IVF_NWAVES][8];
  __shared__ uint32_t rowc[NK][IVF_NWAVES];
  __shared__ uint32_t pick[3];  // digit, keys below it, 1 = the digit holds exactly the rest
  const int tid = threadIdx.x, wave = tid / IVF_WAVE, ln = lane_id();
  const bool b5 = (ln & 32) != 0, b4 = (ln & 16) != 0, b3 = (ln & 8) != 0;
  uint32_t prefix = 0, pmask = 0;
  uint32_t need = (uint32_t)want;
  bool exact = false;  // stopped early: take every key with (o & pmask) <= prefix
  for (int shift = 28; shift >= 0; shift -= 4) {
    uint32_t c4[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const uint32_t v = o[i];
      if (v != 0xffffffffu && (v & pmask) == prefix) {
        const uint32_t d = (v >> shift) & 15u;
        const uint32_t inc = 1u << ((d & 3u) << 3);
#pragma unroll
        for (int k = 0; k < 4; ++k) c4[k] += (d >> 2) == (uint32_t)k ? inc : 0u;
      }
    }
    uint32_t c[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      c[2 * k] = c4[k] & 0x00ff00ffu;
      c[2 * k + 1] = (c4[k] >> 8) & 0x00ff00ffu;
    }
    // Transposing butterfly: after xor 32, 16 and 8, lane ln holds word
    // ln >> 3 summed over the eight lanes that differ from it in bits 5..3;
    // xor 4, 2 and 1 complete the wave sum.
    uint32_t h4[4], h2[2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      h4[i] = (b5 ? c[i + 4] : c[i]) + (uint32_t)__shfl_xor((int)(b5 ? c[i] : c[i + 4]), 32);
#pragma unroll
    for (int i = 0; i < 2; ++i)
      h2[i] = (b4 ? h4[i + 2] : h4[i]) + (uint32_t)__shfl_xor((int)(b4 ? h4[i] : h4[i + 2]), 16);
    uint32_t h1 = (b3 ? h2[1] : h2[0]) + (uint32_t)__shfl_xor((int)(b3 ? h2[0] : h2[1]), 8);
#pragma unroll
    for (int s = 4; s >= 1; s >>= 1) h1 += (uint32_t)__shfl_xor((int)h1, s);
    if ((ln & 7) == 0) wsum[wave][ln >> 3] = h1;
    __syncthreads();
    if (wave == 0) {
      // Lane d < 16: the count of digit d; inclusive scan over the 16 lanes.
      const uint32_t d = (uint32_t)(ln & 15);
      const uint32_t word = ((d >> 2) << 1) | (d & 1u), half = ((d >> 1) & 1u) << 4;
      uint32_t cd = 0;
#pragma unroll
      for (int w = 0; w < IVF_NWAVES; ++w) cd += (wsum[w][word] >> half) & 0xffffu;
      if (ln >= 16) cd = 0;
      uint32_t incl = cd;
      for (int off = 1; off < 16; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off);
        if (ln >= off) incl += v;
      }
      const uint64_t hit = __ballot(ln < 16 && incl >= need);
      const int b = hit ? __builtin_ctzll(hit) : 15;
      if (ln == b) {
        pick[0] = (uint32_t)b;
        pick[1] = incl - cd;
        pick[2] = incl == need ? 1u : 0u;
      }
    }
    __syncthreads();
    need -= pick[1];
    prefix |= pick[0] << shift;
    pmask |= 15u << shift;
    exact = pick[2] != 0;
    __syncthreads();  // wsum and pick are rewritten by the next pass
    if (exact) break;  // uniform
  }
  if (tid == 0) *cnt = 0;
  if (exact) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const bool take = o[i] != 0xffffffffu && (o[i] & pmask) <= prefix;
      wave_append(take, ((uint64_t)o[i] << 32) | (uint32_t)(tid + IVF_BLOCK * i), keys, cnt);
    }
    __syncthreads();
    return;
  }
  const uint32_t tord = prefix;  // the want-th smallest ord; `need` keys equal to it are taken
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    const uint64_t m = __ballot(o[i] == tord);
    if (ln == 0) rowc[i][wave] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  uint32_t before_rows = 0;  // equal keys in rows < i (all waves)
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    const bool eq = o[i] == tord;
    const uint64_t m = __ballot(eq);
    uint32_t rank = before_rows + lanes_below(m);
    for (int w = 0; w < wave; ++w) rank += rowc[i][w];
    const bool take = o[i] < tord || (eq && rank < need);
    wave_append(take, ((uint64_t)o[i] << 32) | (uint32_t)(tid + IVF_BLOCK * i), keys, cnt);
    for (int w = 0; w < IVF_NWAVES; ++w) before_rows += rowc[i][w];
  }
  __syncthreads();
}

// Second half of the selection, shared by both kernels: keys[0..n) hold the
// first selection. With `rescore` they are re-scored canonically and, unless
// n <= 256 (then the whole set is sorted and its first np keys used), cut to
// the np best; then they are sorted (by rank into the free space behind them
// when n <= 512 and 2n <= cap, else bitonic), the adaptive counts are taken
// from the sorted scores, and the probe row is written.
__device__ void select_finish(const Tables& t, const float* __restrict__ Q, int q, int np,
                              int max_nprobe, int rescore, uint64_t* keys, uint32_t n,
                              uint32_t cap, SelectScratch* sc, uint32_t* cnt, float* qv,
                              const AdaptiveArgs& ad, int32_t* __restrict__ probes,
                              int32_t* __restrict__ nprobe_eff,
                              int32_t* __restrict__ reorder_eff) {
  const int tid = threadIdx.x;
  if (rescore) {
    // Canonical FP32 re-score of the kept lists; the query is staged in LDS
    // when it fits, else read from global memory.
    const float* qg = Q + (size_t)q * t.d;
    const bool staged = t.d <= 1024;
    if (staged)
      for (int i = tid; i < t.d; i += blockDim.x) qv[i] = qg[i];
    __syncthreads();
    for (uint32_t i = tid; i < n; i += blockDim.x) {
      int l = (int)(uint32_t)keys[i];
      keys[i] = make_key(canonical_score(t, staged ? qv : qg, l), (uint32_t)l);
    }
    __syncthreads();
    // A short widened set is sorted whole below: its first np keys are the
    // np best. A longer one is cut to np first.
    const bool sort_whole = n <= 256 && 2 * n <= cap;
    if ((uint32_t)np < n && !sort_whole) {
      KeyUnion u{keys, n, nullptr, 0};
      n = block_compact_le(keys, n, block_kth(u, (uint32_t)np, sc), cnt);
    }
  }
  const uint64_t* sorted = keys;
  if (n <= 512 && 2 * n <= cap) {
    __syncthreads();
    block_rank_sort(keys, n, keys + n);
    sorted = keys + n;
  } else {
    const uint32_t n2 = pow2_ceil(n);
    for (uint32_t i = n + tid; i < n2; i += blockDim.x) keys[i] = KEY_NONE;
    block_bitonic_sort(keys, n2);
  }
  // Adaptive probe count and re-rank size from the sorted canonical scores.
  __shared__ int32_t np_used;
  if (tid == 0) {
    int32_t npu = np, reo = ad.R;
    if (ad.on) {
      const int K = ad.nprobe_init < 1 ? 1 : (ad.nprobe_init > np ? np : ad.nprobe_init);
      const bool ip = t.metric == IVF_METRIC_IP;
      const float s1 = ord2f((uint32_t)(sorted[0] >> 32));
      const float sK = ord2f((uint32_t)(sorted[K - 1] >> 32));
      const float e1 = ip ? 1.0f + s1 : s1;
      const float eK = ip ? 1.0f + sK : sK;
      float p = eK > 0.0f ? e1 / eK : 1.0f;
      if (!(p >= 0.0f)) p = p < 0.0f ? 0.0f : 1.0f;
      p = fminf(p, 1.0f);
      npu = eq2_count(p, ad.nprobe_min, np, ad.p0, ad.p1);
      const int32_t rmin = ad.reorder_min < ad.k ? ad.k
                                                 : (ad.reorder_min > ad.R ? ad.R : ad.reorder_min);
      reo = eq2_count(p, rmin, ad.R, ad.p0, ad.p1);
    }
    np_used = npu;
    nprobe_eff[q] = npu;
    if (reorder_eff) reorder_eff[q] = reo;
  }
  __syncthreads();
  const int npu = np_used;
  for (int p = tid; p < max_nprobe; p += blockDim.x)
    probes[(size_t)q * max_nprobe + p] = p < npu ? (int32_t)(uint32_t)sorted[p] : -1;
}

// A request with nprobe out of range: error word, -1 row. True if invalid.
__device__ __forceinline__ bool reject_row(int q, int np, int max_nprobe,
                                           int32_t* __restrict__ probes,
                                           int32_t* __restrict__ nprobe_eff,
                                           int32_t* __restrict__ err,
                                           int32_t* __restrict__ reorder_eff) {
  if (np >= 1 && np <= max_nprobe) return false;
  if (threadIdx.x == 0) {
    nprobe_eff[q] = -1;
    if (reorder_eff) reorder_eff[q] = -1;
    atomicOr(err, 1);
  }
  for (int p = threadIdx.x; p < max_nprobe; p += blockDim.x) probes[(size_t)q * max_nprobe + p] = -1;
  return true;
}

// One workgroup per query, 1024 < L <= 2048: the keys (ord(score) << 32 |
// list) of the whole row in LDS ([cap] = pow2(L) slots) and the wanted count
// picked by the byte-wise radix selection of common.hpp.
__global__ void __launch_bounds__(256) select_lds_kernel(Tables t, const float* __restrict__ Q,
                                                         int32_t nq, const int32_t* __restrict__ nprobe,
                                                         int32_t max_nprobe, int32_t widen,
                                                         int32_t widen_add, int32_t rescore,
                                                         const float* __restrict__ S,
                                                         int32_t* __restrict__ probes,
                                                         int32_t* __restrict__ nprobe_eff,
                                                         int32_t* __restrict__ err, AdaptiveArgs ad,
                                                         int32_t* __restrict__ reorder_eff,
                                                         uint32_t cap) {
  extern __shared__ uint64_t keys[];
  __shared__ SelectScratch sc;
  __shared__ float qv[1024];
  __shared__ uint32_t cnt;
  const int q = blockIdx.x;
  const int L = t.L;
  const int np = nprobe[q];
  if (reject_row(q, np, max_nprobe, probes, nprobe_eff, err, reorder_eff)) return;
  const float* srow = S + (size_t)q * L;
  const int want = rescore ? (int)min((int64_t)L, (int64_t)np * widen + widen_add) : np;
  for (int l = threadIdx.x; l < L; l += blockDim.x) keys[l] = make_key(srow[l], (uint32_t)l);
  __syncthreads();
  uint32_t n = (uint32_t)L;
  if ((uint32_t)want < n) {
    KeyUnion u{keys, n, nullptr, 0};
    n = block_compact_le(keys, n, block_kth(u, (uint32_t)want, &sc), &cnt);
  }
  select_finish(t, Q, q, np, max_nprobe, rescore, keys, n, cap, &sc, &cnt, qv, ad, probes,
                nprobe_eff, reorder_eff);
}

// One workgroup per query, L <= 1024 or L > 2048: the row stays in
// registers (NK keys per thread, row_select) and LDS holds only the selection
// ([cap] = the largest selection rounded up to a power of two, doubled up to
// 512 for the rank sort's output).
template <int NK>
__global__ void __launch_bounds__(256) select_kernel(Tables t, const float* __restrict__ Q,
                                                     int32_t nq, const int32_t* __restrict__ nprobe,
                                                     int32_t max_nprobe, int32_t widen,
                                                     int32_t widen_add, int32_t rescore,
                                                     const float* __restrict__ S,
                                                     int32_t* __restrict__ probes,
                                                     int32_t* __restrict__ nprobe_eff,
                                                     int32_t* __restrict__ err,
                                                     AdaptiveArgs ad,
                                                     int32_t* __restrict__ reorder_eff,
                                                     uint32_t cap) {
  extern __shared__ uint64_t keys[];
  __shared__ SelectScratch sc;
  __shared__ float qv[1024];
  __shared__ uint32_t cnt;
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  const int L = t.L;
  const int np = nprobe[q];
  if (reject_row(q, np, max_nprobe, probes, nprobe_eff, err, reorder_eff)) return;
  const float* srow = S + (size_t)q * L;
  const int want = rescore ? (int)min((int64_t)L, (int64_t)np * widen + widen_add) : np;
  uint32_t o[NK];
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    const int l = tid + IVF_BLOCK * i;
    o[i] = l < L ? f2ord(srow[l]) : 0xffffffffu;
  }
  row_select<NK>(o, want, keys, &cnt);
  select_finish(t, Q, q, np, max_nprobe, rescore, keys, (uint32_t)want, cap, &sc, &cnt, qv, ad,
                probes, nprobe_eff, reorder_eff);
}

hipError_t launch_select_probes(const Tables& t, const float* Q, int32_t nq,
                                const int32_t* nprobe, int32_t max_nprobe, int32_t widen,
                                int32_t widen_add, bool rescore, const Workspace& w,
                                hipStream_t s, const AdaptiveArgs& ad) {
  if (nq == 0) return hipSuccess;
  const int32_t most =
      rescore ? (int32_t)std::min<int64_t>(t.L, (int64_t)max_nprobe * widen + widen_add)
              : max_nprobe;
  const int nk = (t.L + IVF_BLOCK - 1) / IVF_BLOCK;
  // Rows of 1025..2048 lists: the whole row in LDS (measured faster there
  // than the register form); shorter and longer rows: registers, so LDS (and
  // occupancy) depends only on the selection size.
  const bool lds_row = nk > 4 && nk <= 8;
  const uint32_t sel = pow2_ceil((uint32_t)(most > 0 ? most : 1));
  const uint32_t cap = lds_row ? pow2_ceil((uint32_t)t.L) : (sel > 512 ? sel : 2 * sel);
  const size_t lds = (size_t)cap * sizeof(uint64_t);
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(nq), dim3(256), lds, s, t, Q, nq, nprobe, max_nprobe, widen,
                       widen_add,
                       rescore ? 1 : 0, w.scores, w.probes, w.nprobe_eff, w.err, ad,
                       w.reorder_eff, cap);
    return hipGetLastError();
  };
  if (nk <= 4) return go(select_kernel<4>);
  if (nk <= 8) return go(select_lds_kernel);
  if (nk <= 16) return go(select_kernel<16>);
  if (nk <= 32) return go(select_kernel<32>);
  if (nk <= 64) return go(select_kernel<64>);
  return hipErrorInvalidValue;
}

// Caller-given probe sets: validate counts and list indices, copy. The
// used part of a row must name distinct lists in [0, L): a bitmap of the
// lists seen so far (L <= 16384 bits in LDS) finds a repeated one.
__global__ void copy_probes_kernel(const int32_t* __restrict__ probes_in,
                                   const int32_t* __restrict__ nprobe, int32_t nq,
                                   int32_t max_nprobe, int32_t L, int32_t* __restrict__ probes,
                                   int32_t* __restrict__ nprobe_eff, int32_t* __restrict__ err) {
  const int q = blockIdx.x;
  __shared__ int bad;
  __shared__ uint32_t seen[16384 / 32];
  const int words = (L + 31) / 32;
  if (threadIdx.x == 0) bad = 0;
  for (int i = threadIdx.x; i < words; i += blockDim.x) seen[i] = 0u;
  __syncthreads();
  int np = nprobe[q];
  bool okn = np >= 1 && np <= max_nprobe;
  for (int p = threadIdx.x; p < max_nprobe; p += blockDim.x) {
    int l = probes_in[(size_t)q * max_nprobe + p];
    if (okn && p < np) {
      if (l < 0 || l >= L) {
        bad = 1;
      } else {
        const uint32_t bit = 1u << (l & 31);
        if (atomicOr(&seen[l >> 5], bit) & bit) bad = 1;  // listed twice
      }
    }
    probes[(size_t)q * max_nprobe + p] = l;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!okn) atomicOr(err, 1);
    if (bad) atomicOr(err, 2);
    nprobe_eff[q] = (okn && !bad) ? np : -1;
  }
}

hipError_t launch_copy_probes(const int32_t* probes, const int32_t* nprobe, int32_t nq,
                              int32_t max_nprobe, int32_t L, const Workspace& w, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_probes_kernel, dim3(nq), dim3(64), 0, s, probes, nprobe, nq, max_nprobe,
                     L, w.probes, w.nprobe_eff, w.err);
  return hipGetLastError();
}

// Inner-product list constant b = -<q, cm_l> (ip_list_bias: sequential over t,
// FP32, every product and sum rounded on its own) for every probe slot. One
// workgroup per query with the query in LDS; one thread per probe slot walks
// its centroid row. Used where the scan kernel does not compute the
// constants itself (very long probe rows, parity exports).
__global__ void __launch_bounds__(256) bias_kernel(Tables t, const float* __restrict__ Q,
                                                   int32_t max_nprobe,
                                                   const int32_t* __restrict__ probes,
                                                   const int32_t* __restrict__ nprobe_eff,
                                                   float* __restrict__ bias) {
  extern __shared__ __align__(16) float qs[];  // [d]
  const int q = blockIdx.x;
  const int np = nprobe_eff[q];
  if (np <= 0) return;  // uniform
  for (int i = threadIdx.x; i < t.d; i += blockDim.x) qs[i] = Q[(size_t)q * t.d + i];
  __syncthreads();
  // One float4 at a time: the re-score's 16-vector prefetch measured slower
  // here (10M x 768 rows, 4096 queries: 0.1 ms more per search).
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    const int l = probes[(size_t)q * max_nprobe + p];
    bias[(size_t)q * max_nprobe + p] = ip_list_bias(t.cm + (size_t)l * t.d, qs, t.d);
  }
}

hipError_t launch_bias(const Tables& t, const float* Q, int32_t nq, int32_t max_nprobe,
                       const Workspace& w, hipStream_t s) {
  if (t.metric != IVF_METRIC_IP || nq == 0) return hipSuccess;
  hipLaunchKernelGGL(bias_kernel, dim3(nq), dim3(256), (size_t)t.d * 4, s, t, Q, max_nprobe,
                     w.probes, w.nprobe_eff, w.bias);
  return hipGetLastError();
}

// Component filtration (section 4.3): the kept components of each query,
// qf[q][j] = Q[q][dims[j]], for the search steps.
__global__ void gather_queries_kernel(const float* __restrict__ Q, int64_t total, int32_t d,
                                      int32_t d_base, const int32_t* __restrict__ dims,
                                      float* __restrict__ qf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t q = i / d;
  const int j = (int)(i % d);
  qf[i] = Q[q * d_base + dims[j]];
}

hipError_t launch_gather_queries(const Tables& t, const float* Q, int32_t nq, float* qf,
                                 hipStream_t s) {
  const int64_t total = (int64_t)nq * t.d;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_queries_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     Q, total, t.d, t.d_base, t.dims, qf);
  return hipGetLastError();
}

}  // namespace ivf
