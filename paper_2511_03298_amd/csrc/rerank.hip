// Step 5 of the search (Alg. 2, final step): exact distances between the
// query and its candidate rows, FP32 accumulation (BF16 and U8 rows are
// widened exactly), and the top k by (distance, id): ascending squared L2,
// or descending inner product.
#include "common.hpp"
#include "internal.hpp"
#include "rank_sort.hpp"

namespace ivf {

__device__ __forceinline__ float load_base(const Tables& t, int64_t row, int c) {
  if (t.base_dtype == IVF_DTYPE_BF16) {
    const uint16_t* b = reinterpret_cast<const uint16_t*>(t.base);
    return __uint_as_float((uint32_t)b[row * t.d_base + c] << 16);
  }
  if (t.base_dtype == IVF_DTYPE_U8)
    return (float)reinterpret_cast<const uint8_t*>(t.base)[row * t.d_base + c];
  return reinterpret_cast<const float*>(t.base)[row * t.d_base + c];
}

// Sum over one 16-byte vector of the row: 4 FP32 values, or 8 BF16 / 16 U8
// values widened exactly, in element order.
__device__ __forceinline__ float vec_term(const float* qv, const uint4& x, int e0, bool ip,
                                          int dtype) {
  float acc = 0.0f;
  if (dtype == IVF_DTYPE_U8) {
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int h = 0; h < 16; ++h) {
      const float v = (float)((w[h >> 2] >> (8 * (h & 3))) & 0xffu);
      if (ip) {
        acc = acc + qv[e0 + h] * v;
      } else {
        const float df = qv[e0 + h] - v;
        acc = acc + df * df;
      }
    }
  } else if (dtype == IVF_DTYPE_BF16) {
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const float v = __uint_as_float(h & 1 ? (w[h >> 1] & 0xffff0000u) : (w[h >> 1] << 16));
      if (ip) {
        acc = acc + qv[e0 + h] * v;
      } else {
        const float df = qv[e0 + h] - v;
        acc = acc + df * df;
      }
    }
  } else {
    const float v[4] = {__uint_as_float(x.x), __uint_as_float(x.y), __uint_as_float(x.z),
                        __uint_as_float(x.w)};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      if (ip) {
        acc = acc + qv[e0 + h] * v[h];
      } else {
        const float df = qv[e0 + h] - v[h];
        acc = acc + df * df;
      }
    }
  }
  return acc;
}

// One workgroup per query. A candidate row is read by a group of G = 8
// lanes in 16-byte vectors (lane gl takes vectors gl, gl + 8, ...), U rows
// per group at a time, so every lane keeps several loads in flight; the
// group reduces its partial sums with a butterfly in a fixed order. Rows
// whose byte size is not a multiple of 16 take the scalar path.
template <int U>
__global__ void __launch_bounds__(256) rerank_kernel(Tables t, const float* __restrict__ Q,
                                                     int32_t k, int32_t R,
                                                     const int32_t* __restrict__ nprobe_eff,
                                                     const uint64_t* __restrict__ cand,
                                                     const int32_t* __restrict__ reorder,
                                                     int64_t* __restrict__ out_ids,
                                                     float* __restrict__ out_dist) {
  extern __shared__ __align__(16) unsigned char dyn[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(dyn);                   // [pow2(R)]
  float* qv = reinterpret_cast<float*>(keys + pow2_ceil((uint32_t)R));  // [d]
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  const bool ip = t.metric == IVF_METRIC_IP;
  const int dtype = t.base_dtype;
  if (nprobe_eff[q] < 0) {  // invalid request row
    for (int i = tid; i < k; i += blockDim.x) {
      out_ids[(size_t)q * k + i] = -1;
      out_dist[(size_t)q * k + i] = __uint_as_float(0x7fc00000u);
    }
    return;
  }
  for (int i = tid; i < t.d_base; i += blockDim.x) qv[i] = Q[(size_t)q * t.d_base + i];
  // The pool into LDS; with a per-query re-rank size, its `reorder` smallest
  // keys only (the set a pool of that size would hold). Keys are unique apart
  // from the empty-slot value, which sorts last.
  __shared__ SelectScratch sc;
  __shared__ uint32_t cnt;
  for (int i = tid; i < R; i += blockDim.x) keys[i] = cand[(size_t)q * R + i];
  __syncthreads();
  int32_t nc = R;
  if (reorder && reorder[q] < R) {
    KeyUnion u{keys, (uint32_t)R, nullptr, 0};
    const uint64_t thr = block_kth(u, (uint32_t)reorder[q], &sc);
    nc = (int32_t)block_compact_le(keys, (uint32_t)R, thr, &cnt);
  }
  constexpr int G = 8;
  constexpr int GROUPS = IVF_BLOCK / G;
  const int g = tid / G, gl = tid % G;
  const int esize = dtype == IVF_DTYPE_U8 ? 1 : dtype == IVF_DTYPE_BF16 ? 2 : 4;
  const int per_vec = 16 / esize;                         // elements per 16 bytes
  const size_t row_bytes = (size_t)t.d_base * esize;
  const bool vec = row_bytes % 16 == 0;
  const int nvec = t.d_base / per_vec;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(t.base);
  for (int c0 = 0; c0 < nc; c0 += GROUPS * U) {
    uint64_t key[U];
    float acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * GROUPS + g;
      key[u] = c < nc ? keys[c] : KEY_NONE;
      acc[u] = 0.0f;
    }
    if (vec) {
      for (int v0 = gl; v0 < nvec; v0 += G) {
        uint4 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          x[u] = make_uint4(0, 0, 0, 0);
          if (key[u] != KEY_NONE)
            x[u] = *reinterpret_cast<const uint4*>(base + (size_t)(uint32_t)key[u] * row_bytes +
                                                   (size_t)v0 * 16);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (key[u] != KEY_NONE) acc[u] = acc[u] + vec_term(qv, x[u], v0 * per_vec, ip, dtype);
      }
    } else {
      for (int i = gl; i < t.d_base; i += G) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (key[u] == KEY_NONE) continue;
          const float x = load_base(t, (int64_t)(uint32_t)key[u], i);
          if (ip) {
            acc[u] = acc[u] + qv[i] * x;
          } else {
            const float df = qv[i] - x;
            acc[u] = acc[u] + df * df;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      for (int s = 1; s < G; s <<= 1) acc[u] = acc[u] + __shfl_xor(acc[u], s, G);
      const int c = c0 + u * GROUPS + g;
      if (gl == 0 && c < nc) {
        if (key[u] == KEY_NONE) {
          keys[c] = KEY_NONE;
        } else {
          // Ascending key = ascending L2 distance / descending inner
          // product, then ascending id (the key's low 32 bits).
          const float e = plus_zero(acc[u]);
          keys[c] = make_key(ip ? plus_zero(-e) : e, (uint32_t)key[u]);
        }
      }
    }
  }
  __syncthreads();
  // Top k: select the k smallest keys, then sort only those.
  uint32_t n = (uint32_t)nc;
  if ((uint32_t)k < n) {
    KeyUnion u{keys, n, nullptr, 0};
    const uint64_t thr = block_kth(u, (uint32_t)k, &sc);
    n = block_compact_le(keys, n, thr, &cnt);
  }
  // Ascending order of the (at most k) kept keys: by rank into the free space
  // behind them when there is room, else bitonic.
  const uint64_t* sorted = keys;
  if (n <= 512 && n + n <= pow2_ceil((uint32_t)R)) {
    __syncthreads();
    block_rank_sort(keys, n, keys + n);
    sorted = keys + n;
  } else {
    const uint32_t n2 = pow2_ceil(n);
    for (uint32_t i = n + tid; i < n2; i += blockDim.x) keys[i] = KEY_NONE;
    block_bitonic_sort(keys, n2);
  }
  for (int i = tid; i < k; i += blockDim.x) {
    const uint64_t kk = (uint32_t)i < n ? sorted[i] : KEY_NONE;  // n may be < k
    if (kk == KEY_NONE) {
      out_ids[(size_t)q * k + i] = -1;
      out_dist[(size_t)q * k + i] = ip ? -INFINITY : INFINITY;
    } else {
      const float v = ord2f((uint32_t)(kk >> 32));
      out_ids[(size_t)q * k + i] = (int64_t)(uint32_t)kk;
      out_dist[(size_t)q * k + i] = ip ? plus_zero(-v) : v;
    }
  }
}

hipError_t launch_rerank(const Tables& t, const float* Q, int32_t nq, int32_t k, int32_t rerank,
                         const uint64_t* pool, const int32_t* reorder, const Workspace& w,
                         int64_t* out_ids, float* out_dist, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  size_t lds = (size_t)pow2_ceil((uint32_t)rerank) * 8 + (size_t)t.d_base * 4;
  hipLaunchKernelGGL(rerank_kernel<4>, dim3(nq), dim3(256), lds, s, t, Q, k, rerank, w.nprobe_eff,
                     pool, reorder, out_ids, out_dist);
  return hipGetLastError();
}

// Pool of a spilled index (section 4.6.2). The scan keeps the P = R * copies
// smallest keys (ord(a) << 32 | id * copies + c); since keys order by
// (a, id) first and one point has at most `copies` of them, those hold every
// key a point needs to be among the R best distinct points. One workgroup
// per query: re-key as (id << 32 | ord(a)) and sort, so that each point's
// copies are adjacent with its best first; keep the first of every run as
// (ord(a) << 32 | id); then the R smallest of those.
__global__ void __launch_bounds__(256) dedup_kernel(const uint64_t* __restrict__ in, int32_t P,
                                                    int32_t copies, int32_t R,
                                                    uint64_t* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char dyn[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(dyn);  // [pow2(P)]
  __shared__ SelectScratch sc;
  __shared__ uint32_t cnt;
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  const uint32_t n2 = pow2_ceil((uint32_t)P);
  for (uint32_t i = tid; i < n2; i += blockDim.x) {
    const uint64_t v = i < (uint32_t)P ? in[(size_t)q * P + i] : KEY_NONE;
    keys[i] = v == KEY_NONE ? KEY_NONE
                            : ((uint64_t)((uint32_t)v / (uint32_t)copies) << 32) | (v >> 32);
  }
  block_bitonic_sort(keys, n2);
  // First key of each point's run, back in (ord << 32 | id) form; the rest
  // and the padding become KEY_NONE. All reads happen before any write.
  constexpr int PER = 8;  // n2 <= 2048 = 8 * 256
  uint64_t nv[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const uint32_t i = tid + r * blockDim.x;
    nv[r] = KEY_NONE;
    if (i < n2) {
      const uint64_t v = keys[i];
      const bool first = v != KEY_NONE && (i == 0 || (keys[i - 1] >> 32) != (v >> 32));
      if (first) nv[r] = ((v & 0xffffffffull) << 32) | (v >> 32);
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const uint32_t i = tid + r * blockDim.x;
    if (i < n2) keys[i] = nv[r];
  }
  __syncthreads();
  uint32_t n = block_compact_le(keys, n2, KEY_NONE - 1, &cnt);
  if (n > (uint32_t)R) {
    KeyUnion u{keys, n, nullptr, 0};
    const uint64_t thr = block_kth(u, (uint32_t)R, &sc);  // keys are unique now
    n = block_compact_le(keys, n, thr, &cnt);
  }
  for (int i = tid; i < R; i += blockDim.x)
    out[(size_t)q * R + i] = (uint32_t)i < n ? keys[i] : KEY_NONE;
}

hipError_t launch_dedup_pool(const Tables& t, int32_t nq, int32_t rerank, const Workspace& w,
                             hipStream_t s) {
  if (nq == 0) return hipSuccess;
  const int32_t P = rerank * t.copies;
  if (pow2_ceil((uint32_t)P) > 2048u) return hipErrorInvalidValue;
  const size_t lds = (size_t)pow2_ceil((uint32_t)P) * 8;
  hipLaunchKernelGGL(dedup_kernel, dim3(nq), dim3(256), lds, s, w.cand, P, t.copies, rerank,
                     w.cand_u);
  return hipGetLastError();
}

}  // namespace ivf
