// Step 5 of the search (Alg. 2, final step): exact distances between the
// query and its candidate rows, FP32 accumulation (BF16 rows are widened
// exactly), and the top k by (distance, id): ascending squared L2, or
// descending inner product.
#include "common.hpp"
#include "internal.hpp"

namespace ivf {

__device__ __forceinline__ float load_base(const Tables& t, int64_t row, int c) {
  if (t.base_dtype == IVF_DTYPE_BF16) {
    const uint16_t* b = reinterpret_cast<const uint16_t*>(t.base);
    return __uint_as_float((uint32_t)b[row * t.d + c] << 16);
  }
  return reinterpret_cast<const float*>(t.base)[row * t.d + c];
}

// One workgroup per query. Candidates are spread over groups of G lanes
// (G = 64, 32 or 16 depending on d); each lane sums a strided slice of the
// row and the group reduces with a butterfly in a fixed order.
template <int G>
__global__ void __launch_bounds__(256) rerank_kernel(Tables t, const float* __restrict__ Q,
                                                     int32_t k, int32_t R,
                                                     const int32_t* __restrict__ nprobe_eff,
                                                     const uint64_t* __restrict__ cand,
                                                     int64_t* __restrict__ out_ids,
                                                     float* __restrict__ out_dist) {
  extern __shared__ __align__(16) unsigned char dyn[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(dyn);                   // [pow2(R)]
  float* qv = reinterpret_cast<float*>(keys + pow2_ceil((uint32_t)R));  // [d]
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  const bool ip = t.metric == IVF_METRIC_IP;
  if (nprobe_eff[q] < 0) {  // invalid request row
    for (int i = tid; i < k; i += blockDim.x) {
      out_ids[(size_t)q * k + i] = -1;
      out_dist[(size_t)q * k + i] = __uint_as_float(0x7fc00000u);
    }
    return;
  }
  for (int i = tid; i < t.d; i += blockDim.x) qv[i] = Q[(size_t)q * t.d + i];
  __syncthreads();
  constexpr int GROUPS = IVF_BLOCK / G;
  constexpr int U = 4;  // candidates in flight per lane group
  const int g = tid / G, gl = tid % G;
  for (int c0 = 0; c0 < R; c0 += GROUPS * U) {
    uint64_t key[U];
    float acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * GROUPS + g;
      key[u] = c < R ? cand[(size_t)q * R + c] : KEY_NONE;
      acc[u] = 0.0f;
    }
    for (int i = gl; i < t.d; i += G) {
      float x[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        x[u] = key[u] != KEY_NONE ? load_base(t, (int64_t)(uint32_t)key[u], i) : 0.0f;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (ip) {
          acc[u] = acc[u] + qv[i] * x[u];
        } else {
          const float df = qv[i] - x[u];
          acc[u] = acc[u] + df * df;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      for (int s = 1; s < G; s <<= 1) acc[u] = acc[u] + __shfl_xor(acc[u], s, G);
      const int c = c0 + u * GROUPS + g;
      if (gl == 0 && c < R) {
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
  __shared__ SelectScratch sc;
  __shared__ uint32_t cnt;
  uint32_t n = (uint32_t)R;
  if ((uint32_t)k < n) {
    KeyUnion u{keys, n, nullptr, 0};
    const uint64_t thr = block_kth(u, (uint32_t)k, &sc);
    n = block_compact_le(keys, n, thr, &cnt);
  }
  const uint32_t n2 = pow2_ceil(n);
  for (uint32_t i = n + tid; i < n2; i += blockDim.x) keys[i] = KEY_NONE;
  block_bitonic_sort(keys, n2);
  for (int i = tid; i < k; i += blockDim.x) {
    const uint64_t kk = i < R ? keys[i] : KEY_NONE;
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
                         const Workspace& w, int64_t* out_ids, float* out_dist, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  size_t lds = (size_t)pow2_ceil((uint32_t)rerank) * 8 + (size_t)t.d * 4;
  if (t.d >= 256) {
    hipLaunchKernelGGL(rerank_kernel<64>, dim3(nq), dim3(256), lds, s, t, Q, k, rerank,
                       w.nprobe_eff, w.cand, out_ids, out_dist);
  } else if (t.d >= 64) {
    hipLaunchKernelGGL(rerank_kernel<32>, dim3(nq), dim3(256), lds, s, t, Q, k, rerank,
                       w.nprobe_eff, w.cand, out_ids, out_dist);
  } else {
    hipLaunchKernelGGL(rerank_kernel<16>, dim3(nq), dim3(256), lds, s, t, Q, k, rerank,
                       w.nprobe_eff, w.cand, out_ids, out_dist);
  }
  return hipGetLastError();
}

}  // namespace ivf
