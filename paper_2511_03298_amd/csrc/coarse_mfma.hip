// Approximate coarse scores on the matrix cores (step 1, first pass):
//   L2: s~ = |c|^2 - 2 <q, c>      IP: s~ = -<q, c>
// as a dense [nq x d] x [d x L] product with FP32 accumulation, in one of
// three operand precisions:
//   FP32  v_mfma_f32_32x32x2_f32
//   BF16  v_mfma_f32_32x32x16_bf16 (round-to-nearest-even operands)
//   FP8   v_mfma_f32_32x32x16_fp8_fp8 (OCP E4M3 operands with one scale per
//         query row and per centroid row, applied in the epilogue).
// The approximate matrix only pre-selects widen*nprobe lists per query; the
// final probe set comes from the canonical FP32 re-score (coarse.hip).
//
// Operands are row-major with the contraction dimension contiguous and
// zero-padded (queries to [nq_pad x d_pad], centroids to [L_pad x d_pad]),
// so every lane loads its MFMA fragment as one contiguous run straight from
// global memory; several fragments are in flight before their products are
// issued (d_pad is a multiple of 64). Each wave owns 2 x 2 output tiles of
// 32 x 32 (workgroup: 128 queries x 128 lists).
#include "common.hpp"
#include "internal.hpp"

namespace ivf {

typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

// Queries -> padded operand rows (zeros past nq and d), plus FP8 row scales.
__global__ void __launch_bounds__(256) query_operands_kernel(Tables t, const float* __restrict__ Q,
                                                            int32_t nq, int coarse, void* out,
                                                            float* __restrict__ scale) {
  const int q = blockIdx.x;
  const bool live = q < nq;
  __shared__ float red[256];
  float s = 1.0f;
  if (coarse == IVF_COARSE_FP8) {
    float mx = 0.0f;
    for (int c = threadIdx.x; c < t.d; c += blockDim.x)
      mx = fmaxf(mx, live ? fabsf(Q[(size_t)q * t.d + c]) : 0.0f);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
      if (threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
      __syncthreads();
    }
    s = red[0] > 0.0f ? red[0] / 448.0f : 1.0f;
    if (threadIdx.x == 0) scale[q] = s;
  }
  for (int c = threadIdx.x; c < t.d_pad; c += blockDim.x) {
    const float v = (live && c < t.d) ? Q[(size_t)q * t.d + c] : 0.0f;
    const size_t o = (size_t)q * t.d_pad + c;
    if (coarse == IVF_COARSE_F32) reinterpret_cast<float*>(out)[o] = v;
    else if (coarse == IVF_COARSE_BF16) reinterpret_cast<uint16_t*>(out)[o] = bf16_rne(v);
    else reinterpret_cast<uint8_t*>(out)[o] = e4m3_rne(v / s);
  }
}

template <int COARSE>
__global__ void __launch_bounds__(256) coarse_mfma_kernel(Tables t, const void* __restrict__ Aop,
                                                         const float* __restrict__ qscale,
                                                         int32_t nq, float* __restrict__ S) {
  // Wave tile: 64 queries x 64 lists as 2 x 2 MFMA tiles of 32 x 32, so every
  // loaded fragment feeds two products; the workgroup's 4 waves cover 128 x
  // 128. Operand rows are padded to multiples of 64, so a wave is either
  // wholly inside them or has nothing to do.
  const int wave = threadIdx.x / IVF_WAVE, lane = threadIdx.x % IVF_WAVE;
  const int q0 = blockIdx.y * 128 + (wave / 2) * 64;
  const int l0 = blockIdx.x * 128 + (wave % 2) * 64;
  const int nq_pad = (nq + 63) / 64 * 64;
  if (q0 >= nq_pad || l0 >= t.L_pad) return;  // per wave; no barriers in this kernel
  const int r = lane % 32, half = lane / 32;
  const size_t dp = (size_t)t.d_pad;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
  if constexpr (COARSE == IVF_COARSE_F32) {
    const float* a0 = reinterpret_cast<const float*>(Aop) + (size_t)(q0 + r) * dp + half;
    const float* b0 = t.cp_f32 + (size_t)(l0 + r) * dp + half;
    const float* a1 = a0 + 32 * dp;
    const float* b1 = b0 + 32 * dp;
    for (int k0 = 0; k0 < t.d_pad; k0 += 8) {
      float av[2][4], bv[2][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[0][u] = a0[k0 + 2 * u];
        av[1][u] = a1[k0 + 2 * u];
        bv[0][u] = b0[k0 + 2 * u];
        bv[1][u] = b1[k0 + 2 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][u], bv[j][u], acc[i][j], 0, 0, 0);
    }
  } else if constexpr (COARSE == IVF_COARSE_BF16) {
    const uint16_t* a0 = reinterpret_cast<const uint16_t*>(Aop) + (size_t)(q0 + r) * dp + half * 8;
    const uint16_t* b0 = t.cp_bf16 + (size_t)(l0 + r) * dp + half * 8;
    const uint16_t* a1 = a0 + 32 * dp;
    const uint16_t* b1 = b0 + 32 * dp;
    for (int k0 = 0; k0 < t.d_pad; k0 += 32) {
      bf16x8 av[2][2], bv[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        av[0][u] = *reinterpret_cast<const bf16x8*>(a0 + k0 + 16 * u);
        av[1][u] = *reinterpret_cast<const bf16x8*>(a1 + k0 + 16 * u);
        bv[0][u] = *reinterpret_cast<const bf16x8*>(b0 + k0 + 16 * u);
        bv[1][u] = *reinterpret_cast<const bf16x8*>(b1 + k0 + 16 * u);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i][u], bv[j][u], acc[i][j], 0, 0, 0);
    }
  } else {
    const uint8_t* a0 = reinterpret_cast<const uint8_t*>(Aop) + (size_t)(q0 + r) * dp + half * 8;
    const uint8_t* b0 = t.cp_fp8 + (size_t)(l0 + r) * dp + half * 8;
    const uint8_t* a1 = a0 + 32 * dp;
    const uint8_t* b1 = b0 + 32 * dp;
    for (int k0 = 0; k0 < t.d_pad; k0 += 32) {
      long av[2][2], bv[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        av[0][u] = *reinterpret_cast<const long*>(a0 + k0 + 16 * u);
        av[1][u] = *reinterpret_cast<const long*>(a1 + k0 + 16 * u);
        bv[0][u] = *reinterpret_cast<const long*>(b0 + k0 + 16 * u);
        bv[1][u] = *reinterpret_cast<const long*>(b1 + k0 + 16 * u);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(av[i][u], bv[j][u], acc[i][j], 0, 0, 0);
    }
  }
  // Tile (i, j): lane holds D[8*(e/4) + 4*half + e%4][r] for e = 0..15, rows
  // are queries q0 + 32 i + ..., the column is list l0 + 32 j + r.
  const bool ip = t.metric == IVF_METRIC_IP;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int l = l0 + 32 * j + r;
    if (l >= t.L) continue;
    const float cn = t.cp_norm2[l];
    const float cs = COARSE == IVF_COARSE_FP8 ? t.cp_fp8_scale[l] : 1.0f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int q = q0 + 32 * i + 8 * (e / 4) + 4 * half + (e % 4);
        if (q >= nq) continue;
        float dot = acc[i][j][e];
        if (COARSE == IVF_COARSE_FP8) dot = dot * (qscale[q] * cs);
        S[(size_t)q * t.L + l] = ip ? -dot : cn - 2.0f * dot;
      }
    }
  }
}

hipError_t launch_coarse_mfma(const Tables& t, const float* Q, int32_t nq, int coarse,
                              const Workspace& w, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  const int nq_pad = (nq + 63) / 64 * 64;
  hipLaunchKernelGGL(query_operands_kernel, dim3(nq_pad), dim3(256), 0, s, t, Q, nq, coarse,
                     (void*)w.q_lowp, w.q_scale);
  dim3 grid((t.L_pad + 127) / 128, (nq_pad + 127) / 128);
  switch (coarse) {
    case IVF_COARSE_F32:
      hipLaunchKernelGGL(coarse_mfma_kernel<IVF_COARSE_F32>, grid, dim3(256), 0, s, t,
                         (const void*)w.q_lowp, w.q_scale, nq, w.scores);
      break;
    case IVF_COARSE_BF16:
      hipLaunchKernelGGL(coarse_mfma_kernel<IVF_COARSE_BF16>, grid, dim3(256), 0, s, t,
                         (const void*)w.q_lowp, w.q_scale, nq, w.scores);
      break;
    case IVF_COARSE_FP8:
      hipLaunchKernelGGL(coarse_mfma_kernel<IVF_COARSE_FP8>, grid, dim3(256), 0, s, t,
                         (const void*)w.q_lowp, w.q_scale, nq, w.scores);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ivf
