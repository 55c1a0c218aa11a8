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

// BF16 form with operands staged through LDS by direct global-to-LDS loads
// (global_load_lds_dwordx4 writes lane i's 16 bytes at the wave's LDS base
// + 16 i, with no register staging). Workgroup tile: 256 queries x 256
// lists, eight waves of 64 x 128 each (2 x 4 MFMA tiles of 32 x 32), so a
// fragment read from LDS feeds four (query) or two (list) products, and
// each operand row is loaded by L / 256 (queries) or nq / 256 (lists)
// workgroups. K advances 32 at a time through four LDS stages of 32 KB:
// the loads of step ks + 3 are issued while step ks is multiplied.
// Stage layout: rows of 32 BF16 (4 chunks of 16 bytes), queries 0..255 then
// lists 0..255 (rows 256..511).
constexpr int CB_TQ = 256, CB_TL = 256, CB_TK = 32;
constexpr int CB_WAVES = 8;
constexpr int CB_ROWS = CB_TQ + CB_TL;
constexpr int CB_CPR = CB_TK / 8;                       // 16-byte chunks per row
constexpr int CB_STAGE = CB_ROWS * CB_CPR;              // chunks per stage
constexpr int CB_STAGES = 4;
constexpr int CB_DMA = CB_STAGE / (CB_WAVES * IVF_WAVE);  // loads per wave and step

// Chunk position of chunk c of row R: rows of 64 bytes, so rows R and R + 4
// share banks; the chunk index is rotated by (R >> 2) & 3, which spreads any
// 16 consecutive rows' chunk c over 16 distinct 4-bank groups.
__device__ __forceinline__ int cb_pos(int R, int c) { return R * CB_CPR + (c ^ ((R >> 2) & 3)); }

// Workgroup barrier for LDS only: the compiler's __syncthreads() also waits
// for every outstanding global access (including the loads of later steps
// in flight); this one waits for this wave's LDS accesses, and the memory
// clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__global__ void __launch_bounds__(512) coarse_bf16_lds_kernel(Tables t,
                                                             const uint16_t* __restrict__ Aop,
                                                             int32_t nq, float* __restrict__ S) {
  extern __shared__ __align__(16) unsigned char dyn[];
  uint4* lds = reinterpret_cast<uint4*>(dyn);
  const int tid = threadIdx.x, wave = tid / IVF_WAVE, lane = tid % IVF_WAVE;
  const int q0 = blockIdx.y * CB_TQ, l0 = blockIdx.x * CB_TL;
  const int nq_pad = (nq + 63) / 64 * 64;
  const size_t dp = (size_t)t.d_pad;
  // Source of this lane's chunk for its j-th load of a step: LDS position
  // p = (wave * CB_DMA + j) * 64 + lane. Rows past the padded operands read
  // the last padded row instead; they only feed outputs that are not written.
  const uint16_t* src[CB_DMA];
#pragma unroll
  for (int j = 0; j < CB_DMA; ++j) {
    const int p = (wave * CB_DMA + j) * IVF_WAVE + lane;
    const int R = p / CB_CPR, c = (p % CB_CPR) ^ ((R >> 2) & 3);
    if (R < CB_TQ)
      src[j] = Aop + (size_t)min(q0 + R, nq_pad - 1) * dp + 8 * c;
    else
      src[j] = t.cp_bf16 + (size_t)min(l0 + R - CB_TQ, t.L_pad - 1) * dp + 8 * c;
  }
  auto issue = [&](int ks) {
    uint4* dst = lds + (ks % CB_STAGES) * CB_STAGE + wave * CB_DMA * IVF_WAVE;
#pragma unroll
    for (int j = 0; j < CB_DMA; ++j)
      __builtin_amdgcn_global_load_lds(src[j] + ks * CB_TK, dst + j * IVF_WAVE, 16, 0, 0);
  };
  const int wq = wave >> 1, wl = wave & 1;
  const int r = lane & 31, half = lane >> 5;
  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
  const bool ip = t.metric == IVF_METRIC_IP;
  float cn[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int l = l0 + wl * 128 + 32 * j + r;
    cn[j] = (!ip && l < t.L) ? t.cp_norm2[l] : 0.0f;
  }
  const int nk = t.d_pad / CB_TK;
  for (int s0 = 0; s0 < CB_STAGES - 1 && s0 < nk; ++s0) issue(s0);
  for (int ks = 0; ks < nk; ++ks) {
    // This wave's loads of step ks are done once at most the loads of the
    // later steps already issued (CB_DMA each, issued after) are in flight;
    // the barrier then makes every wave's part of the tile visible and frees
    // stage (ks + 3) % 4, which the previous step read.
    const int ahead = min(CB_STAGES - 2, nk - 1 - ks);  // later steps in flight
    if (ahead >= 2)
      __builtin_amdgcn_s_waitcnt(0x0f70 | (2 * CB_DMA));
    else if (ahead == 1)
      __builtin_amdgcn_s_waitcnt(0x0f70 | CB_DMA);
    else
      __builtin_amdgcn_s_waitcnt(0x0f70);
    lds_barrier();
    if (ks + CB_STAGES - 1 < nk) issue(ks + CB_STAGES - 1);
    const uint4* st = lds + (ks % CB_STAGES) * CB_STAGE;
    // Fragments in two register sets: those of substep u + 1 are requested
    // between the products of substep u, so LDS latency overlaps the MFMAs.
    bf16x8 a[2][2], b[2][4];
    auto frags = [&](int u, int set) {
      const int c = 2 * u + half;  // lane's 8 values: k = 16u + 8 half .. + 7
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[set][i] = *reinterpret_cast<const bf16x8*>(&st[cb_pos(wq * 64 + 32 * i + r, c)]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[set][j] =
            *reinterpret_cast<const bf16x8*>(&st[cb_pos(CB_TQ + wl * 128 + 32 * j + r, c)]);
    };
    frags(0, 0);
#pragma unroll
    for (int u = 0; u < CB_TK / 16; ++u) {
      if (u + 1 < CB_TK / 16) frags(u + 1, (u + 1) & 1);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[u & 1][i], b[u & 1][j],
                                                              acc[i][j], 0, 0, 0);
    }
    // Schedule: the first substep's 6 fragment reads, then one read of the
    // next substep after each of the first 6 products of a substep.
    __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);  // DS read
#pragma unroll
    for (int u = 0; u + 1 < CB_TK / 16; ++u) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
  }
  // Tile (i, j): lane holds D[8*(e/4) + 4*half + e%4][r], rows are queries
  // q0 + 64 wq + 32 i + ..., the column is list l0 + 128 wl + 32 j + r.
  // Every load (the squared norms included) is complete here; waiting
  // explicitly tells the compiler so, and no store then waits on a load.
  __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e)
        acc[i][j][e] = ip ? -acc[i][j][e] : cn[j] - 2.0f * acc[i][j][e];
  const bool full = q0 + CB_TQ <= nq && l0 + CB_TL <= t.L;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int l = l0 + wl * 128 + 32 * j + r;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int q = q0 + wq * 64 + 32 * i + 8 * (e / 4) + 4 * half + (e % 4);
        if (full || (q < nq && l < t.L)) S[(size_t)q * t.L + l] = acc[i][j][e];
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
    case IVF_COARSE_BF16: {
      const dim3 g2((t.L_pad + CB_TL - 1) / CB_TL, (nq_pad + CB_TQ - 1) / CB_TQ);
      hipLaunchKernelGGL(coarse_bf16_lds_kernel, g2, dim3(CB_WAVES * IVF_WAVE), (size_t)CB_STAGES * CB_STAGE * 16, s, t,
                         (const uint16_t*)w.q_lowp, nq, w.scores);
      break;
    }
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
