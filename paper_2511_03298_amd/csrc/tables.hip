// Device tables of a trained index (one-time, untimed): the packed 4-bit code
// blocks the ADC scan streams (the GPU counterpart of the SIMD data blocks of
// Alg. 1, BuildBlocks) and the centroid tables used by coarse scoring.
#include "common.hpp"
#include "internal.hpp"

namespace ivf {

// One thread per 64-point slot: find the slot's list, fetch the point's m
// codes and write its words. Layout per block: word-major, 64 lanes
// contiguous, so that a wavefront reading word w of a block reads 256
// consecutive bytes.
__global__ void __launch_bounds__(256) pack_kernel(Tables t, const uint8_t* __restrict__ codes,
                                                   const int64_t* __restrict__ list_off,
                                                   const int32_t* __restrict__ list_ids,
                                                   uint32_t* __restrict__ out_codes,
                                                   int32_t* __restrict__ out_ids,
                                                   int32_t* __restrict__ flag) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= (int64_t)t.blocks * BLOCK_PTS) return;
  const int blk = (int)(slot / BLOCK_PTS);
  const int lane = (int)(slot % BLOCK_PTS);
  int lo = 0, hi = t.L;  // block_off[lo] <= blk < block_off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (t.block_off[mid] <= blk) lo = mid; else hi = mid;
  }
  const int l = lo;
  const int64_t p = (int64_t)(blk - t.block_off[l]) * BLOCK_PTS + lane;
  const bool entry = p < t.list_len[l];
  const int32_t id = entry ? list_ids[list_off[l] + p] : -1;
  // An entry naming no row of base is reported (and its codes not read).
  const bool in_range = id >= 0 && (int64_t)id < t.n;
  if (entry && !in_range) flag[0] = 1;
  const bool valid = entry && in_range;
  // Code row: the point's (one copy per point) or the list entry's (spilled).
  const int64_t row = t.copies > 1 ? list_off[l] + p : (int64_t)id;
  for (int w = 0; w < t.words; ++w) {
    uint32_t word = 0;
    if (valid) {
      for (int s = 0; s < 8; ++s) {
        int j = 8 * w + s;
        if (j < t.m) word |= (uint32_t)(codes[row * t.m + j] & 15) << (4 * s);
      }
    }
    out_codes[((size_t)blk * t.words + w) * BLOCK_PTS + lane] = word;
  }
  out_ids[slot] = id;
}

hipError_t launch_pack(const Tables& t, const uint8_t* codes, const int64_t* list_off_dev,
                       const int32_t* list_ids, int32_t* flag, hipStream_t s) {
  const int64_t slots = (int64_t)t.blocks * BLOCK_PTS;
  if (slots == 0) return hipSuccess;
  const int grid = (int)((slots + 255) / 256);
  hipLaunchKernelGGL(pack_kernel, dim3(grid), dim3(256), 0, s, t, codes, list_off_dev, list_ids,
                     const_cast<uint32_t*>(t.codes), const_cast<int32_t*>(t.slot_ids), flag);
  return hipGetLastError();
}

// Low-precision copies of the probe centroids for the MFMA coarse scores:
// squared norms, BF16 rows, FP8 rows with one scale per row; zero padded to
// [L_pad][d_pad].
__global__ void __launch_bounds__(256) aux_kernel(Tables t) {
  const int l = blockIdx.x;
  const bool live = l < t.L;
  __shared__ float red[256];
  float amax = 0.0f, nrm = 0.0f;
  for (int c = threadIdx.x; c < t.d; c += blockDim.x) {
    float v = live ? t.cp[(size_t)l * t.d + c] : 0.0f;
    amax = fmaxf(amax, fabsf(v));
    nrm += v * v;
  }
  red[threadIdx.x] = amax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const float rmax = red[0];
  __syncthreads();
  red[threadIdx.x] = nrm;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const float scale = rmax > 0.0f ? rmax / 448.0f : 1.0f;
  if (threadIdx.x == 0) {
    const_cast<float*>(t.cp_norm2)[l] = red[0];
    const_cast<float*>(t.cp_fp8_scale)[l] = scale;
  }
  for (int c = threadIdx.x; c < t.d_pad; c += blockDim.x) {
    float v = (live && c < t.d) ? t.cp[(size_t)l * t.d + c] : 0.0f;
    const_cast<float*>(t.cp_f32)[(size_t)l * t.d_pad + c] = v;
    const_cast<uint16_t*>(t.cp_bf16)[(size_t)l * t.d_pad + c] = bf16_rne(v);
    const_cast<uint8_t*>(t.cp_fp8)[(size_t)l * t.d_pad + c] = e4m3_rne(v / scale);
  }
}

hipError_t launch_aux_tables(const Tables& t, hipStream_t s) {
  hipLaunchKernelGGL(aux_kernel, dim3(t.L_pad), dim3(256), 0, s, t);
  return hipGetLastError();
}

// Spilled index (section 4.6.2): the slots of one point get distinct values
// id * copies + c, c = 0, 1, ... in slot order, so that every search key
// (ord(a) << 32 | slot value) is unique and id = value / copies. Round r
// finds, per point, the first slot not numbered yet (atomicMin into first[]),
// numbers it r and marks it with the top bit (values stay below 2^31 - 1, so
// a marked slot never reads as the -1 padding). A slot still unmarked after
// `copies` rounds belongs to a point in more lists than allowed (or is not a
// row of base): flag[0] = 1.
__global__ void copies_min_kernel(const int32_t* __restrict__ slot_ids, int64_t slots, int64_t n,
                                  int32_t* __restrict__ first) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= slots) return;
  const int32_t v = slot_ids[sl];
  if (v >= 0 && v < n) atomicMin(&first[v], (int32_t)sl);
}

__global__ void copies_mark_kernel(int32_t* __restrict__ slot_ids, int64_t slots, int64_t n,
                                   const int32_t* __restrict__ first, int32_t copies, int32_t r) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= slots) return;
  const int32_t v = slot_ids[sl];
  if (v >= 0 && v < n && first[v] == (int32_t)sl)
    slot_ids[sl] = (int32_t)(0x80000000u | (uint32_t)(v * copies + r));
}

__global__ void copies_final_kernel(int32_t* __restrict__ slot_ids, int64_t slots,
                                    int32_t* __restrict__ flag) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= slots) return;
  const int32_t v = slot_ids[sl];
  if (v == -1) return;
  if (v >= 0)
    flag[0] = 1;
  else
    slot_ids[sl] = (int32_t)((uint32_t)v & 0x7fffffffu);
}

hipError_t launch_number_copies(const Tables& t, int32_t* first, int32_t* flag, hipStream_t s) {
  const int64_t slots = (int64_t)t.blocks * BLOCK_PTS;
  hipError_t e = hipSuccess;
  if (slots == 0) return e;
  const unsigned grid = (unsigned)((slots + 255) / 256);
  int32_t* ids = const_cast<int32_t*>(t.slot_ids);
  for (int r = 0; r < t.copies; ++r) {
    e = launch_fill_u32((uint32_t*)first, 0x7fffffffu, (size_t)t.n, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(copies_min_kernel, dim3(grid), dim3(256), 0, s, ids, slots, t.n, first);
    hipLaunchKernelGGL(copies_mark_kernel, dim3(grid), dim3(256), 0, s, ids, slots, t.n, first,
                       t.copies, r);
  }
  hipLaunchKernelGGL(copies_final_kernel, dim3(grid), dim3(256), 0, s, ids, slots, flag);
  return hipGetLastError();
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace ivf
