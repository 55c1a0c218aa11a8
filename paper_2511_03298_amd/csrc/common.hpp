// Shared device helpers for the gfx950 IVF-PQ kernels: order-preserving key
// encoding, wave (64-lane) primitives, and workgroup-wide selection / sort
// over 64-bit keys held in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define IVF_WAVE 64
#define IVF_BLOCK 256
#define IVF_NWAVES (IVF_BLOCK / IVF_WAVE)

namespace ivf {

constexpr uint64_t KEY_NONE = ~0ull;

// Map a float onto uint32 so that unsigned order equals float order
// (-0 < +0; callers normalise -0 to +0 first where the two must compare equal).
__device__ __forceinline__ uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  return __uint_as_float(u);
}
__device__ __forceinline__ float plus_zero(float x) {
  // -0.0 -> +0.0, every other value unchanged.
  return x == 0.0f ? 0.0f : x;
}

// Inner-product list constant b = -<q, c> over d components: sequential in
// the component index, FP32, every product and sum rounded on its own
// (16-byte loads of the row when d is a multiple of 4, in the same order).
// qv may live in LDS.
__device__ __forceinline__ float ip_list_bias(const float* __restrict__ c, const float* qv, int d) {
  float acc = 0.0f;
  if ((d & 3) == 0) {
    const float4* c4 = reinterpret_cast<const float4*>(c);
    for (int k4 = 0; k4 < d / 4; ++k4) {
      const float4 v = c4[k4];
      acc = acc + qv[4 * k4 + 0] * v.x;
      acc = acc + qv[4 * k4 + 1] * v.y;
      acc = acc + qv[4 * k4 + 2] * v.z;
      acc = acc + qv[4 * k4 + 3] * v.w;
    }
  } else {
    for (int k = 0; k < d; ++k) acc = acc + qv[k] * c[k];
  }
  return plus_zero(-acc);
}
__device__ __forceinline__ uint64_t make_key(float v, uint32_t idx) {
  return ((uint64_t)f2ord(v) << 32) | (uint64_t)idx;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ int wave_index() { return threadIdx.x / IVF_WAVE; }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Append the keys of the lanes with `pred` set to buf[*count ...]; one LDS
// atomic per wave. Returns nothing; order inside the buffer is arbitrary.
__device__ __forceinline__ void wave_append(bool pred, uint64_t key, uint64_t* buf,
                                            uint32_t* count) {
  uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  uint32_t base = 0;
  if (lane_id() == 0) base = atomicAdd(count, (uint32_t)__popcll(mask));
  base = __shfl(base, 0);
  if (pred) buf[base + lanes_below(mask)] = key;
}

// Scratch a workgroup needs for block_kth.
struct alignas(8) SelectScratch {
  uint32_t hist[256];
  uint32_t bin, below, cnt, pad;
};

// Accessor over a key set that is the union of two LDS ranges:
// a[0..na) followed by b[0..nb).
struct KeyUnion {
  const uint64_t* a;
  uint32_t na;
  const uint64_t* b;
  uint32_t nb;
  __device__ __forceinline__ uint32_t size() const { return na + nb; }
  __device__ __forceinline__ uint64_t operator[](uint32_t i) const {
    return i < na ? a[i] : b[i - na];
  }
};

// Returns the smallest threshold t such that exactly K keys of `keys` are
// <= t, by MSB-first radix selection in 8-bit digits. Keys must be unique,
// 1 <= K <= keys.size(). Must be called by all threads of the workgroup.
// Digits above the highest byte in which the smallest and largest key differ
// are common to every key, so selection starts at that byte.
template <class Keys>
__device__ uint64_t block_kth(const Keys& keys, uint32_t K, SelectScratch* sc) {
  const int tid = threadIdx.x;
  const uint32_t n = keys.size();
  uint64_t lo = ~0ull, hi = 0;
  for (uint32_t i = tid; i < n; i += blockDim.x) {
    const uint64_t k = keys[i];
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
  }
  for (int off = 1; off < IVF_WAVE; off <<= 1) {
    const uint64_t a = __shfl_xor(lo, off), c = __shfl_xor(hi, off);
    lo = a < lo ? a : lo;
    hi = c > hi ? c : hi;
  }
  uint64_t* mm = reinterpret_cast<uint64_t*>(sc->hist);  // [waves][2], before the histograms
  const int nw = (int)(blockDim.x / IVF_WAVE);
  if (lane_id() == 0) {
    mm[2 * wave_index()] = lo;
    mm[2 * wave_index() + 1] = hi;
  }
  __syncthreads();
  lo = mm[0];
  hi = mm[1];
  for (int w = 1; w < nw; ++w) {
    lo = mm[2 * w] < lo ? mm[2 * w] : lo;
    hi = mm[2 * w + 1] > hi ? mm[2 * w + 1] : hi;
  }
  __syncthreads();
  const uint64_t diff = lo ^ hi;
  if (diff == 0) return lo;  // a single distinct key (K == 1)
  const int top = (63 - __builtin_clzll(diff)) & ~7;  // lowest bit of the first differing byte
  uint64_t mask = top == 56 ? 0ull : ~0ull << (top + 8);
  uint64_t prefix = lo & mask;
  uint32_t need = K;
  for (int shift = top; shift >= 0; shift -= 8) {
    for (int i = tid; i < 256; i += blockDim.x) sc->hist[i] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += blockDim.x) {
      uint64_t k = keys[i];
      if ((k & mask) == prefix) atomicAdd(&sc->hist[(k >> shift) & 255], 1u);
    }
    __syncthreads();
    if (tid < IVF_WAVE) {
      // Each lane owns 4 consecutive bins; inclusive scan across lanes.
      uint32_t h0 = sc->hist[tid * 4 + 0], h1 = sc->hist[tid * 4 + 1];
      uint32_t h2 = sc->hist[tid * 4 + 2], h3 = sc->hist[tid * 4 + 3];
      uint32_t local = h0 + h1 + h2 + h3;
      uint32_t incl = local;
      for (int off = 1; off < IVF_WAVE; off <<= 1) {
        uint32_t v = __shfl_up(incl, off);
        if (tid >= off) incl += v;
      }
      uint32_t excl = incl - local;
      bool hit = excl < need && incl >= need;
      if (hit) {
        uint32_t c = excl;
        int b = tid * 4;
        uint32_t hs[4] = {h0, h1, h2, h3};
        for (int j = 0; j < 4; ++j) {
          if (c + hs[j] >= need) { b = tid * 4 + j; break; }
          c += hs[j];
        }
        sc->bin = (uint32_t)b;
        sc->below = c;
        sc->cnt = sc->hist[b];
      }
    }
    __syncthreads();
    uint32_t b = sc->bin, below = sc->below, cnt = sc->cnt;
    need -= below;
    prefix |= (uint64_t)b << shift;
    mask |= 0xffull << shift;
    __syncthreads();
    if (cnt == need) break;
  }
  return prefix | ~mask;
}

// In-place ascending bitonic sort of keys[0..n), n a power of two.
__device__ inline void block_bitonic_sort(uint64_t* keys, uint32_t n) {
  for (uint32_t size = 2; size <= n; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < n / 2; i += blockDim.x) {
        uint32_t lo = 2 * i - (i & (stride - 1));
        uint32_t hi = lo + stride;
        bool up = ((lo & size) == 0);
        uint64_t a = keys[lo], b = keys[hi];
        if ((a > b) == up) {
          keys[lo] = b;
          keys[hi] = a;
        }
      }
    }
  }
  __syncthreads();
}

// Moves the keys <= thr among keys[0..n) to the front of the array (in
// arbitrary order) and returns how many there are. Works in place: each
// segment of blockDim*8 keys is read into registers before any thread
// writes, and write positions never pass the end of the segment being read.
__device__ inline uint32_t block_compact_le(uint64_t* keys, uint32_t n, uint64_t thr,
                                            uint32_t* counter) {
  constexpr int PER = 8;
  if (threadIdx.x == 0) *counter = 0;
  __syncthreads();
  const uint32_t seg = blockDim.x * PER;
  for (uint32_t s0 = 0; s0 < n; s0 += seg) {
    uint64_t v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      uint32_t idx = s0 + i * blockDim.x + threadIdx.x;
      v[i] = idx < n ? keys[idx] : KEY_NONE;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      uint32_t idx = s0 + i * blockDim.x + threadIdx.x;
      wave_append(idx < n && v[i] <= thr, v[i], keys, counter);
    }
    __syncthreads();
  }
  const uint32_t c = *counter;
  __syncthreads();
  return c;
}

// Round a float to bfloat16, nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Encode a float as OCP FP8 E4M3 (3 mantissa bits, exponent bias 7, largest
// finite 448, subnormal spacing 2^-9), round to nearest even, saturating;
// values that round to zero encode as +0 (0x00), never as 0x80.
__device__ __forceinline__ uint8_t e4m3_rne(float x) {
  const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fminf(fabsf(x), 448.0f);
  if (!(a > 0.0f)) return 0;
  int e = 0;
  frexpf(a, &e);  // a = f * 2^e, f in [0.5, 1)
  int eu = e - 1;
  if (eu < -6) eu = -6;
  const float quantum = ldexpf(1.0f, eu - 3);
  const float qv = fminf(rintf(a / quantum) * quantum, 448.0f);
  if (qv == 0.0f) return 0;
  int e2 = 0;
  const float f2 = frexpf(qv, &e2);
  const int eu2 = e2 - 1;
  const uint32_t bits =
      eu2 < -6 ? (uint32_t)rintf(qv * 512.0f)
               : (((uint32_t)(eu2 + 7) << 3) | (uint32_t)rintf((f2 * 2.0f - 1.0f) * 8.0f));
  return (uint8_t)(sign | bits);
}

__host__ __device__ inline uint32_t pow2_ceil(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Pairwise sum of v[0..m) padded with zeros to a power of two, by one wavefront
// (adjacent pairs first, then pairs of pairs, ...).
__device__ __forceinline__ float wave_pairwise_sum(const float* v, int m) {
  const int lane = lane_id();
  const int p2 = (int)pow2_ceil((uint32_t)m);
  float x;
  int width;
  if (p2 <= IVF_WAVE) {
    x = lane < m ? v[lane] : 0.0f;
    width = p2;
  } else {
    const int per = p2 / IVF_WAVE;  // 2 or 4 consecutive elements per lane
    float e[4];
    for (int i = 0; i < 4; ++i) {
      int idx = lane * per + i;
      e[i] = (i < per && idx < m) ? v[idx] : 0.0f;
    }
    x = per == 2 ? e[0] + e[1] : (e[0] + e[1]) + (e[2] + e[3]);
    width = IVF_WAVE;
  }
  for (int s = 1; s < width; s <<= 1) x = x + __shfl_xor(x, s);
  return __shfl(x, 0);
}

}  // namespace ivf
