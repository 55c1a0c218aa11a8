// Index construction on the GPU (Alg. 1): nearest-list assignment of every
// vector (the top-1 of the coarse step, reusing its kernels), PQ encoding
// of residuals (Quantize), and the SOAR spill loss of a spilled index.
//
// Encoding, canonical FP32 like the search path:
//   r_u = x_u - c_{list(x),u} (rounded once)
//   code_j(x) = argmin_i sum_u (r_{j d'+u} - B[j,i,u])^2, sequential in u,
//   ties to the smallest i.
#include "common.hpp"
#include "internal.hpp"

namespace ivf {

__global__ void __launch_bounds__(256) encode_kernel(const float* __restrict__ X, int64_t n,
                                                     int32_t d, int32_t m,
                                                     const float* __restrict__ cm,
                                                     const int32_t* __restrict__ lists,
                                                     const float* __restrict__ codebooks,
                                                     uint8_t* __restrict__ codes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * m) return;
  const int64_t row = i / m;
  const int j = (int)(i % m);
  const int ds = d / m;
  const float* x = X + row * d + j * ds;
  const float* c = cm + (int64_t)lists[row] * d + j * ds;
  float best = 0.0f;
  int besti = 0;
  for (int k = 0; k < KSUB; ++k) {
    const float* b = codebooks + ((int64_t)j * KSUB + k) * ds;
    float acc = 0.0f;
    for (int u = 0; u < ds; ++u) {
      const float ru = x[u] - c[u];  // the same rounded residual every time
      const float df = ru - b[u];
      acc = acc + df * df;
    }
    if (k == 0 || acc < best) {
      best = acc;
      besti = k;
    }
  }
  codes[i] = (uint8_t)besti;
}

hipError_t launch_encode(const float* X, int64_t n, int32_t d, int32_t m, const float* cm,
                         const int32_t* lists, const float* codebooks, uint8_t* codes,
                         hipStream_t s) {
  const int64_t total = n * m;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(encode_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, X, n,
                     d, m, cm, lists, codebooks, codes);
  return hipGetLastError();
}

// SOAR spill loss (section 4.6.2 integrates SOAR): for row x with primary
// list p and r = x - c_p, loss(l) = dist + lam * (proj * proj / rr) with
//   dist = sum_t (x_t - c_lt)^2, proj = sum_t r_t (x_t - c_lt), rr = sum_t r_t^2,
// every difference rounded once and each sum sequential in t; loss(p) = +inf
// and, for rr = 0, loss = dist. Tiles of 32 rows x 64 lists as in the exact
// coarse kernel; each thread owns 2 rows x 4 lists and walks t in order.
constexpr int SQ = 32, SL = 64, SD = 32;

__global__ void __launch_bounds__(256) spill_loss_kernel(const float* __restrict__ X, int32_t rows,
                                                         int32_t d, const float* __restrict__ C,
                                                         int32_t L,
                                                         const int32_t* __restrict__ primary,
                                                         float lam, float* __restrict__ loss) {
  __shared__ float xs[SQ][SD + 1];
  __shared__ float rs[SQ][SD + 1];
  __shared__ float cs[SL][SD + 1];
  const int tid = threadIdx.x;
  const int l0 = blockIdx.x * SL, q0 = blockIdx.y * SQ;
  const int tq = (tid / 16) * 2;
  const int tl = tid % 16;
  float dist[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  float proj[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  float rr[2] = {0.f, 0.f};
  for (int d0 = 0; d0 < d; d0 += SD) {
    const int dn = min(SD, d - d0);
    __syncthreads();
    for (int e = tid; e < SQ * SD; e += 256) {
      const int r = e / SD, c = e % SD;
      const int q = q0 + r;
      float xv = 0.0f, rv = 0.0f;
      if (q < rows && c < dn) {
        xv = X[(size_t)q * d + d0 + c];
        const int p = primary[q];
        rv = (p >= 0 && p < L) ? xv - C[(size_t)p * d + d0 + c] : 0.0f;
      }
      xs[r][c] = xv;
      rs[r][c] = rv;
    }
    for (int e = tid; e < SL * SD; e += 256) {
      const int r = e / SD, c = e % SD;
      const int l = l0 + r;
      cs[r][c] = (l < L && c < dn) ? C[(size_t)l * d + d0 + c] : 0.0f;
    }
    __syncthreads();
    for (int c = 0; c < dn; ++c) {
      const float x0 = xs[tq][c], x1 = xs[tq + 1][c];
      const float r0 = rs[tq][c], r1 = rs[tq + 1][c];
      rr[0] = rr[0] + r0 * r0;
      rr[1] = rr[1] + r1 * r1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float cv = cs[tl + 16 * j][c];
        const float e0 = x0 - cv, e1 = x1 - cv;
        dist[0][j] = dist[0][j] + e0 * e0;
        dist[1][j] = dist[1][j] + e1 * e1;
        proj[0][j] = proj[0][j] + r0 * e0;
        proj[1][j] = proj[1][j] + r1 * e1;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int q = q0 + tq + i;
    if (q >= rows) continue;
    const int p = primary[q];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int l = l0 + tl + 16 * j;
      if (l >= L) continue;
      float v = dist[i][j];
      if (rr[i] > 0.0f) {
        const float pp = proj[i][j] * proj[i][j];
        v = v + lam * (pp / rr[i]);
      }
      loss[(size_t)q * L + l] = l == p ? INFINITY : v;
    }
  }
}

hipError_t launch_spill_loss(const float* X, int32_t rows, int32_t d, const float* C, int32_t L,
                             const int32_t* primary, float lam, float* loss, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  dim3 grid((L + SL - 1) / SL, (rows + SQ - 1) / SQ);
  hipLaunchKernelGGL(spill_loss_kernel, grid, dim3(256), 0, s, X, rows, d, C, L, primary, lam,
                     loss);
  return hipGetLastError();
}

// Rows whose primary list is out of range get no spill list (-1).
__global__ void spill_fix_kernel(const int32_t* __restrict__ primary, int32_t rows, int32_t L,
                                 int32_t* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rows) return;
  const int p = primary[q];
  if (p < 0 || p >= L) out[q] = -1;
}

hipError_t launch_spill_fix(const int32_t* primary, int32_t rows, int32_t L, int32_t* out,
                            hipStream_t s) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(spill_fix_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, primary, rows,
                     L, out);
  return hipGetLastError();
}

}  // namespace ivf
