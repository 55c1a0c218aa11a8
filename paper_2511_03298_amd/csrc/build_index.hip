// Index construction on the GPU (Alg. 1): nearest-list assignment of every
// vector (the top-1 of the coarse step, reusing its kernels) and PQ encoding
// of residuals (Quantize).
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

}  // namespace ivf
