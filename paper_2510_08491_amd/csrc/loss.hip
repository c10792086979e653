// L1 image loss and its gradient; float64 accumulation in a fixed order
// (per-block partial sums, then one block sums the partials), so the loss is
// deterministic for a given launch shape.
#include "snp_internal.h"

namespace snp {

constexpr int kLossBlocks = 1024;
constexpr int kLossThreads = 256;

__global__ void __launch_bounds__(kLossThreads) l1_partial_kernel(const float* __restrict__ img,
                                                                  const float* __restrict__ tgt, int64_t n,
                                                                  double inv_norm, float* __restrict__ grad,
                                                                  double* __restrict__ partials) {
  __shared__ double s[kLossThreads];
  double acc = 0.0;
  const float ginv = (float)inv_norm;
  for (int64_t i = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLossThreads) {
    const float d = img[i] - tgt[i];
    acc += fabs((double)d);
    grad[i] = d > 0.f ? ginv : (d < 0.f ? -ginv : 0.f);
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kLossThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(kLossThreads) l1_final_kernel(const double* __restrict__ partials, int nparts,
                                                                double inv_norm, double* out) {
  __shared__ double s[kLossThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kLossThreads) acc += partials[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kLossThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0] * inv_norm;
}

size_t loss_scratch_bytes() { return kLossBlocks * sizeof(double); }

hipError_t launch_l1(const float* img, const float* tgt, int64_t n, double n_norm, float* grad, double* partials,
                     double* out, hipStream_t st) {
  const double inv = 1.0 / n_norm;
  hipLaunchKernelGGL(l1_partial_kernel, dim3(kLossBlocks), dim3(kLossThreads), 0, st, img, tgt, n, inv, grad, partials);
  hipLaunchKernelGGL(l1_final_kernel, dim3(1), dim3(kLossThreads), 0, st, partials, kLossBlocks, inv, out);
  return hipGetLastError();
}

// zero a float buffer (a kernel rather than a memset, so it can sit in a graph)
__global__ void zero_f32_kernel(float* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.f;
}

hipError_t zero_f32(float* p, int64_t n, hipStream_t st) {
  if (!p || n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

hipError_t zero_counters(unsigned long long* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

__global__ void zero_one_u64_kernel(unsigned long long* p) { *p = 0ull; }

hipError_t zero_counter(unsigned long long* p, hipStream_t st) {
  hipLaunchKernelGGL(zero_one_u64_kernel, dim3(1), dim3(1), 0, st, p);
  return hipGetLastError();
}

}  // namespace snp
