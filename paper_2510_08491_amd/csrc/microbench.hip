// Device-rate and accuracy probes for the roofline denominators of the
// rasterizer: plain FP32 FMA issue rate, the hardware transcendentals
// (sin/cos in revolutions, exp2, rcp, sqrt) issue rate and accuracy, and HBM
// copy bandwidth.  Prints one JSON object.
//
// Built as a stand-alone executable; every kernel indexes only inside the
// buffers it is given (grid * block == element count, checked on the host).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                      \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      std::fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, \
                   __LINE__);                                                         \
      std::exit(1);                                                                   \
    }                                                                                 \
  } while (0)

enum Op { OP_FMA = 0, OP_SIN, OP_COS, OP_EXP2, OP_RCP, OP_SQRT, OP_MIX };

template <int OP>
__global__ void __launch_bounds__(256) rate_kernel(float* out, int iters, float seed) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  float a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = seed * (gid + 1) * (k + 1) * 1e-7f;
  const float m = 0.999f, c = 1e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (OP == OP_FMA) a[k] = __builtin_fmaf(a[k], m, c);
      if (OP == OP_SIN) a[k] = __builtin_amdgcn_sinf(a[k]);
      if (OP == OP_COS) a[k] = __builtin_amdgcn_cosf(a[k]);
      if (OP == OP_EXP2) a[k] = __builtin_amdgcn_exp2f(a[k]) - 1.0f;
      if (OP == OP_RCP) a[k] = __builtin_amdgcn_rcpf(a[k] + 2.0f);
      if (OP == OP_SQRT) a[k] = __builtin_amdgcn_sqrtf(a[k]);
      if (OP == OP_MIX) {  // one transcendental per 4 FMAs
        a[k] = __builtin_fmaf(a[k], m, c);
        a[k] = __builtin_fmaf(a[k], m, c);
        a[k] = __builtin_fmaf(a[k], m, c);
        a[k] = __builtin_amdgcn_sinf(__builtin_fmaf(a[k], m, c));
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  out[gid] = s;
}

__global__ void __launch_bounds__(256) accuracy_kernel(const float* x, float* out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = x[i];
  out[5 * i + 0] = __builtin_amdgcn_sinf(v);
  out[5 * i + 1] = __builtin_amdgcn_cosf(v);
  out[5 * i + 2] = __builtin_amdgcn_exp2f(-v * v);
  out[5 * i + 3] = __builtin_amdgcn_rcpf(1.0f + v * v);
  out[5 * i + 4] = __builtin_amdgcn_sqrtf(1.0f + v * v);
}

__global__ void __launch_bounds__(256) copy_kernel(const float4* __restrict__ a, float4* __restrict__ b,
                                                   long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long stride = (long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) b[i] = a[i];
}

int main() {
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  const int cus = prop.multiProcessorCount;
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));

  // --- issue rates ---------------------------------------------------------
  const int blocks = cus * 16, threads = 256, iters = 4096;
  float* out;
  CHECK(hipMalloc(&out, sizeof(float) * blocks * threads));
  const char* names[] = {"fma", "sin", "cos", "exp2", "rcp", "sqrt", "mix_4fma_1sin"};
  double rates[7];
  for (int op = 0; op < 7; ++op) {
    auto launch = [&]() {
      switch (op) {
        case 0: rate_kernel<OP_FMA><<<blocks, threads>>>(out, iters, 1.f); break;
        case 1: rate_kernel<OP_SIN><<<blocks, threads>>>(out, iters, 1.f); break;
        case 2: rate_kernel<OP_COS><<<blocks, threads>>>(out, iters, 1.f); break;
        case 3: rate_kernel<OP_EXP2><<<blocks, threads>>>(out, iters, 1.f); break;
        case 4: rate_kernel<OP_RCP><<<blocks, threads>>>(out, iters, 1.f); break;
        case 5: rate_kernel<OP_SQRT><<<blocks, threads>>>(out, iters, 1.f); break;
        default: rate_kernel<OP_MIX><<<blocks, threads>>>(out, iters, 1.f); break;
      }
    };
    launch();
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0));
    for (int r = 0; r < 3; ++r) launch();
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double per = (op == 6) ? 5.0 : 1.0;
    const double ops = 3.0 * blocks * threads * (double)iters * 8.0 * per;
    rates[op] = ops / (ms * 1e-3);  // lane-instructions per second
  }

  // --- accuracy --------------------------------------------------------------
  const int n = 1 << 22;
  std::vector<float> hx(n);
  for (int i = 0; i < n; ++i) hx[i] = -4.0f + 8.0f * (float)i / (float)n;
  float *dx, *dy;
  CHECK(hipMalloc(&dx, sizeof(float) * n));
  CHECK(hipMalloc(&dy, sizeof(float) * 5 * n));
  CHECK(hipMemcpy(dx, hx.data(), sizeof(float) * n, hipMemcpyHostToDevice));
  if ((n + 255) / 256 * 256 < n) return 1;
  accuracy_kernel<<<(n + 255) / 256, 256>>>(dx, dy, n);
  CHECK(hipDeviceSynchronize());
  std::vector<float> hy(5 * (size_t)n);
  CHECK(hipMemcpy(hy.data(), dy, sizeof(float) * 5 * n, hipMemcpyDeviceToHost));
  double err[5] = {0, 0, 0, 0, 0}, rel[5] = {0, 0, 0, 0, 0};
  const double twopi = 6.283185307179586476925286766559;
  for (int i = 0; i < n; ++i) {
    const double v = hx[i];
    const double ref[5] = {std::sin(twopi * v), std::cos(twopi * v), std::exp2(-(double)(hx[i] * hx[i])),
                           1.0 / (1.0 + (double)(hx[i] * hx[i])), std::sqrt(1.0 + (double)(hx[i] * hx[i]))};
    for (int k = 0; k < 5; ++k) {
      const double e = std::fabs((double)hy[5 * (size_t)i + k] - ref[k]);
      if (e > err[k]) err[k] = e;
      const double r = e / std::fmax(std::fabs(ref[k]), 1e-30);
      if (k >= 2 && r > rel[k]) rel[k] = r;
    }
  }
  // small-argument relative accuracy of sin (revolutions)
  double sin_small_rel = 0;
  {
    std::vector<float> hs(n);
    for (int i = 0; i < n; ++i) hs[i] = 1e-6f + 0.01f * (float)i / (float)n;
    CHECK(hipMemcpy(dx, hs.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    accuracy_kernel<<<(n + 255) / 256, 256>>>(dx, dy, n);
    CHECK(hipDeviceSynchronize());
    CHECK(hipMemcpy(hy.data(), dy, sizeof(float) * 5 * n, hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) {
      const double ref = std::sin(twopi * (double)hs[i]);
      const double r = std::fabs((double)hy[5 * (size_t)i] - ref) / ref;
      if (r > sin_small_rel) sin_small_rel = r;
    }
  }

  // --- HBM copy ------------------------------------------------------------------
  const long nbytes = 4L << 30;
  const long n4 = nbytes / 16;
  float4 *a, *b;
  CHECK(hipMalloc(&a, nbytes));
  CHECK(hipMalloc(&b, nbytes));
  CHECK(hipMemset(a, 0, nbytes));
  copy_kernel<<<cus * 32, 256>>>(a, b, n4);
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0));
  for (int r = 0; r < 5; ++r) copy_kernel<<<cus * 32, 256>>>(a, b, n4);
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  const double copy_gbs = 5.0 * 2.0 * nbytes / (ms * 1e-3) / 1e9;

  std::printf("{\"device\": \"%s\", \"cus\": %d, \"clock_khz\": %d,\n", prop.gcnArchName, cus,
              prop.clockRate);
  for (int op = 0; op < 7; ++op)
    std::printf("  \"rate_%s_lane_ops_per_s\": %.4e,\n", names[op], rates[op]);
  std::printf("  \"fma_over_sin\": %.3f, \"fma_over_exp2\": %.3f, \"fma_over_rcp\": %.3f, \"fma_over_sqrt\": %.3f,\n",
              rates[0] / rates[1], rates[0] / rates[3], rates[0] / rates[4], rates[0] / rates[5]);
  std::printf("  \"abs_err_sin_rev\": %.3e, \"abs_err_cos_rev\": %.3e, \"rel_err_exp2\": %.3e,"
              " \"rel_err_rcp\": %.3e, \"rel_err_sqrt\": %.3e, \"rel_err_sin_small\": %.3e,\n",
              err[0], err[1], rel[2], rel[3], rel[4], sin_small_rel);
  std::printf("  \"copy_GBps\": %.1f}\n", copy_gbs);
  return 0;
}
