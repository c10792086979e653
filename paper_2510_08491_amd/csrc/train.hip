// Training-step extras after the backward: Adam over every parameter group
// in one launch, the scale regulariser, and population control by the
// gradient magnitude of the primitives' density-MLP weights (Sec. 3.3,
// "Training" and "Population Control"; the appendix on hyperparameters).
//
// All of it is bound by HBM traffic (a few flops per float moved): plain
// grid-stride loops over coalesced rows, no LDS.
#include "snp_internal.h"

namespace snp {

// ---------------------------------------------------------------------------
// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// theta -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps); a log-space group
// updates theta = log p with gradient g p and stores p = exp(theta).
// ---------------------------------------------------------------------------
struct AdamGroupDev {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  float lr;
  int32_t log_space;
};

struct AdamArgs {
  AdamGroupDev gr[SNP_MAX_ADAM_GROUPS];
  int64_t start[SNP_MAX_ADAM_GROUPS + 1];  // first flat index of each group
  int32_t ng;
  float b1, b2, eps, inv_bc1, inv_bc2;
  float omb1, omb2;  // 1 - b1, 1 - b2 rounded from float64
};

__global__ void __launch_bounds__(256) adam_kernel(AdamArgs a) {
  const int64_t total = a.start[a.ng];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int k = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    while (i >= a.start[k + 1]) ++k;  // indices only grow, so k only moves forward
    const AdamGroupDev& G = a.gr[k];
    const int64_t j = i - a.start[k];
    const float p = G.p[j];
    float g = G.g[j];
    float theta = p;
    if (G.log_space) {
      theta = logf(p);
      g *= p;
    }
    const float m = a.b1 * G.m[j] + a.omb1 * g;
    const float v = a.b2 * G.v[j] + a.omb2 * g * g;
    G.m[j] = m;
    G.v[j] = v;
    theta -= G.lr * (m * a.inv_bc1) / (sqrtf(v * a.inv_bc2) + a.eps);
    G.p[j] = G.log_space ? expf(theta) : theta;
  }
}

hipError_t launch_adam(const snp_adam_group* groups, int ng, int64_t step, double b1, double b2, double eps,
                       hipStream_t st) {
  AdamArgs a;
  a.ng = ng;
  a.b1 = (float)b1;
  a.b2 = (float)b2;
  a.eps = (float)eps;
  a.omb1 = (float)(1.0 - b1);
  a.omb2 = (float)(1.0 - b2);
  a.inv_bc1 = (float)(1.0 / (1.0 - std::pow(b1, (double)step)));
  a.inv_bc2 = (float)(1.0 / (1.0 - std::pow(b2, (double)step)));
  int64_t total = 0;
  for (int k = 0; k < ng; ++k) {
    a.start[k] = total;
    a.gr[k] = AdamGroupDev{groups[k].param, groups[k].grad, groups[k].m, groups[k].v, groups[k].n, groups[k].lr,
                           groups[k].log_space};
    total += groups[k].n;
  }
  for (int k = ng; k <= SNP_MAX_ADAM_GROUPS; ++k) a.start[k] = total;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scale regulariser: weight / P * sum_p std(s_p) (population std of the three
// components); gradient weight / P * (s_i - mean) / (3 std), 0 at std = 0.
// Loss summed in float64, per-block partials then one block, fixed order.
// ---------------------------------------------------------------------------
constexpr int kRegBlocks = 1024;  // fits the workspace's loss scratch

__global__ void __launch_bounds__(256) scale_reg_kernel(int64_t P, const float* __restrict__ s, float wp,
                                                        float* __restrict__ gs, double* __restrict__ partials) {
  // no contraction: s_i - mean fused into one FMA would keep the unrounded
  // product and make an exactly isotropic primitive look anisotropic
#pragma clang fp contract(off)
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256) {
    const float s0 = s[3 * p], s1 = s[3 * p + 1], s2 = s[3 * p + 2];
    const float mean = (s0 + s1 + s2) * (1.f / 3.f);
    const float d0 = s0 - mean, d1 = s1 - mean, d2 = s2 - mean;
    const float sd = sqrtf((d0 * d0 + d1 * d1 + d2 * d2) * (1.f / 3.f));
    acc += (double)sd;
    if (gs && sd > 0.f) {
      const float c = wp / (3.f * sd);
      gs[3 * p] += c * d0;
      gs[3 * p + 1] += c * d1;
      gs[3 * p + 2] += c * d2;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) reg_final_kernel(const double* __restrict__ partials, int n, double scale,
                                                        double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += partials[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
}

hipError_t launch_scale_reg(int64_t P, const float* scales, float weight, float* grad, double* partials,
                            double* loss_out, hipStream_t st) {
  int64_t blocks = (P + 255) / 256;
  if (blocks > kRegBlocks) blocks = kRegBlocks;
  const double wp = (double)weight / (double)P;
  hipLaunchKernelGGL(scale_reg_kernel, dim3((unsigned)blocks), dim3(256), 0, st, P, scales, (float)wp, grad, partials);
  hipLaunchKernelGGL(reg_final_kernel, dim3(1), dim3(256), 0, st, partials, (int)blocks, wp, loss_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// population control
// ---------------------------------------------------------------------------
// acc += ||d loss / d (W1, b1, W2, b2)||_2, count += 1 if the primitive covers
// a tile of any view (tile counts of the last preprocess, V x P).  Sixteen
// lanes (one row of the wave) per primitive, so that a row reads each of
// the primitive's gradient arrays in 64-byte runs; the row then sums its
// squares and ORs its visibility.
__global__ void __launch_bounds__(256) densify_acc_kernel(int64_t P, int N, int V, const float* __restrict__ gw1,
                                                          const float* __restrict__ gb1, const float* __restrict__ gw2,
                                                          const float* __restrict__ gb2,
                                                          const uint32_t* __restrict__ tile_counts,
                                                          float* __restrict__ acc, float* __restrict__ cnt) {
  const int64_t p = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4;
  const int l = threadIdx.x & 15;
  float ss = 0.f;
  bool vis = false;
  if (p < P) {
    for (int k = l; k < 3 * N; k += 16) {
      const float x = gw1[p * 3 * N + k];
      ss += x * x;
    }
    for (int k = l; k < N; k += 16) {
      const float x = gb1[p * N + k], y = gw2[p * N + k];
      ss += x * x + y * y;
    }
    if (l == 0) ss += gb2[p] * gb2[p];
    for (int v = l; v < V; v += 16) vis = vis || tile_counts[(int64_t)v * P + p] > 0;
  }
  // the row's sum (partners within the row of 16 lanes)
  ss += __shfl_xor(ss, 1);
  ss += __shfl_xor(ss, 2);
  ss += __shfl_xor(ss, 4);
  ss += __shfl_xor(ss, 8);
  const unsigned long long vm = __ballot(vis);
  const int row = (threadIdx.x & 63) >> 4;
  if (l == 0 && p < P) {
    acc[p] += sqrtf(ss);
    if ((vm >> (16 * row)) & 0xFFFFull) cnt[p] += 1.f;
  }
}

hipError_t launch_densify_acc(int64_t P, int N, int V, const snp_grads& g, const uint32_t* tile_counts, float* acc,
                              float* cnt, hipStream_t st) {
  hipLaunchKernelGGL(densify_acc_kernel, dim3((unsigned)((P * 16 + 255) / 256)), dim3(256), 0, st, P, N, V, g.w1,
                     g.b1, g.w2, g.b2, tile_counts, acc, cnt);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) densify_plan_kernel(int64_t P, const float* __restrict__ s,
                                                           const float* __restrict__ acc,
                                                           const float* __restrict__ cnt, snp_density_control dc,
                                                           int32_t* __restrict__ action, uint32_t* __restrict__ rows) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const float c = cnt[p];
  const float stat = c > 0.f ? acc[p] / c : 0.f;
  const float smax = fmaxf(s[3 * p], fmaxf(s[3 * p + 1], s[3 * p + 2]));
  int32_t a = SNP_KEEP;
  if (smax > dc.prune_scale)
    a = SNP_PRUNE;
  else if (c > 0.f && stat < dc.prune_threshold)
    a = SNP_PRUNE;
  else if (stat > dc.densify_threshold)
    a = smax <= dc.grow_scale ? SNP_CLONE : SNP_SPLIT;
  action[p] = a;
  rows[p] = a == SNP_PRUNE ? 0u : (a == SNP_KEEP ? 1u : 2u);
}

size_t densify_scratch_bytes(int64_t P) { return ((size_t)P * 4 + 255) / 256 * 256 + scan_scratch_bytes(P); }

hipError_t launch_densify_plan(int64_t P, const float* scales, const float* acc, const float* cnt,
                               const snp_density_control& dc, int32_t* action, uint32_t* offsets, int64_t* new_count,
                               void* scratch, hipStream_t st) {
  uint32_t* rows = reinterpret_cast<uint32_t*>(scratch);
  char* scan_scr = reinterpret_cast<char*>(scratch) + ((size_t)P * 4 + 255) / 256 * 256;
  hipLaunchKernelGGL(densify_plan_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, scales, acc, cnt,
                     dc, action, rows);
  return scan_exclusive_u32(rows, offsets, P, scan_scr, reinterpret_cast<uint64_t*>(new_count), st);
}

// One array: thread per (primitive, column); the output rows of primitive p
// start at offsets[p].
__global__ void __launch_bounds__(256) densify_apply_kernel(int64_t P, const int32_t* __restrict__ action,
                                                            const uint32_t* __restrict__ offsets,
                                                            const float* __restrict__ centers,
                                                            const float* __restrict__ scales,
                                                            const float* __restrict__ quats,
                                                            const float* __restrict__ noise, float shrink,
                                                            snp_row_array arr) {
  const int w = arr.width;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= P * w) return;
  const int64_t p = t / w;
  const int c = (int)(t - p * w);
  const int32_t a = action[p];
  if (a == SNP_PRUNE) return;
  const float val = arr.src[t];
  const int64_t r0 = offsets[p];
  const int nrows = a == SNP_KEEP ? 1 : 2;
  for (int r = 0; r < nrows; ++r) {
    float out = val;
    if (arr.kind == SNP_ROWS_STATE) {
      out = (r == 0 && a != SNP_SPLIT) ? val : 0.f;  // new rows start from zero
    } else if (a == SNP_SPLIT && arr.kind == SNP_ROWS_SCALES) {
      out = val / shrink;
    } else if (a == SNP_SPLIT && arr.kind == SNP_ROWS_CENTERS) {
      // x + R(q) diag(s) u, u the child's standard normal draw
      const float q0 = quats[4 * p], q1 = quats[4 * p + 1], q2 = quats[4 * p + 2], q3 = quats[4 * p + 3];
      const float qn = rsqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
      const float qw = q0 * qn, qx = q1 * qn, qy = q2 * qn, qz = q3 * qn;
      float R0, R1, R2;  // row c of R
      if (c == 0) {
        R0 = 1.f - 2.f * (qy * qy + qz * qz); R1 = 2.f * (qx * qy - qw * qz); R2 = 2.f * (qx * qz + qw * qy);
      } else if (c == 1) {
        R0 = 2.f * (qx * qy + qw * qz); R1 = 1.f - 2.f * (qx * qx + qz * qz); R2 = 2.f * (qy * qz - qw * qx);
      } else {
        R0 = 2.f * (qx * qz - qw * qy); R1 = 2.f * (qy * qz + qw * qx); R2 = 1.f - 2.f * (qx * qx + qy * qy);
      }
      const float* u = noise + (p * 2 + r) * 3;
      out = val + R0 * scales[3 * p] * u[0] + R1 * scales[3 * p + 1] * u[1] + R2 * scales[3 * p + 2] * u[2];
    }
    arr.dst[(r0 + r) * w + c] = out;
  }
}

hipError_t launch_densify_apply(int64_t P, const int32_t* action, const uint32_t* offsets, const float* centers,
                                const float* scales, const float* quats, const float* noise, float shrink,
                                const snp_row_array& arr, hipStream_t st) {
  const int64_t n = P * arr.width;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(densify_apply_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, action, offsets,
                     centers, scales, quats, noise, shrink, arr);
  return hipGetLastError();
}

}  // namespace snp
