// Per-ray relighting colour (colour mode 4), the preprocess side: the colour
// network in the ellipsoid's unit-sphere frame, and its adjoint back to the
// network's parameters, the rotation, the scales and the centres.
//
// The relighting application colours each view ray by a constant colour plus
// a per-primitive colour network of the 3D position, the ray direction and
// the light direction, the latter relative to the primitive's centre; the
// position is the ray's entry point into the bounding ellipsoid, normalised
// as the density network's input (Eq. 5).  The rasterizer evaluates it per
// (pixel, primitive) pair from the table built here (see RayColourLayout).
#include "snp_internal.h"

namespace snp {

__device__ __forceinline__ void rotation_f64(const float* qf, double Rp[3][3]) {
  const double q0 = qf[0], q1 = qf[1], q2 = qf[2], q3 = qf[3];
  const double qn = sqrt(((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3);
  const double w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
  Rp[0][0] = 1.0 - 2.0 * (y * y + z * z);
  Rp[0][1] = 2.0 * (x * y - w * z);
  Rp[0][2] = 2.0 * (x * z + w * y);
  Rp[1][0] = 2.0 * (x * y + w * z);
  Rp[1][1] = 1.0 - 2.0 * (x * x + z * z);
  Rp[1][2] = 2.0 * (y * z - w * x);
  Rp[2][0] = 2.0 * (x * z - w * y);
  Rp[2][1] = 2.0 * (y * z + w * x);
  Rp[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

// one thread per primitive: Au, Ad and the copied hidden and output layers
template <int W, int D>
__global__ void __launch_bounds__(256) ray_table_kernel(RayColourArgs a) {
  using Lt = RayColourLayout<W, D>;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.P) return;
  constexpr int K = kRayIn * W + W + (D - 1) * (W * W + W) + 3 * W + 3;
  const float* c = a.cmlp + p * K;
  double Rp[3][3];
  rotation_f64(a.quats + 4 * p, Rp);
  const double s[3] = {a.scales[3 * p], a.scales[3 * p + 1], a.scales[3 * p + 2]};
  const double m = fmax(s[0], fmax(s[1], s[2]));
  float* row = a.ctab + p * Lt::CTS;
  for (int k = 0; k < W; ++k) {
    const float* w1 = c + k * kRayIn;
    for (int j = 0; j < 3; ++j) {
      const double rs = s[j];
      row[Lt::AU + 3 * k + j] = (float)(((w1[0] * Rp[0][j] + w1[1] * Rp[1][j]) + w1[2] * Rp[2][j]) * rs / m);
      row[Lt::AD + 3 * k + j] = (float)(((w1[3] * Rp[0][j] + w1[4] * Rp[1][j]) + w1[5] * Rp[2][j]) * rs);
    }
  }
  int pos = kRayIn * W + W;  // after W1 and b1
  if (D == 2) {
    for (int i = 0; i < W * W + W; ++i) row[Lt::WH + i] = c[pos + i];
    pos += W * W + W;
  }
  for (int i = 0; i < 3 * W + 3; ++i) row[Lt::WO + i] = c[pos + i];
  for (int i = Lt::CT; i < Lt::CTS; ++i) row[i] = 0.f;
}

// one thread per (view, primitive): cb = b1 + W1[:, 6:9] normalize(l_v - x_B)
template <int W>
__global__ void __launch_bounds__(256) ray_bias_kernel(RayColourArgs a, int K) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.P * a.V) return;
  const int v = (int)(i / a.P);
  const int64_t p = i - (int64_t)v * a.P;
  float* cb = a.cbias + i * W;
  if (a.tile_counts[i] == 0) {
    for (int k = 0; k < W; ++k) cb[k] = 0.f;
    return;
  }
  const CamDev& cam = a.cams[v];
  const float lx = cam.light[0] - a.centers[3 * p];
  const float ly = cam.light[1] - a.centers[3 * p + 1];
  const float lz = cam.light[2] - a.centers[3 * p + 2];
  const float il = 1.0f / sqrtf(lx * lx + ly * ly + lz * lz);
  const float* c = a.cmlp + p * K;
  for (int k = 0; k < W; ++k) {
    const float* w1 = c + k * kRayIn;
    cb[k] = c[kRayIn * W + k] + (w1[6] * lx + w1[7] * ly + w1[8] * lz) * il;
  }
}

// Adjoint, one thread per primitive.  From the table gradients: the hidden
// and output layers directly, W1's position and direction columns, and the
// rotation and scales through Au = W1p R S / m, Ad = W1d R S (written to
// extra_rs for the preprocess adjoint, which chains them to the raw
// quaternion and the scales); from the bias gradients over the views: b1,
// W1's light columns and the centre through the light direction.
template <int W, int D>
__global__ void __launch_bounds__(256) ray_colour_bwd_kernel(RayColourArgs a) {
  using Lt = RayColourLayout<W, D>;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.P) return;
  constexpr int K = kRayIn * W + W + (D - 1) * (W * W + W) + 3 * W + 3;
  const float* c = a.cmlp + p * K;
  const float* gt = a.gctab + p * Lt::CTS;
  float* gc = a.g_cmlp ? a.g_cmlp + p * K : nullptr;
  double Rp[3][3];
  rotation_f64(a.quats + 4 * p, Rp);
  const double s[3] = {a.scales[3 * p], a.scales[3 * p + 1], a.scales[3 * p + 2]};
  const double m = fmax(s[0], fmax(s[1], s[2]));
  const int am = (s[0] >= s[1] && s[0] >= s[2]) ? 0 : (s[1] >= s[2] ? 1 : 2);
  double gR[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double gs[3] = {0, 0, 0}, gm = 0.0;
  for (int k = 0; k < W; ++k) {
    const float* w1 = c + k * kRayIn;
    for (int j = 0; j < 3; ++j) {
      const double gau = gt[Lt::AU + 3 * k + j], gad = gt[Lt::AD + 3 * k + j];
      const double au = ((w1[0] * Rp[0][j] + w1[1] * Rp[1][j]) + w1[2] * Rp[2][j]) * s[j] / m;
      gm -= gau * au / m;
      for (int ii = 0; ii < 3; ++ii) {
        gR[ii][j] += gau * w1[ii] * s[j] / m + gad * w1[3 + ii] * s[j];
        gs[j] += gau * w1[ii] * Rp[ii][j] / m + gad * w1[3 + ii] * Rp[ii][j];
      }
    }
    if (gc) {
      for (int ii = 0; ii < 3; ++ii) {
        double gp = 0.0, gd = 0.0;
        for (int j = 0; j < 3; ++j) {
          gp += (double)gt[Lt::AU + 3 * k + j] * Rp[ii][j] * s[j] / m;
          gd += (double)gt[Lt::AD + 3 * k + j] * Rp[ii][j] * s[j];
        }
        gc[k * kRayIn + ii] += (float)gp;
        gc[k * kRayIn + 3 + ii] += (float)gd;
      }
    }
  }
  gs[am] += gm;
  if (gc) {
    int pos = kRayIn * W + W;
    if (D == 2) {
      for (int i = 0; i < W * W + W; ++i) gc[pos + i] += gt[Lt::WH + i];
      pos += W * W + W;
    }
    for (int i = 0; i < 3 * W + 3; ++i) gc[pos + i] += gt[Lt::WO + i];
  }
  // bias: b1 and the light columns per view, the light direction to x_B
  double gx[3] = {0, 0, 0};
  for (int v = 0; v < a.V; ++v) {
    const int64_t i = (int64_t)v * a.P + p;
    if (a.tile_counts[i] == 0) continue;
    const float* gb = a.gcbias + i * W;
    const CamDev& cam = a.cams[v];
    const double lv[3] = {(double)cam.light[0] - a.centers[3 * p], (double)cam.light[1] - a.centers[3 * p + 1],
                          (double)cam.light[2] - a.centers[3 * p + 2]};
    const double len = sqrt(lv[0] * lv[0] + lv[1] * lv[1] + lv[2] * lv[2]);
    const double ld[3] = {lv[0] / len, lv[1] / len, lv[2] / len};
    double gld[3] = {0, 0, 0};
    for (int k = 0; k < W; ++k) {
      const double g = gb[k];
      if (gc) {
        gc[kRayIn * W + k] += (float)g;
        for (int ii = 0; ii < 3; ++ii) gc[k * kRayIn + 6 + ii] += (float)(g * ld[ii]);
      }
      for (int ii = 0; ii < 3; ++ii) gld[ii] += g * c[k * kRayIn + 6 + ii];
    }
    // ld = (l - x_B) / |l - x_B|:  d ld / d x_B = -(I - ld ld^T) / |l - x_B|
    const double dd = ld[0] * gld[0] + ld[1] * gld[1] + ld[2] * gld[2];
    for (int ii = 0; ii < 3; ++ii) gx[ii] -= (gld[ii] - ld[ii] * dd) / len;
  }
  if (a.g_centers)
    for (int ii = 0; ii < 3; ++ii) a.g_centers[3 * p + ii] += (float)gx[ii];
  float* ex = a.extra_rs + p * 12;
  for (int ii = 0; ii < 3; ++ii)
    for (int j = 0; j < 3; ++j) ex[3 * ii + j] = (float)gR[ii][j];
  for (int j = 0; j < 3; ++j) ex[9 + j] = (float)gs[j];
}

// the rasterizers evaluate the network with one hidden layer of 16 units
bool ray_colour_supported(int width, int depth) { return width == 16 && depth == 1; }

int ray_colour_param_count(int width, int depth) {
  return kRayIn * width + width + (depth - 1) * (width * width + width) + 3 * width + 3;
}

hipError_t launch_ray_colour_fwd(const RayColourArgs& a, hipStream_t st) {
  const dim3 block(256);
  const dim3 gp((unsigned)((a.P + 255) / 256)), gv((unsigned)((a.P * a.V + 255) / 256));
  const int K = ray_colour_param_count(a.W, a.D);
  if (a.W != 16) return hipErrorInvalidValue;
  if (a.D == 1)
    hipLaunchKernelGGL((ray_table_kernel<16, 1>), gp, block, 0, st, a);
  else if (a.D == 2)
    hipLaunchKernelGGL((ray_table_kernel<16, 2>), gp, block, 0, st, a);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(ray_bias_kernel<16>, gv, block, 0, st, a, K);
  return hipGetLastError();
}

hipError_t launch_ray_colour_bwd(const RayColourArgs& a, hipStream_t st) {
  const dim3 block(256), gp((unsigned)((a.P + 255) / 256));
  if (a.W != 16) return hipErrorInvalidValue;
  if (a.D == 1)
    hipLaunchKernelGGL((ray_colour_bwd_kernel<16, 1>), gp, block, 0, st, a);
  else if (a.D == 2)
    hipLaunchKernelGGL((ray_colour_bwd_kernel<16, 2>), gp, block, 0, st, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace snp
