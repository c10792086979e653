// Per-(primitive, view) preprocessing, colour MLP, and their adjoints.
//
// Sec. 3.1 (ellipsoid bound B = {x_B, s_B, q_B}, density field Eq. 5-6) and
// Sec. 3.2 (line-ellipsoid intersection) define everything here.  The
// quantities that do not depend on the pixel are computed once per
// (primitive, view) in float64 and rounded to float32 records that the
// rasterizer evaluates per pixel:
//
//   U  = diag(1/s) R(q)^T               world -> unit-sphere frame of B
//   o' = U (o - x_B)                    camera centre in that frame
//   d'(px,py) = U R_cam^-1 ((px-cx)/fx, (py-cy)/fy, 1)   (affine in the pixel)
//   m'(px,py) = o' x d'(px,py)          moment of the ray (affine in the pixel)
//
// With A = |d'|^2 and M = |m'|^2 the ray meets B iff disc = A - M > 0; the
// chord midpoint in the frame is p' = d' x m' / A and the chord half-length
// (per unit of the un-normalised direction) is sqrt(disc) / A.
//
// The density MLP's phase along the chord is linear in p' (Eq. 5-6 with the
// normalisation of Eq. 5 made explicit); per primitive the table stores
//   Wt_k = omega0 / (2 pi m) W1_k R diag(s)   (m = max s)
//   bt_k = (omega0 b1_k + xi_t W_t,k) / (2 pi)  reduced to [-1/2, 1/2]
//          (the time term only for the time-conditioned density)
// so that phase_k / (2 pi) = Wt_k . p' + bt_k (revolutions).
//
// Culling, screen bounds and depth keys follow one fixed order of float64
// operations with contraction disabled, so that any float64 implementation
// that follows the same order produces bit-identical integers.
#include "snp_internal.h"

#pragma clang fp contract(off)

namespace snp {

// ---------------------------------------------------------------------------
// per-view constants
// ---------------------------------------------------------------------------
__global__ void setup_cams_kernel(CamChunk ch, CamDev* out) {
  const int i = threadIdx.x;
  if (i >= ch.count) return;
  const snp_camera& c = ch.cam[i];
  CamDev d;
  d.width = c.width;
  d.height = c.height;
  d.tile_w = ch.tile_w;
  d.tile_h = ch.tile_h;
  d.ntx = (c.width + ch.tile_w - 1) / ch.tile_w;
  d.nty = (c.height + ch.tile_h - 1) / ch.tile_h;
  d.tile_base = ch.tile_base[i];
  for (int k = 0; k < 3; ++k) d.light[k] = c.light[k];
  d.pad0 = 0;
  d.pix_base = ch.pix_base[i];
  d.fx = c.fx;
  d.fy = c.fy;
  d.cx = c.cx;
  d.cy = c.cy;
  for (int k = 0; k < 9; ++k) d.R[k] = c.R[k];
  for (int k = 0; k < 3; ++k) d.t[k] = c.t[k];
  // exact inverse of the stored (float32, nearly orthogonal) matrix
  const double a = c.R[0], b = c.R[1], e = c.R[2];
  const double f = c.R[3], g = c.R[4], h = c.R[5];
  const double p = c.R[6], q = c.R[7], r = c.R[8];
  const double A0 = g * r - h * q, A1 = -(b * r - e * q), A2 = b * h - e * g;
  const double B0 = -(f * r - h * p), B1 = a * r - e * p, B2 = -(a * h - e * f);
  const double C0 = f * q - g * p, C1 = -(a * q - b * p), C2 = a * g - b * f;
  const double det = a * A0 + b * B0 + e * C0;
  const double inv = 1.0 / det;
  const double Ri[9] = {A0 * inv, A1 * inv, A2 * inv, B0 * inv, B1 * inv, B2 * inv, C0 * inv, C1 * inv, C2 * inv};
  for (int k = 0; k < 9; ++k) {
    d.Rinv[k] = Ri[k];
    d.Rinv_f[k] = (float)Ri[k];
  }
  for (int k = 0; k < 3; ++k) {
    d.o[k] = -(Ri[3 * k] * (double)c.t[0] + Ri[3 * k + 1] * (double)c.t[1] + Ri[3 * k + 2] * (double)c.t[2]);
    d.o_f[k] = (float)d.o[k];
  }
  out[ch.first + i] = d;
}

// Rotation of a quaternion (w, x, y, z), normalised first; fixed op order.
__device__ __forceinline__ void quat_rot_f64(const float* qf, double Rp[3][3], double qn_out[4], double* qnorm) {
  const double q0 = qf[0], q1 = qf[1], q2 = qf[2], q3 = qf[3];
  const double qn = sqrt(((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3);
  const double w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
  const double xx = x * x, yy = y * y, zz = z * z;
  const double xy = x * y, xz = x * z, yz = y * z;
  const double wx = w * x, wy = w * y, wz = w * z;
  Rp[0][0] = 1.0 - 2.0 * (yy + zz);
  Rp[0][1] = 2.0 * (xy - wz);
  Rp[0][2] = 2.0 * (xz + wy);
  Rp[1][0] = 2.0 * (xy + wz);
  Rp[1][1] = 1.0 - 2.0 * (xx + zz);
  Rp[1][2] = 2.0 * (yz - wx);
  Rp[2][0] = 2.0 * (xz - wy);
  Rp[2][1] = 2.0 * (yz + wx);
  Rp[2][2] = 1.0 - 2.0 * (xx + yy);
  if (qn_out) {
    qn_out[0] = w;
    qn_out[1] = x;
    qn_out[2] = y;
    qn_out[3] = z;
  }
  if (qnorm) *qnorm = qn;
}

// ---------------------------------------------------------------------------
// per-primitive density table (view independent)
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(256) prim_table_kernel(int64_t P, float omega0, const float* __restrict__ scales,
                                                         const float* __restrict__ quats,
                                                         const float* __restrict__ w1, const float* __restrict__ b1,
                                                         const float* __restrict__ w2, const float* __restrict__ b2,
                                                         const float* __restrict__ w_time, float time,
                                                         float* __restrict__ table, unsigned long long* counters) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  constexpr int TS = 5 * N + 4;
  double Rp[3][3];
  quat_rot_f64(quats + 4 * p, Rp, nullptr, nullptr);
  const double s0 = scales[3 * p], s1 = scales[3 * p + 1], s2 = scales[3 * p + 2];
  const double m = fmax(s0, fmax(s1, s2));
  const double K = (double)omega0 / (6.283185307179586476925 * m);
  const double s[3] = {s0, s1, s2};
  float* row = table + p * TS;
  bool bad = false;
  for (int k = 0; k < N; ++k) {
    const float* wk = w1 + (p * N + k) * 3;
    double wt[3];
    double l1 = 0.0;
    for (int j = 0; j < 3; ++j) {
      wt[j] = K * ((wk[0] * Rp[0][j] + wk[1] * Rp[1][j] + wk[2] * Rp[2][j]) * s[j]);
      l1 += fabs(wt[j]);
    }
    double bt = (double)omega0 * (double)b1[p * N + k] / 6.283185307179586476925;
    if (w_time) bt += (double)time * (double)w_time[p * N + k] / 6.283185307179586476925;  // time-conditioned phase
    bt -= rint(bt);
    if (!(l1 < 255.0)) bad = true;
    row[4 * k + 0] = (float)wt[0];
    row[4 * k + 1] = (float)wt[1];
    row[4 * k + 2] = (float)wt[2];
    row[4 * k + 3] = (float)bt;
    row[4 * N + k] = (float)((double)w2[p * N + k] / 6.283185307179586476925);
  }
  row[5 * N] = b2[p];
  row[5 * N + 1] = 0.f;
  row[5 * N + 2] = 0.f;
  row[5 * N + 3] = 0.f;
  if (bad) atomicOr(&counters[CNT_RANGE], 1ull);
}

// ---------------------------------------------------------------------------
// per-(view, primitive): key path + record
// ---------------------------------------------------------------------------

// one tangent-line pair of the projected outline -> inclusive pixel range
__device__ __forceinline__ void outline_extent(double Ma, double Mb, double M22, double f, double cc, double size,
                                               double* lo, double* hi, double* p_lo, double* p_hi) {
  double disc = Mb * Mb - Ma * M22;
  disc = disc > 0.0 ? disc : 0.0;
  const double sq = sqrt(disc);
  const double u_lo = (Mb + sq) / M22;
  const double u_hi = (Mb - sq) / M22;
  *p_lo = f * u_lo + cc;
  *p_hi = f * u_hi + cc;
  double l = ceil((*p_lo - 0.5) - kEpsPx);
  double h = floor((*p_hi - 0.5) + kEpsPx);
  l = l > 0.0 ? l : 0.0;
  h = h < size - 1.0 ? h : size - 1.0;
  *lo = l;
  *hi = h;
}

// ---------------------------------------------------------------------------
// Gaussian splats (the 3DGS kernel the paper compares against, App. A):
// key path and record of one (view, primitive) pair.  Steps in one fixed
// float64 order (contraction off):
//   Sigma = Rc diag(s^2) Rc^T in camera space, mu = C x_B + t;
//   kept iff mu_z > z_near and det > 0 below;
//   J = [[fx/z, 0, -fx xc/z^2], [0, fy/z, -fy yc/z^2]] with x/z, y/z clamped
//   to 1.3 times the view for xc, yc;
//   (a, b; b, c) = J Sigma J^T + 0.3 I, computed as (J Sigma) J^T;
//   r = ceil(3 sqrt(mid + sqrt(max(0.1, mid^2 - det)))), mid = (a + c)/2;
//   pixel columns [ceil(u - r - 1/2), floor(u + r - 1/2)], u = fx x/z + cx.
// ---------------------------------------------------------------------------
constexpr double kLowPass = 0.3;     // px^2 on the diagonal of the 2D covariance
constexpr double kViewClamp = 1.3;   // Jacobian evaluated within 1.3x the view
constexpr double kEigFloor = 0.1;    // floor of the eigenvalue discriminant

__device__ void gaussian_view(const ViewArgs& a, int64_t i, int64_t p, const CamDev& cam) {
  double Rp[3][3];
  quat_rot_f64(a.quats + 4 * p, Rp, nullptr, nullptr);
  const double xb[3] = {a.centers[3 * p], a.centers[3 * p + 1], a.centers[3 * p + 2]};
  const double ss[3] = {(double)a.scales[3 * p] * a.scales[3 * p], (double)a.scales[3 * p + 1] * a.scales[3 * p + 1],
                        (double)a.scales[3 * p + 2] * a.scales[3 * p + 2]};
  double C[3][3], t[3];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) C[r][c] = cam.R[3 * r + c];
    t[r] = cam.t[r];
  }
  double Rc[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Rc[r][c] = (C[r][0] * Rp[0][c] + C[r][1] * Rp[1][c]) + C[r][2] * Rp[2][c];
  double mu[3];
  for (int r = 0; r < 3; ++r) mu[r] = ((C[r][0] * xb[0] + C[r][1] * xb[1]) + C[r][2] * xb[2]) + t[r];
  double S[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      S[r][c] = ((Rc[r][0] * ss[0]) * Rc[c][0] + (Rc[r][1] * ss[1]) * Rc[c][1]) + (Rc[r][2] * ss[2]) * Rc[c][2];
  const double mz = mu[2];
  const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
  const double xzr = mu[0] / mz, yzr = mu[1] / mz;
  const double lxl = -kViewClamp * (cx / fx), lxh = kViewClamp * (((double)cam.width - cx) / fx);
  const double lyl = -kViewClamp * (cy / fy), lyh = kViewClamp * (((double)cam.height - cy) / fy);
  const double xc = fmin(fmax(xzr, lxl), lxh) * mz;
  const double yc = fmin(fmax(yzr, lyl), lyh) * mz;
  const double zz2 = mz * mz;
  const double j00 = fx / mz, j02 = -(fx * xc) / zz2;
  const double j11 = fy / mz, j12 = -(fy * yc) / zz2;
  double T0[3], T1[3];
  for (int k = 0; k < 3; ++k) {
    T0[k] = j00 * S[0][k] + j02 * S[2][k];
    T1[k] = j11 * S[1][k] + j12 * S[2][k];
  }
  const double ca = (T0[0] * j00 + T0[2] * j02) + kLowPass;
  const double cb = T0[1] * j11 + T0[2] * j12;
  const double cc = (T1[1] * j11 + T1[2] * j12) + kLowPass;
  const double det = ca * cc - cb * cb;
  const bool keep = mz > (double)a.z_near && det > 0.0;

  uint32_t count = 0;
  int32_t rect[4] = {0, 0, 0, 0};
  uint32_t dbits = 0;
  if (keep) {
    const double mid = 0.5 * (ca + cc);
    const double lam = mid + sqrt(fmax(kEigFloor, mid * mid - det));
    const double r = ceil(3.0 * sqrt(lam));
    const double u = fx * xzr + cx, v = fy * yzr + cy;
    double x0 = ceil((u - r) - 0.5), x1 = floor((u + r) - 0.5);
    double y0 = ceil((v - r) - 0.5), y1 = floor((v + r) - 0.5);
    x0 = x0 > 0.0 ? x0 : 0.0;
    x1 = x1 < (double)cam.width - 1.0 ? x1 : (double)cam.width - 1.0;
    y0 = y0 > 0.0 ? y0 : 0.0;
    y1 = y1 < (double)cam.height - 1.0 ? y1 : (double)cam.height - 1.0;
    if (x0 <= x1 && y0 <= y1) {
      rect[0] = (int32_t)x0;
      rect[1] = (int32_t)x1;
      rect[2] = (int32_t)y0;
      rect[3] = (int32_t)y1;
      const int tx0 = rect[0] / cam.tile_w, tx1 = rect[1] / cam.tile_w;
      const int ty0 = rect[2] / cam.tile_h, ty1 = rect[3] / cam.tile_h;
      count = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
      dbits = __float_as_uint((float)mz);
      // conic (the inverse covariance) scaled to log2 of the Gaussian factor
      const double L2 = 1.4426950408889634074;
      const double ka = -0.5 * L2 * (cc / det), kb = L2 * (cb / det), kc = -0.5 * L2 * (ca / det);
      float* rec = a.records + i * kRecFloats;
      float4* r4 = reinterpret_cast<float4*>(rec);
      const float cr = a.color_mode == 0 ? a.colors[3 * p] : 0.f;
      const float cg = a.color_mode == 0 ? a.colors[3 * p + 1] : 0.f;
      const float cbl = a.color_mode == 0 ? a.colors[3 * p + 2] : 0.f;
      r4[0] = make_float4(0.f, 0.f, 0.f, 0.f);
      r4[1] = make_float4(0.f, 0.f, 0.f, 0.f);
      r4[2] = make_float4((float)u, (float)v, (float)ka, cr);
      r4[3] = make_float4((float)kb, (float)kc, a.opacity[p], cg);
      r4[4] = make_float4(0.f, 0.f, 0.f, cbl);
      r4[5] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  a.rects[4 * i + 0] = rect[0];
  a.rects[4 * i + 1] = rect[1];
  a.rects[4 * i + 2] = rect[2];
  a.rects[4 * i + 3] = rect[3];
  a.depth_bits[i] = dbits;
  a.tile_counts[i] = count;
}

__global__ void __launch_bounds__(256) preprocess_views_kernel(ViewArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.P * a.V) return;
  const int v = (int)(i / a.P);
  const int64_t p = i - (int64_t)v * a.P;
  const CamDev& cam = a.cams[v];
  if (a.primitive == 1) {
    gaussian_view(a, i, p, cam);
    return;
  }

  double Rp[3][3];
  quat_rot_f64(a.quats + 4 * p, Rp, nullptr, nullptr);
  const double xb[3] = {a.centers[3 * p], a.centers[3 * p + 1], a.centers[3 * p + 2]};
  const double s[3] = {a.scales[3 * p], a.scales[3 * p + 1], a.scales[3 * p + 2]};
  double C[3][3], t[3];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) C[r][c] = cam.R[3 * r + c];
    t[r] = cam.t[r];
  }
  // camera-frame rotation, centre and shape matrix
  double Rc[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Rc[r][c] = (C[r][0] * Rp[0][c] + C[r][1] * Rp[1][c]) + C[r][2] * Rp[2][c];
  double mu[3];
  for (int r = 0; r < 3; ++r) mu[r] = ((C[r][0] * xb[0] + C[r][1] * xb[1]) + C[r][2] * xb[2]) + t[r];
  const double ss[3] = {s[0] * s[0], s[1] * s[1], s[2] * s[2]};
  auto sig = [&](int r, int c) {
    return (((Rc[r][0] * ss[0]) * Rc[c][0] + (Rc[r][1] * ss[1]) * Rc[c][1]) + (Rc[r][2] * ss[2]) * Rc[c][2]);
  };
  const double S00 = sig(0, 0), S02 = sig(0, 2), S11 = sig(1, 1), S12 = sig(1, 2), S22 = sig(2, 2);
  const bool keep = (mu[2] - sqrt(S22)) > (double)a.z_near;

  uint32_t count = 0;
  int32_t rect[4] = {0, 0, 0, 0};
  uint32_t dbits = 0;
  float* rec = a.records + i * kRecFloats;
  if (keep) {
    const double M00 = S00 - mu[0] * mu[0];
    const double M02 = S02 - mu[0] * mu[2];
    const double M11 = S11 - mu[1] * mu[1];
    const double M12 = S12 - mu[1] * mu[2];
    const double M22 = S22 - mu[2] * mu[2];
    double x0, x1, y0, y1, pxl, pxh, pyl, pyh;
    outline_extent(M00, M02, M22, (double)cam.fx, (double)cam.cx, (double)cam.width, &x0, &x1, &pxl, &pxh);
    outline_extent(M11, M12, M22, (double)cam.fy, (double)cam.cy, (double)cam.height, &y0, &y1, &pyl, &pyh);
    if (x0 <= x1 && y0 <= y1) {
      rect[0] = (int32_t)x0;
      rect[1] = (int32_t)x1;
      rect[2] = (int32_t)y0;
      rect[3] = (int32_t)y1;
      const int tx0 = rect[0] / cam.tile_w, tx1 = rect[1] / cam.tile_w;
      const int ty0 = rect[2] / cam.tile_h, ty1 = rect[3] / cam.tile_h;
      count = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
      dbits = __float_as_uint((float)mu[2]);

      // ---- record (float64 -> float32) ----
      const float rxf = (float)(0.5 * (pxl + pxh));
      const float ryf = (float)(0.5 * (pyl + pyh));
      double U[3][3];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) U[r][c] = Rp[c][r] / s[r];
      double om[3] = {cam.o[0] - xb[0], cam.o[1] - xb[1], cam.o[2] - xb[2]};
      double op[3], G[3][3];
      for (int r = 0; r < 3; ++r) {
        op[r] = U[r][0] * om[0] + U[r][1] * om[1] + U[r][2] * om[2];
        for (int c = 0; c < 3; ++c)
          G[r][c] = U[r][0] * cam.Rinv[c] + U[r][1] * cam.Rinv[3 + c] + U[r][2] * cam.Rinv[6 + c];
      }
      const double vr[3] = {((double)rxf - cam.cx) / cam.fx, ((double)ryf - cam.cy) / cam.fy, 1.0};
      double dc[3], gx[3], gy[3];
      for (int r = 0; r < 3; ++r) {
        dc[r] = G[r][0] * vr[0] + G[r][1] * vr[1] + G[r][2] * vr[2];
        gx[r] = G[r][0] / cam.fx;
        gy[r] = G[r][1] / cam.fy;
      }
      auto cross = [](const double* u, const double* w, double* out) {
        out[0] = u[1] * w[2] - u[2] * w[1];
        out[1] = u[2] * w[0] - u[0] * w[2];
        out[2] = u[0] * w[1] - u[1] * w[0];
      };
      double mc[3], hx[3], hy[3];
      cross(op, dc, mc);
      cross(op, gx, hx);
      cross(op, gy, hy);
      float4* r4 = reinterpret_cast<float4*>(rec);
      r4[0] = make_float4((float)dc[0], (float)dc[1], (float)dc[2], rxf);
      r4[1] = make_float4((float)gx[0], (float)gx[1], (float)gx[2], ryf);
      float cr = 0.f, cg = 0.f, cb = 0.f;
      if (a.color_mode == 0 || a.color_mode == 4) {  // the constant colour, or c_dc of the per-ray colour
        cr = a.colors[3 * p];
        cg = a.colors[3 * p + 1];
        cb = a.colors[3 * p + 2];
      }
      r4[2] = make_float4((float)gy[0], (float)gy[1], (float)gy[2], cr);
      r4[3] = make_float4((float)mc[0], (float)mc[1], (float)mc[2], cg);
      r4[4] = make_float4((float)hx[0], (float)hx[1], (float)hx[2], cb);
      // Width of the band around the silhouette in which the rasterizer
      // decides a hit by the float64 coefficients below: 64 times a bound on
      // the error of the float32 discriminant A - M it evaluates from this
      // record over the rectangle's pixel centres.  Per component of d' and
      // m' the error is at most 3 roundings (coefficients, two FMAs) of
      // S = |c0| + |c1| |dx| + |c2| |dy|; the squares and the difference add
      // 7 more, so |error| <= 10 u (sum S_d^2 + sum S_m^2), u = 2^-24.
      const double ex = fmax(fabs((double)rect[0] + 0.5 - rxf), fabs((double)rect[1] + 0.5 - rxf));
      const double ey = fmax(fabs((double)rect[2] + 0.5 - ryf), fabs((double)rect[3] + 0.5 - ryf));
      double sum_s2 = 0.0;
      for (int r = 0; r < 3; ++r) {
        const double sdr = fabs(dc[r]) + fabs(gx[r]) * ex + fabs(gy[r]) * ey;
        const double smr = fabs(mc[r]) + fabs(hx[r]) * ex + fabs(hy[r]) * ey;
        sum_s2 += sdr * sdr + smr * smr;
      }
      const float band = (float)(64.0 * 10.0 * 0x1p-24 * sum_s2);
      r4[5] = make_float4((float)hy[0], (float)hy[1], (float)hy[2], band);
      auto dot = [](const double* u, const double* w) { return u[0] * w[0] + u[1] * w[1] + u[2] * w[2]; };
      double* dq = a.disc_coef + i * 6;
      dq[0] = dot(dc, dc) - dot(mc, mc);
      dq[1] = 2.0 * (dot(dc, gx) - dot(mc, hx));
      dq[2] = 2.0 * (dot(dc, gy) - dot(mc, hy));
      dq[3] = dot(gx, gx) - dot(hx, hx);
      dq[4] = 2.0 * (dot(gx, gy) - dot(hx, hy));
      dq[5] = dot(gy, gy) - dot(hy, hy);
    }
  }
  a.rects[4 * i + 0] = rect[0];
  a.rects[4 * i + 1] = rect[1];
  a.rects[4 * i + 2] = rect[2];
  a.rects[4 * i + 3] = rect[3];
  a.depth_bits[i] = dbits;
  a.tile_counts[i] = count;
}

// ---------------------------------------------------------------------------
// colour MLP: input [normalize(x_B - o_v), xi_p], DEPTH ReLU layers of WIDTH
// units, sigmoid RGB, with weights of its own for every primitive.
// ---------------------------------------------------------------------------

// IN = 11: [view direction, xi] (colour mode 1); IN = 14: [view direction,
// light direction, xi] (relighting colour, mode 3)
template <int WIDTH, int DEPTH, int IN>
struct CmlpShape {
  static constexpr int K = IN * WIDTH + WIDTH + (DEPTH - 1) * (WIDTH * WIDTH + WIDTH) + WIDTH * 3 + 3;
};

// light direction normalize(l_v - x_B) of the relighting colour
__device__ __forceinline__ void light_dir(const CmlpArgs& a, int64_t p, const CamDev& cam, float* ld, float* inv_len) {
  const float dx = cam.light[0] - a.centers[3 * p];
  const float dy = cam.light[1] - a.centers[3 * p + 1];
  const float dz = cam.light[2] - a.centers[3 * p + 2];
  const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  ld[0] = dx * il;
  ld[1] = dy * il;
  ld[2] = dz * il;
  *inv_len = il;
}

template <int IN>
__device__ __forceinline__ void cmlp_input(const CmlpArgs& a, int64_t p, int v, float* x, float* rawdir,
                                           float* inv_len) {
  const CamDev& cam = a.cams[v];
  const float dx = a.centers[3 * p] - cam.o_f[0];
  const float dy = a.centers[3 * p + 1] - cam.o_f[1];
  const float dz = a.centers[3 * p + 2] - cam.o_f[2];
  const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  rawdir[0] = dx * il;
  rawdir[1] = dy * il;
  rawdir[2] = dz * il;
  *inv_len = il;
  x[0] = rawdir[0];
  x[1] = rawdir[1];
  x[2] = rawdir[2];
  if constexpr (IN == kCmlpIn + 3) {
    float il2;
    light_dir(a, p, cam, x + 3, &il2);
  }
#pragma unroll
  for (int k = 0; k < kXiDim; ++k) x[IN - kXiDim + k] = a.xi[p * kXiDim + k];
}

// Forward of the colour MLP on the matrix cores, one wave per primitive and 16
// of its views at a time.  Every layer is a product W (units x inputs) times X^T
// (inputs x views) in 16x16x4 FP32 steps: lane (g, c) = (lane / 16, lane %
// 16) supplies the weight of unit 16 t + c for input 4 s + g (operand A) and
// input 4 s + g of view c (operand B), and receives units 16 t + 4 g + r of
// view c in register r.  rows_to_regs then transposes those four registers
// with the wave's four rows of 16 lanes, so that lane (g, c) holds unit
// 16 t + 4 s + g of view c in register s: the next layer's operand B as it
// stands.  Each weight is loaded once per 16 views by exactly one lane.
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f rows_to_regs(v4f d) {
  // v_permlane32_swap(x, y): the upper two rows of x trade places with the
  // lower two of y; v_permlane16_swap(x, y): the odd rows of x with the even
  // rows of y.  Element (row g, register r) ends at (row r, register g).
  const auto a02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(d[0]), __float_as_uint(d[2]), false, false);
  const auto a13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(d[1]), __float_as_uint(d[3]), false, false);
  const auto b01 = __builtin_amdgcn_permlane16_swap(a02[0], a13[0], false, false);
  const auto b23 = __builtin_amdgcn_permlane16_swap(a02[1], a13[1], false, false);
  return v4f{__uint_as_float(b01[0]), __uint_as_float(b01[1]), __uint_as_float(b23[0]), __uint_as_float(b23[1])};
}

template <int WIDTH, int DEPTH, int IN>
__global__ void __launch_bounds__(256) cmlp_fwd_mfma_kernel(CmlpArgs a) {
  const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);  // one wave per primitive
  if (p >= a.P) return;  // wave-uniform
  const int lane = (int)(threadIdx.x & 63), g = lane >> 4, c = lane & 15;
  constexpr int K = CmlpShape<WIDTH, DEPTH, IN>::K;
  constexpr int T = WIDTH / 16;     // tiles of 16 units
  constexpr int S0 = (IN + 3) / 4;  // steps of four inputs in the first layer
  const float* Wp = a.cmlp + p * K;
  for (int v0 = 0; v0 < a.V; v0 += 16) {
    const int v = v0 + c;
    const bool vis = v < a.V && a.tile_counts[(int64_t)v * a.P + p] != 0;
    if (__ballot(vis) == 0) continue;  // wave-uniform
    float x[IN], dir[3], il;
    cmlp_input<IN>(a, p, v < a.V ? v : v0, x, dir, &il);  // lanes past the last view repeat a valid one
    float bx[S0];
#pragma unroll
    for (int s = 0; s < S0; ++s) {
      float t = 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (4 * s + q < IN) t = g == q ? x[4 * s + q] : t;
      bx[s] = t;
    }
    v4f h[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < S0; ++s) {
        const int k = 4 * s + g;
        const float w = k < IN ? Wp[(16 * t + c) * IN + k] : 0.f;
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(w, bx[s], d, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) d[r] = fmaxf(d[r] + Wp[IN * WIDTH + 16 * t + 4 * g + r], 0.f);
      h[t] = rows_to_regs(d);
    }
    int off = IN * WIDTH + WIDTH;
#pragma unroll
    for (int l = 1; l < DEPTH; ++l) {
      v4f nh[T];
#pragma unroll
      for (int to = 0; to < T; ++to) {
        v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int s = 0; s < 4; ++s)
            d = __builtin_amdgcn_mfma_f32_16x16x4f32(Wp[off + (16 * to + c) * WIDTH + 16 * t + 4 * s + g], h[t][s], d,
                                                     0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) d[r] = fmaxf(d[r] + Wp[off + WIDTH * WIDTH + 16 * to + 4 * g + r], 0.f);
        nh[to] = rows_to_regs(d);
      }
#pragma unroll
      for (int t = 0; t < T; ++t) h[t] = nh[t];
      off += WIDTH * WIDTH + WIDTH;
    }
    // output layer: rows 0..2 of the tile (units c < 3 carry weights)
    v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float w = c < 3 ? Wp[off + c * WIDTH + 16 * t + 4 * s + g] : 0.f;
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(w, h[t][s], d, 0, 0, 0);
      }
    if (g == 0 && vis) {  // row group 0 holds outputs 0..3 of view c
      float out[3];
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        out[o] = 1.0f / (1.0f + expf(-(d[o] + Wp[off + 3 * WIDTH + o])));
        if (IN == 14) out[o] += a.colors[3 * p + o];  // relighting: c_dc + network
      }
      float* rec = a.records + ((int64_t)v * a.P + p) * kRecFloats;
      rec[11] = out[0];
      rec[15] = out[1];
      rec[19] = out[2];
    }
  }
}

// Backward of the colour MLP, one wave per primitive, 16 of its views at a
// time, every product on the matrix cores in the tile layout of the forward
// (lane (g, c) = (lane / 16, lane % 16) holds units 16 t + 4 g + r of view c
// in register r; rows_to_regs makes that the B operand of the next product).
// The forward is recomputed; the deltas run back through the transposed
// weights (operand A = W^T, the lanes along the rows of W: 64-byte runs);
// the input gradient is one more such product.  The weights are read from
// global memory (L1 and L2 after the first touch): an LDS copy would cost
// more workgroups per CU than it saves.  Activations, deltas and inputs also
// go to LDS as [view][unit], the operands of the weight gradients: products
// over the views, each entry added to HBM by its one owning lane (no
// atomics).  Views culled for the primitive carry zero deltas.
template <int WIDTH, int DEPTH, int IN>
__global__ void __launch_bounds__(64) cmlp_bwd_kernel(CmlpArgs a) {
  constexpr int K = CmlpShape<WIDTH, DEPTH, IN>::K;
  constexpr int XI0 = IN - kXiDim;  // first xi input
  constexpr int VC = 16;            // views per chunk
  constexpr int T = WIDTH / 16;     // tiles of 16 units
  constexpr int S0 = (IN + 3) / 4;  // steps of four inputs in the first layer
  constexpr int LAST = IN * WIDTH + WIDTH + (DEPTH - 1) * (WIDTH * WIDTH + WIDTH);  // output layer offset
  __shared__ float sX[VC][IN + 1];
  __shared__ float sH[DEPTH][VC][WIDTH + 1];  // post-ReLU activations
  __shared__ float sD[DEPTH][VC][WIDTH + 1];  // deltas of the hidden pre-activations
  __shared__ float sDo[VC][4];                // deltas of the output pre-activations
  __shared__ float sGx[VC][IN + 1];           // d loss / d input
  const int64_t p = blockIdx.x;
  const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
  const float* Wg = a.cmlp + p * K;
  float xi_acc = 0.f;  // lanes 0..7: sum over views of d loss / d xi[lane]
  float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f;  // relighting: d loss / d x_B through the light direction
  for (int v0 = 0; v0 < a.V; v0 += VC) {
    const int v = v0 + c;
    const int64_t i = (int64_t)(v < a.V ? v : v0) * a.P + p;
    const bool act = v < a.V && a.tile_counts[i] != 0;
    // ---- inputs (every lane of view c computes them; row 0 stores them)
    float x[IN], dir[3], il = 0.f;
#pragma unroll
    for (int k = 0; k < IN; ++k) x[k] = 0.f;
    if (act) cmlp_input<IN>(a, p, v, x, dir, &il);
    if (g == 0) {
#pragma unroll
      for (int k = 0; k < IN; ++k) sX[c][k] = x[k];
    }
    float bx[S0];
#pragma unroll
    for (int s = 0; s < S0; ++s) {
      float t = 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (4 * s + q < IN) t = g == q ? x[4 * s + q] : t;
      bx[s] = t;
    }
    // ---- forward: activations in the tile layout, their transposes as the
    // next operands, and a [view][unit] copy in LDS
    v4f hb[T];  // B operands of the next layer
#pragma unroll
    for (int t = 0; t < T; ++t) {
      v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < S0; ++s) {
        const int k = 4 * s + g;
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(k < IN ? Wg[(16 * t + c) * IN + k] : 0.f, bx[s], d, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        d[r] = fmaxf(d[r] + Wg[IN * WIDTH + 16 * t + 4 * g + r], 0.f);
        sH[0][c][16 * t + 4 * g + r] = d[r];
      }
      hb[t] = rows_to_regs(d);
    }
#pragma unroll
    for (int l = 1; l < DEPTH; ++l) {
      const int off = IN * WIDTH + WIDTH + (l - 1) * (WIDTH * WIDTH + WIDTH);
      v4f nb[T];
#pragma unroll
      for (int to = 0; to < T; ++to) {
        v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int s = 0; s < 4; ++s)
            d = __builtin_amdgcn_mfma_f32_16x16x4f32(Wg[off + (16 * to + c) * WIDTH + 16 * t + 4 * s + g], hb[t][s], d,
                                                     0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          d[r] = fmaxf(d[r] + Wg[off + WIDTH * WIDTH + 16 * to + 4 * g + r], 0.f);
          sH[l][c][16 * to + 4 * g + r] = d[r];
        }
        nb[to] = rows_to_regs(d);
      }
#pragma unroll
      for (int t = 0; t < T; ++t) hb[t] = nb[t];
    }
    // ---- output: sigmoid and d loss / d pre-sigmoid (row group 0 holds
    // outputs 0..3 of view c)
    v4f dout;
    {
      v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s)
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(c < 3 ? Wg[LAST + c * WIDTH + 16 * t + 4 * s + g] : 0.f, hb[t][s],
                                                   d, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float dv = 0.f;
        if (g == 0 && r < 3 && act) {
          const float sg = 1.0f / (1.0f + expf(-(d[r] + Wg[LAST + 3 * WIDTH + r])));
          dv = a.gview[i * kGViewFloats + 18 + r] * sg * (1.0f - sg);
        }
        dout[r] = dv;
        if (g == 0) sDo[c][r] = dv;
      }
    }
    // ---- deltas: last hidden layer from the output, then down the layers;
    // operand B = the layer above's deltas, transposed
    v4f db[T];  // transposed deltas of the layer above
    {
      const v4f ob = rows_to_regs(dout);  // lane (g, c) register 0: output g of view c
#pragma unroll
      for (int t = 0; t < T; ++t) {
        v4f d = {0.f, 0.f, 0.f, 0.f};
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(g < 3 ? Wg[LAST + g * WIDTH + 16 * t + c] : 0.f, ob[0], d, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int u = 16 * t + 4 * g + r;
          d[r] = sH[DEPTH - 1][c][u] > 0.f ? d[r] : 0.f;
          sD[DEPTH - 1][c][u] = d[r];
        }
        db[t] = rows_to_regs(d);
      }
    }
#pragma unroll
    for (int l = DEPTH - 1; l >= 1; --l) {
      const int off = IN * WIDTH + WIDTH + (l - 1) * (WIDTH * WIDTH + WIDTH);
      v4f nb[T];
#pragma unroll
      for (int t = 0; t < T; ++t) {  // units of layer l - 1
        v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int to = 0; to < T; ++to)  // units of layer l
#pragma unroll
          for (int s = 0; s < 4; ++s)
            d = __builtin_amdgcn_mfma_f32_16x16x4f32(Wg[off + (16 * to + 4 * s + g) * WIDTH + 16 * t + c], db[to][s], d,
                                                     0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int u = 16 * t + 4 * g + r;
          d[r] = sH[l - 1][c][u] > 0.f ? d[r] : 0.f;
          sD[l - 1][c][u] = d[r];
        }
        nb[t] = rows_to_regs(d);
      }
#pragma unroll
      for (int t = 0; t < T; ++t) db[t] = nb[t];
    }
    // ---- d loss / d input: rows = inputs (one tile), K = the first layer's units
    {
      v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int to = 0; to < T; ++to)
#pragma unroll
        for (int s = 0; s < 4; ++s)
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(c < IN ? Wg[(16 * to + 4 * s + g) * IN + c] : 0.f, db[to][s], d, 0,
                                                   0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (4 * g + r < IN) sGx[c][4 * g + r] = d[r];
    }
    __syncthreads();
    if (g == 0 && act) {  // direction gradient for the chain to the centre
      float* gv = a.gview + i * kGViewFloats;
      gv[21] = sGx[c][0];
      gv[22] = sGx[c][1];
      gv[23] = sGx[c][2];
      if constexpr (IN == 14) {
        // ld = normalize(l - x_B): d loss / d x_B = -(g - ld (ld . g)) / |l - x_B|
        float ld[3], il2;
        light_dir(a, p, a.cams[v], ld, &il2);
        const float g0 = sGx[c][3], g1 = sGx[c][4], g2 = sGx[c][5];
        const float dd = ld[0] * g0 + ld[1] * g1 + ld[2] * g2;
        gc0 -= (g0 - ld[0] * dd) * il2;
        gc1 -= (g1 - ld[1] * dd) * il2;
        gc2 -= (g2 - ld[2] * dd) * il2;
      }
    }
    if (lane < kXiDim) {
#pragma unroll
      for (int w = 0; w < VC; ++w) xi_acc += sGx[w][XI0 + lane];
    }
    // ---- weight gradients: sum over the chunk's 16 views of delta[o] x a[k]
    // on the matrix cores (K = views, four per step): lane (g, c) supplies
    // delta[view 4 s + g][unit 16 t + c] (A) and a[view 4 s + g][input
    // 16 t2 + c] (B) from LDS and receives the gradient of weight (16 t +
    // 4 g + r, 16 t2 + c) in register r, added to its entry in HBM (each
    // entry has one owner).  The biases, sums of the deltas alone, are
    // summed by one lane per unit.
    float* G = a.g_cmlp ? a.g_cmlp + p * K : nullptr;
    if (G) {
      // the lane index through an empty asm, so that the compiler does not
      // hoist this section's addresses out of the view loop and keep them
      // live through the passes above
      int ln = lane;
      asm volatile("" : "+v"(ln));
      const int gw = ln >> 4, cw = ln & 15;
      // Per layer, the gradient entries are loaded first (all tiles at once,
      // so that their latencies overlap), then the products are added.
      // First layer: inputs as columns cw < IN of one tile.
      {
        float old[WIDTH / 16][4];
#pragma unroll
        for (int t = 0; t < WIDTH / 16; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) old[t][r] = cw < IN ? G[(16 * t + 4 * gw + r) * IN + cw] : 0.f;
#pragma unroll
        for (int t = 0; t < WIDTH / 16; ++t) {
          v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < 4; ++s)
            d = __builtin_amdgcn_mfma_f32_16x16x4f32(sD[0][4 * s + gw][16 * t + cw], cw < IN ? sX[4 * s + gw][cw] : 0.f,
                                                     d, 0, 0, 0);
          if (cw < IN) {
#pragma unroll
            for (int r = 0; r < 4; ++r) G[(16 * t + 4 * gw + r) * IN + cw] = old[t][r] + d[r];
          }
        }
      }
#pragma unroll
      for (int l = 1; l < DEPTH; ++l) {
        const int off = IN * WIDTH + WIDTH + (l - 1) * (WIDTH * WIDTH + WIDTH);
        float old[WIDTH / 16][WIDTH / 16][4];
#pragma unroll
        for (int t = 0; t < WIDTH / 16; ++t)
#pragma unroll
          for (int t2 = 0; t2 < WIDTH / 16; ++t2)
#pragma unroll
            for (int r = 0; r < 4; ++r) old[t][t2][r] = G[off + (16 * t + 4 * gw + r) * WIDTH + 16 * t2 + cw];
#pragma unroll
        for (int t = 0; t < WIDTH / 16; ++t)
#pragma unroll
          for (int t2 = 0; t2 < WIDTH / 16; ++t2) {
            v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 4; ++s)
              d = __builtin_amdgcn_mfma_f32_16x16x4f32(sD[l][4 * s + gw][16 * t + cw], sH[l - 1][4 * s + gw][16 * t2 + cw],
                                                       d, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) G[off + (16 * t + 4 * gw + r) * WIDTH + 16 * t2 + cw] = old[t][t2][r] + d[r];
          }
      }
      // output layer: rows 0..2 of one tile
      {
        float old[WIDTH / 16][3];
#pragma unroll
        for (int t2 = 0; t2 < WIDTH / 16; ++t2)
#pragma unroll
          for (int r = 0; r < 3; ++r) old[t2][r] = gw == 0 ? G[LAST + r * WIDTH + 16 * t2 + cw] : 0.f;
#pragma unroll
        for (int t2 = 0; t2 < WIDTH / 16; ++t2) {
          v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < 4; ++s)
            d = __builtin_amdgcn_mfma_f32_16x16x4f32(cw < 3 ? sDo[4 * s + gw][cw] : 0.f,
                                                     sH[DEPTH - 1][4 * s + gw][16 * t2 + cw], d, 0, 0, 0);
          if (gw == 0) {
#pragma unroll
            for (int r = 0; r < 3; ++r) G[LAST + r * WIDTH + 16 * t2 + cw] = old[t2][r] + d[r];
          }
        }
      }
      // biases
      if (lane < WIDTH) {
#pragma unroll 1
        for (int l = 0; l < DEPTH; ++l) {
          const int boff = l == 0 ? IN * WIDTH : IN * WIDTH + WIDTH + (l - 1) * (WIDTH * WIDTH + WIDTH) + WIDTH * WIDTH;
          float sum = 0.f;
#pragma unroll
          for (int w = 0; w < VC; ++w) sum += sD[l][w][lane];
          G[boff + lane] += sum;
        }
      } else if (lane < WIDTH + 3) {
        const int o = lane - WIDTH;
        float sum = 0.f;
#pragma unroll
        for (int w = 0; w < VC; ++w) sum += sDo[w][o];
        G[LAST + 3 * WIDTH + o] += sum;
      }
    }
    __syncthreads();
  }
  if (a.g_xi && lane < kXiDim) a.g_xi[p * kXiDim + lane] += xi_acc;
  if (IN == 14 && a.g_centers) {
    // the light-direction terms of the 16 view lanes (lanes 0..15, q = 0)
    gc0 += __shfl_xor(gc0, 1); gc1 += __shfl_xor(gc1, 1); gc2 += __shfl_xor(gc2, 1);
    gc0 += __shfl_xor(gc0, 2); gc1 += __shfl_xor(gc1, 2); gc2 += __shfl_xor(gc2, 2);
    gc0 += __shfl_xor(gc0, 4); gc1 += __shfl_xor(gc1, 4); gc2 += __shfl_xor(gc2, 4);
    gc0 += __shfl_xor(gc0, 8); gc1 += __shfl_xor(gc1, 8); gc2 += __shfl_xor(gc2, 8);
    if (lane == 0) {
      a.g_centers[3 * p] += gc0;
      a.g_centers[3 * p + 1] += gc1;
      a.g_centers[3 * p + 2] += gc2;
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint of the preprocessing: per primitive, summed over the views
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) preprocess_bwd_kernel(PreBwdArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.P) return;
  const int N = a.N;
  double Rp[3][3], qh[4], qnorm;
  quat_rot_f64(a.quats + 4 * p, Rp, qh, &qnorm);
  const double xb[3] = {a.centers[3 * p], a.centers[3 * p + 1], a.centers[3 * p + 2]};
  const double s[3] = {a.scales[3 * p], a.scales[3 * p + 1], a.scales[3 * p + 2]};
  double U[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) U[r][c] = Rp[c][r] / s[r];

  double gU[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double gxb[3] = {0, 0, 0};
  double gcol[3] = {0, 0, 0};
  auto cross = [](const double* u, const double* w, double* out) {
    out[0] = u[1] * w[2] - u[2] * w[1];
    out[1] = u[2] * w[0] - u[0] * w[2];
    out[2] = u[0] * w[1] - u[1] * w[0];
  };
  for (int v = 0; v < a.V; ++v) {
    const int64_t i = (int64_t)v * a.P + p;
    if (a.tile_counts[i] == 0) continue;
    const CamDev& cam = a.cams[v];
    const float* rec = a.records + i * kRecFloats;
    const float* gv = a.gview + i * kGViewFloats;
    const double rx = rec[3], ry = rec[7];
    double om[3] = {cam.o[0] - xb[0], cam.o[1] - xb[1], cam.o[2] - xb[2]};
    double op[3], G[3][3];
    for (int r = 0; r < 3; ++r) {
      op[r] = U[r][0] * om[0] + U[r][1] * om[1] + U[r][2] * om[2];
      for (int c = 0; c < 3; ++c)
        G[r][c] = U[r][0] * cam.Rinv[c] + U[r][1] * cam.Rinv[3 + c] + U[r][2] * cam.Rinv[6 + c];
    }
    const double vr[3] = {(rx - cam.cx) / cam.fx, (ry - cam.cy) / cam.fy, 1.0};
    double dc[3], gx[3], gy[3];
    for (int r = 0; r < 3; ++r) {
      dc[r] = G[r][0] * vr[0] + G[r][1] * vr[1] + G[r][2] * vr[2];
      gx[r] = G[r][0] / cam.fx;
      gy[r] = G[r][1] / cam.fy;
    }
    double g_dc[3] = {gv[0], gv[1], gv[2]}, g_gx[3] = {gv[3], gv[4], gv[5]}, g_gy[3] = {gv[6], gv[7], gv[8]};
    const double g_mc[3] = {gv[9], gv[10], gv[11]}, g_hx[3] = {gv[12], gv[13], gv[14]},
                 g_hy[3] = {gv[15], gv[16], gv[17]};
    // m = o' x b  ->  g_o' += b x g_m,  g_b += g_m x o'
    double g_op[3] = {0, 0, 0}, t3[3];
    cross(dc, g_mc, t3);
    for (int r = 0; r < 3; ++r) g_op[r] += t3[r];
    cross(gx, g_hx, t3);
    for (int r = 0; r < 3; ++r) g_op[r] += t3[r];
    cross(gy, g_hy, t3);
    for (int r = 0; r < 3; ++r) g_op[r] += t3[r];
    cross(g_mc, op, t3);
    for (int r = 0; r < 3; ++r) g_dc[r] += t3[r];
    cross(g_hx, op, t3);
    for (int r = 0; r < 3; ++r) g_gx[r] += t3[r];
    cross(g_hy, op, t3);
    for (int r = 0; r < 3; ++r) g_gy[r] += t3[r];
    // G: dc = G vr, gx = G e0 / fx, gy = G e1 / fy
    double gG[3][3];
    for (int r = 0; r < 3; ++r) {
      gG[r][0] = g_dc[r] * vr[0] + g_gx[r] / cam.fx;
      gG[r][1] = g_dc[r] * vr[1] + g_gy[r] / cam.fy;
      gG[r][2] = g_dc[r] * vr[2];
    }
    // G = U Rinv, o' = U (o - x_B)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        gU[r][c] += gG[r][0] * cam.Rinv[3 * c] + gG[r][1] * cam.Rinv[3 * c + 1] + gG[r][2] * cam.Rinv[3 * c + 2];
        gU[r][c] += g_op[r] * om[c];
      }
    for (int c = 0; c < 3; ++c) gxb[c] -= U[0][c] * g_op[0] + U[1][c] * g_op[1] + U[2][c] * g_op[2];
    // colour (the constant colour, or the relighting colour's c_dc)
    if (a.color_mode == 0 || a.color_mode == 3 || a.color_mode == 4) {
      gcol[0] += gv[18];
      gcol[1] += gv[19];
      gcol[2] += gv[20];
    }
    if (a.color_mode >= 1 && a.color_mode <= 3) {
      // dir = normalize(x_B - o): d dir / d x_B = (I - dir dir^T) / |x_B - o|
      const double dvec[3] = {-om[0], -om[1], -om[2]};
      const double len = sqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2]);
      const double dir[3] = {dvec[0] / len, dvec[1] / len, dvec[2] / len};
      const double gd[3] = {gv[21], gv[22], gv[23]};
      const double dd = dir[0] * gd[0] + dir[1] * gd[1] + dir[2] * gd[2];
      for (int c = 0; c < 3; ++c) gxb[c] += (gd[c] - dir[c] * dd) / len;
    }
  }
  // U[r][c] = Rp[c][r] / s[r]; plus the per-ray colour network's own
  // rotation and scale gradients
  double gR[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double gs[3] = {0, 0, 0};
  if (a.extra_rs) {
    const float* ex = a.extra_rs + p * 12;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) gR[r][c] = ex[3 * r + c];
    for (int c = 0; c < 3; ++c) gs[c] = ex[9 + c];
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      gR[c][r] += gU[r][c] / s[r];
      gs[r] -= gU[r][c] * Rp[c][r] / (s[r] * s[r]);
    }
  // table: Wt_k[j] = K sum_i W1_k[i] Rp[i][j] s_j,  K = omega0 / (2 pi m)
  const double m = fmax(s[0], fmax(s[1], s[2]));
  const int am = (s[0] >= s[1] && s[0] >= s[2]) ? 0 : (s[1] >= s[2] ? 1 : 2);
  const double twopi = 6.283185307179586476925;
  const double K = (double)a.omega0 / (twopi * m);
  const int TS = table_stride(N);
  const float* gt = a.gtable + p * TS;
  double gK = 0.0;
  for (int k = 0; k < N; ++k) {
    const float* wk = a.w1 + (p * N + k) * 3;
    const double gwt[3] = {gt[4 * k], gt[4 * k + 1], gt[4 * k + 2]};
    double wt[3];
    for (int j = 0; j < 3; ++j) wt[j] = K * ((wk[0] * Rp[0][j] + wk[1] * Rp[1][j] + wk[2] * Rp[2][j]) * s[j]);
    for (int j = 0; j < 3; ++j) gK += gwt[j] * wt[j] / K;
    if (a.g.w1) {
      for (int ii = 0; ii < 3; ++ii) {
        double acc = 0.0;
        for (int j = 0; j < 3; ++j) acc += gwt[j] * Rp[ii][j] * s[j];
        a.g.w1[(p * N + k) * 3 + ii] += (float)(K * acc);
      }
    }
    for (int ii = 0; ii < 3; ++ii)
      for (int j = 0; j < 3; ++j) {
        gR[ii][j] += K * gwt[j] * wk[ii] * s[j];
        gs[j] += K * gwt[j] * wk[ii] * Rp[ii][j];
      }
    if (a.g.b1) a.g.b1[p * N + k] += (float)((double)gt[4 * k + 3] * a.omega0 / twopi);
    if (a.g.wt) a.g.wt[p * N + k] += (float)((double)gt[4 * k + 3] * a.time / twopi);
    if (a.g.w2) a.g.w2[p * N + k] += (float)((double)gt[4 * N + k] / twopi);
  }
  if (a.g.b2) a.g.b2[p] += gt[5 * N];
  gs[am] += gK * (-K / m);
  // rotation -> normalised quaternion -> raw quaternion
  const double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
  double gq[4];
  gq[0] = 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
  gq[1] = 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.0 * x * gR[1][1] - w * gR[1][2] + z * gR[2][0] +
                 w * gR[2][1] - 2.0 * x * gR[2][2]);
  gq[2] = 2.0 * (-2.0 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] - w * gR[2][0] +
                 z * gR[2][1] - 2.0 * y * gR[2][2]);
  gq[3] = 2.0 * (-2.0 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2.0 * z * gR[1][1] +
                 y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
  const double dq = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;
  if (a.g.quats)
    for (int k = 0; k < 4; ++k) a.g.quats[4 * p + k] += (float)((gq[k] - qh[k] * dq) / qnorm);
  if (a.g.scales)
    for (int k = 0; k < 3; ++k) a.g.scales[3 * p + k] += (float)gs[k];
  if (a.g.centers)
    for (int k = 0; k < 3; ++k) a.g.centers[3 * p + k] += (float)gxb[k];
  if ((a.color_mode == 0 || a.color_mode == 3 || a.color_mode == 4) && a.g.colors)
    for (int k = 0; k < 3; ++k) a.g.colors[3 * p + k] += (float)gcol[k];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_setup_cams(const CamChunk& ch, CamDev* out, hipStream_t st) {
  hipLaunchKernelGGL(setup_cams_kernel, dim3(1), dim3(kMaxCamsPerChunk), 0, st, ch, out);
  return hipGetLastError();
}

hipError_t launch_prim_table(int N, int64_t P, float omega0, float time, const snp_prims& pr, float* table,
                             unsigned long long* counters, hipStream_t st) {
  const dim3 grid((unsigned)((P + 255) / 256)), block(256);
  switch (N) {
    case 4: hipLaunchKernelGGL(prim_table_kernel<4>, grid, block, 0, st, P, omega0, pr.scales, pr.quats, pr.w1, pr.b1, pr.w2, pr.b2, pr.wt, time, table, counters); break;
    case 8: hipLaunchKernelGGL(prim_table_kernel<8>, grid, block, 0, st, P, omega0, pr.scales, pr.quats, pr.w1, pr.b1, pr.w2, pr.b2, pr.wt, time, table, counters); break;
    case 16: hipLaunchKernelGGL(prim_table_kernel<16>, grid, block, 0, st, P, omega0, pr.scales, pr.quats, pr.w1, pr.b1, pr.w2, pr.b2, pr.wt, time, table, counters); break;
    case 32: hipLaunchKernelGGL(prim_table_kernel<32>, grid, block, 0, st, P, omega0, pr.scales, pr.quats, pr.w1, pr.b1, pr.w2, pr.b2, pr.wt, time, table, counters); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_preprocess_views(const ViewArgs& a, hipStream_t st) {
  const int64_t n = a.P * a.V;
  hipLaunchKernelGGL(preprocess_views_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

#define SNP_CMLP_DISPATCH_IN(KERNEL, IN, width, depth, grid, block, st, a)                                \
  do {                                                                                                     \
    if (width == 16 && depth == 1) hipLaunchKernelGGL((KERNEL<16, 1, IN>), grid, block, 0, st, a);         \
    else if (width == 16 && depth == 2) hipLaunchKernelGGL((KERNEL<16, 2, IN>), grid, block, 0, st, a);    \
    else if (width == 16 && depth == 3) hipLaunchKernelGGL((KERNEL<16, 3, IN>), grid, block, 0, st, a);    \
    else if (width == 32 && depth == 1) hipLaunchKernelGGL((KERNEL<32, 1, IN>), grid, block, 0, st, a);    \
    else if (width == 32 && depth == 2) hipLaunchKernelGGL((KERNEL<32, 2, IN>), grid, block, 0, st, a);    \
    else if (width == 32 && depth == 3) hipLaunchKernelGGL((KERNEL<32, 3, IN>), grid, block, 0, st, a);    \
    else return hipErrorInvalidValue;                                                                      \
  } while (0)
#define SNP_CMLP_DISPATCH(KERNEL, width, depth, grid, block, st, a)                 \
  do {                                                                               \
    if (a.relight) SNP_CMLP_DISPATCH_IN(KERNEL, 14, width, depth, grid, block, st, a); \
    else SNP_CMLP_DISPATCH_IN(KERNEL, 11, width, depth, grid, block, st, a);           \
  } while (0)

hipError_t launch_cmlp_fwd(int width, int depth, CmlpArgs a, hipStream_t st) {
  if (a.P <= 0) return hipSuccess;
  const dim3 grid((unsigned)((a.P + 3) / 4)), block(256);
  SNP_CMLP_DISPATCH(cmlp_fwd_mfma_kernel, width, depth, grid, block, st, a);
  return hipGetLastError();
}

hipError_t launch_cmlp_bwd(int width, int depth, CmlpArgs a, hipStream_t st) {
  if (a.P <= 0) return hipSuccess;
  const dim3 grid((unsigned)a.P), block(64);
  SNP_CMLP_DISPATCH(cmlp_bwd_kernel, width, depth, grid, block, st, a);
  return hipGetLastError();
}

bool cmlp_supported(int width, int depth) {
  return (width == 16 || width == 32) && depth >= 1 && depth <= 3;
}

int cmlp_param_count(int width, int depth, bool relight) {
  const int in = kCmlpIn + (relight ? 3 : 0);
  return in * width + width + (depth - 1) * (width * width + width) + width * 3 + 3;
}

hipError_t launch_preprocess_bwd(const PreBwdArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(preprocess_bwd_kernel, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace snp
