// Binary32 tile-membership specification, device side.
//
// Membership decides which Gaussians a pixel sums over (Sec. 4.2, additive
// rasterisation over N(p)) and which (Gaussian, slice) pairs survive the axial
// cull (Sec. 4.2, opacity modulation: "cull primitives with opacity below a
// small threshold").  It is defined as a fixed sequence of correctly rounded
// binary32 operations with no fused multiply-add, so that any IEEE-754 machine
// reproduces it bit for bit.  Every function here compiles with floating-point
// contraction off; the library is built with correctly rounded division and
// square root and with denormals preserved.
//
//   s_j   = exp_spec(l_j) * mod                       (S = diag(mod * s))
//   q^    = q / sqrt(((qw^2 + qx^2) + qy^2) + qz^2)
//   R     = quatToMatrix(q^)
//           (both from the supplement, "Derivation of Forward rendering process")
//   Sigma = R diag(s^2) R^T, adj = R diag(P) R^T with P = (s1^2 s2^2, s0^2 s2^2, s0^2 s1^2)
//           (entries summed left to right)
//   m = mu_z - z, D = sigma_z^2 + Sigma_zz, q_ax = m^2 / D        axial test q_ax <= q_cut
//   w = 1 / (1 + Sigma_zz / sigma_z^2), 1/D
//   A = w Sigma_xx + adj_11 / D,  C = w Sigma_yy + adj_00 / D     (= Sigma_2d diagonal)
//   mu_2d = (mu_x - (Sigma_xz / D) m, mu_y - (Sigma_yz / D) m)
//   footprint = k-sigma box of Sigma_2d in 16x16 tiles of the slice grid, clamped
//
// q_ax equals the change in Mahalanobis distance of the opacity-modulation
// equation; A, C and mu_2d equal the Focus Gaussian's marginal (Sec. 4.2) by
// the Sherman-Morrison identity, written through the adjugate so that no
// catastrophic cancellation occurs.  exp_spec is Cody-Waite range reduction
// (C1 = 355/512) and the degree-7 Taylor polynomial of e^r by Horner's rule.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gp {

struct SpecCov {
  float s0, s1, s2;              // activated scales
  float w, x, y, z;              // normalised quaternion
  float R[3][3];
  float sxx, sxy, sxz, syy, syz, szz;
  float a00, a01, a11, a22, detS;
  float n2;
};

__device__ __forceinline__ float exp_spec(float x) {
#pragma clang fp contract(off)
  x = fminf(fmaxf(x, -87.0f), 88.0f);
  const float k = rintf(x * 1.4426950408889634f);
  const float r = (x - k * 0.693359375f) - k * -2.12194440054690583e-4f;
  float p = (float)(1.0 / 5040.0);
  p = p * r + (float)(1.0 / 720.0);
  p = p * r + (float)(1.0 / 120.0);
  p = p * r + (float)(1.0 / 24.0);
  p = p * r + (float)(1.0 / 6.0);
  p = p * r + 0.5f;
  p = p * r + 1.0f;
  p = p * r + 1.0f;
  const int ki = (int)k;
  return p * __int_as_float((ki + 127) << 23);
}

__device__ __forceinline__ float quad3(const float (&R)[3][3], int a, int b, float w0, float w1,
                                       float w2) {
#pragma clang fp contract(off)
  return ((R[a][0] * R[b][0]) * w0 + (R[a][1] * R[b][1]) * w1) + (R[a][2] * R[b][2]) * w2;
}

__device__ __forceinline__ void spec_forms(SpecCov& c);

__device__ __forceinline__ void spec_cov(float l0, float l1, float l2, float qw, float qx, float qy,
                                         float qz, float mod, SpecCov& c) {
#pragma clang fp contract(off)
  c.s0 = exp_spec(l0) * mod;
  c.s1 = exp_spec(l1) * mod;
  c.s2 = exp_spec(l2) * mod;
  c.n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  const float rn = sqrtf(c.n2);
  const float w = qw / rn, x = qx / rn, y = qy / rn, z = qz / rn;
  c.w = w; c.x = x; c.y = y; c.z = z;
  const float xx = x * x, yy = y * y, zz = z * z;
  const float xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  c.R[0][0] = 1.0f - 2.0f * (yy + zz);
  c.R[0][1] = 2.0f * (xy - wz);
  c.R[0][2] = 2.0f * (xz + wy);
  c.R[1][0] = 2.0f * (xy + wz);
  c.R[1][1] = 1.0f - 2.0f * (xx + zz);
  c.R[1][2] = 2.0f * (yz - wx);
  c.R[2][0] = 2.0f * (xz - wy);
  c.R[2][1] = 2.0f * (yz + wx);
  c.R[2][2] = 1.0f - 2.0f * (xx + yy);
  spec_forms(c);
}

// Covariance R diag(v) R^T and adjugate entries R diag(v1 v2, v0 v2, v0 v1) R^T
// of c.R and c's scales (v_i = s_i^2).
__device__ __forceinline__ void spec_forms(SpecCov& c) {
#pragma clang fp contract(off)
  const float v0 = c.s0 * c.s0, v1 = c.s1 * c.s1, v2 = c.s2 * c.s2;
  const float P0 = v1 * v2, P1 = v0 * v2, P2 = v0 * v1;
  c.sxx = quad3(c.R, 0, 0, v0, v1, v2);
  c.sxy = quad3(c.R, 0, 1, v0, v1, v2);
  c.sxz = quad3(c.R, 0, 2, v0, v1, v2);
  c.syy = quad3(c.R, 1, 1, v0, v1, v2);
  c.syz = quad3(c.R, 1, 2, v0, v1, v2);
  c.szz = quad3(c.R, 2, 2, v0, v1, v2);
  c.a00 = quad3(c.R, 0, 0, P0, P1, P2);
  c.a01 = quad3(c.R, 0, 1, P0, P1, P2);
  c.a11 = quad3(c.R, 1, 1, P0, P1, P2);
  c.a22 = quad3(c.R, 2, 2, P0, P1, P2);
  c.detS = (v0 * v1) * v2;
}

// The Gaussian seen from a posed slice's camera frame (supplement, forward
// derivation: mu_c = R_c mu + t, Sigma_c = R_c Sigma R_c^T), pose = R_c
// row-major then t: the rotation becomes R_c R (entry by entry, left to
// right), covariance and adjugate follow from it as in spec_cov, and the mean
// is ((R_c[i][0] mu_x + R_c[i][1] mu_y) + R_c[i][2] mu_z) + t[i].  The identity
// pose reproduces c and mu bit for bit.
__device__ __forceinline__ void spec_pose(const SpecCov& c, const float* mu, const float* pose, SpecCov& o,
                                          float* mo) {
#pragma clang fp contract(off)
  o = c;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j)
      o.R[i][j] = (pose[3 * i] * c.R[0][j] + pose[3 * i + 1] * c.R[1][j]) + pose[3 * i + 2] * c.R[2][j];
    mo[i] = ((pose[3 * i] * mu[0] + pose[3 * i + 1] * mu[1]) + pose[3 * i + 2] * mu[2]) + pose[9 + i];
  }
  spec_forms(o);
}

// Axial quantities of one (Gaussian, slice) pair.
struct SpecAxial {
  float m, s2, D, q;
};

__device__ __forceinline__ SpecAxial spec_axial(float muz, float szz, float z, float sigma_z) {
#pragma clang fp contract(off)
  SpecAxial a;
  a.m = muz - z;
  a.s2 = sigma_z * sigma_z;
  a.D = a.s2 + szz;
  a.q = (a.m * a.m) / a.D;
  return a;
}

// Footprint of one (Gaussian, slice) pair in tiles; returns false if it lies
// outside the grid.  Also returns the quantities shared with the image path.
struct SpecRect {
  float invD, w, A, C, u, v, mx, my;
  int tx0, tx1, ty0, ty1;
};

// The part of the footprint that depends on the slice only through sigma_z
// (through s2 and D): equal for every slice of one sigma_z, so a loop over
// slices may reuse it (the same operations on the same operands).
struct SpecSigma {
  float invD, w, A, C, u, v, rx, ry;
};
__device__ __forceinline__ SpecSigma spec_sigma(const SpecCov& c, const SpecAxial& ax, float bbox) {
#pragma clang fp contract(off)
  SpecSigma g;
  g.invD = 1.0f / ax.D;
  g.w = 1.0f / (1.0f + c.szz / ax.s2);
  g.A = g.w * c.sxx + c.a11 * g.invD;
  g.C = g.w * c.syy + c.a00 * g.invD;
  g.u = c.sxz * g.invD;
  g.v = c.syz * g.invD;
  g.rx = bbox * sqrtf(g.A);
  g.ry = bbox * sqrtf(g.C);
  return g;
}
__device__ __forceinline__ bool spec_rect_from(const SpecSigma& g, float mux, float muy, const SpecAxial& ax,
                                               float x0, float y0, float dx, float dy, int ntx, int nty,
                                               SpecRect& r) {
#pragma clang fp contract(off)
  r.invD = g.invD;
  r.w = g.w;
  r.A = g.A;
  r.C = g.C;
  r.u = g.u;
  r.v = g.v;
  r.mx = mux - r.u * ax.m;
  r.my = muy - r.v * ax.m;
  const float xl = floorf((((r.mx - g.rx) - x0) / dx) * 0.0625f);
  const float xh = floorf((((r.mx + g.rx) - x0) / dx) * 0.0625f);
  const float yl = floorf((((r.my - g.ry) - y0) / dy) * 0.0625f);
  const float yh = floorf((((r.my + g.ry) - y0) / dy) * 0.0625f);
  const float fx = (float)(ntx - 1), fy = (float)(nty - 1);
  const bool vis = (xh >= 0.0f) && (xl <= fx) && (yh >= 0.0f) && (yl <= fy);
  if (!vis) return false;
  r.tx0 = (int)fmaxf(xl, 0.0f);
  r.tx1 = (int)fminf(xh, fx);
  r.ty0 = (int)fmaxf(yl, 0.0f);
  r.ty1 = (int)fminf(yh, fy);
  return true;
}
__device__ __forceinline__ bool spec_rect(const SpecCov& c, float mux, float muy, const SpecAxial& ax,
                                          float x0, float y0, float dx, float dy, int ntx, int nty,
                                          float bbox, SpecRect& r) {
  return spec_rect_from(spec_sigma(c, ax, bbox), mux, muy, ax, x0, y0, dx, dy, ntx, nty, r);
}

}  // namespace gp
