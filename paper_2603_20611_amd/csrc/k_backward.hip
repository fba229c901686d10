// Backward of the preprocess (Sec. 4.3 "Backward pass": screen-space
// projection -> Focus Gaussian (mu_e, Sigma_e) -> camera space -> world
// parameters (mu, s, q, alpha), with the determinant coupling of alpha~;
// supplement, "Derivation of Differentiable Backward Pass").  The chain
// implemented is the exact derivative of the forward as computed, through the
// closed form of the Focus Gaussian:
//
//   D = sigma_z^2 + Sigma_zz, u = Sigma_xz / D, v = Sigma_yz / D, m = mu_z - z
//   A = Sigma_xx - u Sigma_xz, B = Sigma_xy - u Sigma_yz, C = Sigma_yy - v Sigma_yz
//   mu_2d = (mu_x - u m, mu_y - v m), q_ax = m^2 / D, opacity_r = exp(-q_ax / 2)
//   alpha~ = alpha opacity_r / sqrt(AC - B^2), conic = (C, -B, A) / (AC - B^2)
//
// L lanes per Gaussian (1, 2, 4 or 8: the most that still give every
// Gaussian of a workgroup's list its lanes in one round; a batch of a few
// slices leaves few Gaussians with records, and one lane's serial chain over
// up to eight of them had set the kernel's time): lane i of the group takes
// the Gaussian's records i, i + L, ... (one per slice it reaches), sums the
// six moments of each record's tiles in footprint order and applies the
// chain rule; the group adds its lanes' sums by a fixed butterfly, and its
// first lane maps Sigma = R diag(s^2) R^T back to (log-scale, quaternion).  The gradient is added to the caller's buffer
// with plain loads and stores: every element has exactly one writer, so the
// result is deterministic.
#include "gp_internal.h"
#include "gp_spec.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace gp {
namespace {


struct BwdPreArgs {
  RenderConst rc;
  const BatchHdr* hdr;
  const GroupDev* groups;
  const SliceDev* slices;
  const RecPay* rec_pay;
  const RecMeta* rec_meta;
  const uint32_t* g_rbase;
  const uint32_t* g_nrec;
  const float4* moments;
  float* grad;
  int64_t grad_stride;
  float* st_grad_norm;      // optional densification statistics
  int32_t* st_count;
  float* st_max_radius;
  int64_t st_n;
  const float* poses;       // [n_slices][12] of a posed batch
  int chunk;                // Gaussians per workgroup round (a multiple of 256, at most kBwdChunk)
};

// Every lane of a group of L calls this for the group's Gaussian t (active
// false: the group has none); the group's lanes exchange their sums.
template <int DT, bool POSED, int L>
__device__ __forceinline__ void backward_one(const BwdPreArgs& a, int n_groups, int t, bool active) {
  const uint32_t li = L > 1 ? (threadIdx.x & (uint32_t)(L - 1)) : 0u;
  bool go = active;
  uint32_t nrec = 0u, rbase = 0u;
  int j = 0;
  GroupDev G{};
  if (go) {
    nrec = a.g_nrec[t];
    G = a.groups[group_of(a.groups, n_groups, (t & ~63))];
    j = t - G.gbase;
    go = nrec > 0u && j < G.n;
  }
  float p[11];
#pragma unroll
  for (int r = 0; r < 11; ++r) p[r] = 0.0f;
  SpecCov c{};
  if (go) {
    rbase = a.g_rbase[t];
    p[0] = G.means[j];
    p[1] = G.means[G.stride + j];
    p[2] = G.means[2 * G.stride + j];
#pragma unroll
    for (int r = 0; r < 8; ++r) p[3 + r] = load_attr<DT>(G.attrs, r, G.stride, j);
    spec_cov(p[3], p[4], p[5], p[6], p[7], p[8], p[9], a.rc.scale_mod, c);
  }
  const float alpha = p[10];

  float gmx = 0.f, gmy = 0.f, gmz = 0.f, galpha = 0.f;
  float st_norm = 0.f, st_rad = 0.f;
  int32_t st_cnt = 0;
  float gxx = 0.f, gxy = 0.f, gxz = 0.f, gyy = 0.f, gyz = 0.f, gzz = 0.f;
  float gls = 0.f;   // common part of the three log-scale gradients (exact convolution)

  // the next record's bookkeeping is loaded while this record is summed (the
  // moments' addresses depend on it: two dependent loads per record otherwise)
  const uint32_t rend = !go ? 0u : (rbase + nrec < a.rc.rec_cap ? rbase + nrec : a.rc.rec_cap);
  RecMeta meta_next{};
  if (rbase + li < rend) meta_next = a.rec_meta[rbase + li];
  for (uint32_t r = rbase + li; r < rend; r += (uint32_t)L) {
    const RecMeta meta = meta_next;
    if (r + (uint32_t)L < rend) meta_next = a.rec_meta[r + (uint32_t)L];
    const SliceDev sl = a.slices[meta.slice];
    const uint32_t ntiles = rec_ntiles(meta);
    float M0 = 0.f, Mx = 0.f, My = 0.f, Mxx = 0.f, Mxy = 0.f, Myy = 0.f;
    for (uint32_t s = 0; s < ntiles; ++s) {
      const float4 m0 = a.moments[2 * (size_t)(meta.ibase + s)];
      const float4 m1 = a.moments[2 * (size_t)(meta.ibase + s) + 1];
      M0 += m0.x; Mx += m0.y; My += m0.z; Mxx += m0.w; Mxy += m1.x; Myy += m1.y;
    }
    // forward quantities of this (Gaussian, slice) pair, in the slice's camera
    // frame (the world frame for axial batches)
    SpecCov cpose;
    float mpose[3];
    if (POSED) spec_pose(c, p, a.poses + 12 * meta.slice, cpose, mpose);
    const SpecCov& cv = POSED ? cpose : c;
    const float* mv = POSED ? mpose : p;
    const SpecAxial ax = spec_axial(mv[2], cv.szz, sl.z, sl.sigma_z);
    const float invD = 1.0f / ax.D;
    const float w = 1.0f / (1.0f + cv.szz / ax.s2);
    const float A = w * cv.sxx + cv.a11 * invD;
    const float C = w * cv.syy + cv.a00 * invD;
    const float B = w * cv.sxy - cv.a01 * invD;
    const float u = cv.sxz * invD, v = cv.syz * invD;
    const float det = w * cv.a22 + cv.detS * invD;
    if (!(det > 0.0f) || !isfinite(det)) continue;
    const float rho = expf(-0.5f * ax.q);
    // exact convolution integral: alpha~ carries f = sqrt(2 pi det Sigma w)
    const bool conv = (a.rc.flags & GP_FLAG_CONV_EXACT) != 0;
    const float f = conv ? sqrtf(6.28318530717958648f * cv.detS * w) : 1.0f;
    const float sq = sqrtf(det) / f;
    const float at = alpha * rho / sq;
    const float inv_det = 1.0f / det;
    const float ca = C * inv_det, cb = -B * inv_det, cc = A * inv_det;
    const float m = ax.m;
    const float ddx = sl.dx, ddy = sl.dy;

    // record gradients in world units
    const float g_at = M0;
    const float g_m2x = at * (ca * ddx * Mx + cb * ddy * My);
    const float g_m2y = at * (cb * ddx * Mx + cc * ddy * My);
    const float g_ca = -0.5f * at * Mxx * ddx * ddx;
    const float g_cb = -at * Mxy * ddx * ddy;
    const float g_cc = -0.5f * at * Myy * ddy * ddy;
    // conic -> Sigma_2d (inverse of a symmetric 2x2, b counted once)
    float gA = -(ca * ca * g_ca + ca * cb * g_cb + cb * cb * g_cc);
    float gB = -(2.f * ca * cb * g_ca + (ca * cc + cb * cb) * g_cb + 2.f * cb * cc * g_cc);
    float gC = -(cb * cb * g_ca + cb * cc * g_cb + cc * cc * g_cc);
    // alpha~ = alpha opacity_r det^(-1/2)
    const float g_det = -0.5f * g_at * at * inv_det;
    gA += C * g_det;
    gB += -2.f * B * g_det;
    gC += A * g_det;
    galpha += g_at * rho / sq;
    const float g_rho = g_at * alpha / sq;
    const float g_q = -0.5f * rho * g_rho;
    // Focus Gaussian -> camera-frame Sigma_c, mu_c
    const float g_u = -m * g_m2x, g_v = -m * g_m2y;
    float lzz = u * u * gA + u * v * gB + v * v * gC - (u * g_u + v * g_v) * invD - g_q * m * m * invD * invD;
    // d ln f = (1/2) (d ln det Sigma + d ln w), d ln det Sigma / d l_i = 2,
    // d ln w / d Sigma_zz = -1 / D
    if (conv) {
      gls += g_at * at;
      lzz += -0.5f * g_at * at * invD;
    }
    const float lxx = gA, lxy = gB, lyy = gC;
    const float lxz = -2.f * u * gA - v * gB + g_u * invD;
    const float lyz = -2.f * v * gC - u * gB + g_v * invD;
    const float lmx = g_m2x, lmy = g_m2y;
    const float lmz = -(u * g_m2x + v * g_m2y) + 2.f * g_q * m * invD;
    if (POSED) {
      // back to the world frame: dL/dSigma = R_c^T G R_c (symmetric G with the
      // off-diagonal gradients halved), dL/dmu = R_c^T dL/dmu_c
      const float* Rc = a.poses + 12 * meta.slice;
      const float G[3][3] = {{lxx, 0.5f * lxy, 0.5f * lxz}, {0.5f * lxy, lyy, 0.5f * lyz}, {0.5f * lxz, 0.5f * lyz, lzz}};
      float T[3][3];   // G R_c
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) T[i][jj] = G[i][0] * Rc[jj] + G[i][1] * Rc[3 + jj] + G[i][2] * Rc[6 + jj];
      float W[3][3];   // R_c^T T
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int jj = i; jj < 3; ++jj) W[i][jj] = Rc[i] * T[0][jj] + Rc[3 + i] * T[1][jj] + Rc[6 + i] * T[2][jj];
      gxx += W[0][0];
      gyy += W[1][1];
      gzz += W[2][2];
      gxy += 2.f * W[0][1];
      gxz += 2.f * W[0][2];
      gyz += 2.f * W[1][2];
      gmx += Rc[0] * lmx + Rc[3] * lmy + Rc[6] * lmz;
      gmy += Rc[1] * lmx + Rc[4] * lmy + Rc[7] * lmz;
      gmz += Rc[2] * lmx + Rc[5] * lmy + Rc[8] * lmz;
    } else {
      gxx += lxx;
      gxy += lxy;
      gyy += lyy;
      gxz += lxz;
      gyz += lyz;
      gzz += lzz;
      gmx += lmx;
      gmy += lmy;
      gmz += lmz;
    }
    // densification statistics in pixel units
    st_norm += sqrtf((g_m2x * ddx) * (g_m2x * ddx) + (g_m2y * ddy) * (g_m2y * ddy));
    st_rad = fmaxf(st_rad, a.rc.bbox * fmaxf(sqrtf(A) / ddx, sqrtf(C) / ddy));
    st_cnt += 1;
  }
  if constexpr (L > 1) {
    // the group's sums (the same butterfly on every lane: a fixed order)
#pragma unroll
    for (int o = 1; o < L; o <<= 1) {
      gmx += __shfl_xor(gmx, o, 64);
      gmy += __shfl_xor(gmy, o, 64);
      gmz += __shfl_xor(gmz, o, 64);
      galpha += __shfl_xor(galpha, o, 64);
      gxx += __shfl_xor(gxx, o, 64);
      gxy += __shfl_xor(gxy, o, 64);
      gxz += __shfl_xor(gxz, o, 64);
      gyy += __shfl_xor(gyy, o, 64);
      gyz += __shfl_xor(gyz, o, 64);
      gzz += __shfl_xor(gzz, o, 64);
      gls += __shfl_xor(gls, o, 64);
      st_norm += __shfl_xor(st_norm, o, 64);
      st_cnt += __shfl_xor(st_cnt, o, 64);
      st_rad = fmaxf(st_rad, __shfl_xor(st_rad, o, 64));
    }
  }
  if (!go || li != 0u) return;

  // Sigma = M M^T with M = R diag(s): dL/dM = 2 Gs M, Gs symmetric
  const float Gs[3][3] = {{gxx, 0.5f * gxy, 0.5f * gxz},
                          {0.5f * gxy, gyy, 0.5f * gyz},
                          {0.5f * gxz, 0.5f * gyz, gzz}};
  const float s[3] = {c.s0, c.s1, c.s2};
  float gM[3][3], gR[3][3], gl[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      const float mij = 2.f * (Gs[i][0] * c.R[0][jj] + Gs[i][1] * c.R[1][jj] + Gs[i][2] * c.R[2][jj]) * s[jj];
      gM[i][jj] = mij;
      gR[i][jj] = mij * s[jj];
    }
#pragma unroll
  for (int jj = 0; jj < 3; ++jj) gl[jj] = (gM[0][jj] * c.R[0][jj] + gM[1][jj] * c.R[1][jj] + gM[2][jj] * c.R[2][jj]) * s[jj];
  // rotation matrix of (w, x, y, z) -> quaternion gradient
  const float qw = c.w, qx = c.x, qy = c.y, qz = c.z;
  const float gqw = 2.f * (-qz * gR[0][1] + qy * gR[0][2] + qz * gR[1][0] - qx * gR[1][2] - qy * gR[2][0] + qx * gR[2][1]);
  const float gqx = 2.f * (qy * gR[0][1] + qz * gR[0][2] + qy * gR[1][0] - qw * gR[1][2] + qz * gR[2][0] + qw * gR[2][1])
                    - 4.f * qx * (gR[1][1] + gR[2][2]);
  const float gqy = 2.f * (qx * gR[0][1] + qw * gR[0][2] + qx * gR[1][0] + qz * gR[1][2] - qw * gR[2][0] + qz * gR[2][1])
                    - 4.f * qy * (gR[0][0] + gR[2][2]);
  const float gqz = 2.f * (-qw * gR[0][1] + qx * gR[0][2] + qw * gR[1][0] + qy * gR[1][2] + qx * gR[2][0] + qy * gR[2][1])
                    - 4.f * qz * (gR[0][0] + gR[1][1]);
  const float dotq = qw * gqw + qx * gqx + qy * gqy + qz * gqz;
  const float inv_n = 1.0f / sqrtf(c.n2);
  const float gq[4] = {(gqw - qw * dotq) * inv_n, (gqx - qx * dotq) * inv_n, (gqy - qy * dotq) * inv_n,
                       (gqz - qz * dotq) * inv_n};

  float* gp = a.grad + j;
  const int64_t gs = a.grad_stride;
  gp[0] += gmx;
  gp[gs] += gmy;
  gp[2 * gs] += gmz;
  gp[3 * gs] += gl[0] + gls;
  gp[4 * gs] += gl[1] + gls;
  gp[5 * gs] += gl[2] + gls;
  gp[6 * gs] += gq[0];
  gp[7 * gs] += gq[1];
  gp[8 * gs] += gq[2];
  gp[9 * gs] += gq[3];
  gp[10 * gs] += galpha;
  if (a.st_grad_norm && j < a.st_n) {
    a.st_grad_norm[j] += st_norm;
    a.st_count[j] += st_cnt;
    a.st_max_radius[j] = fmaxf(a.st_max_radius[j], st_rad);
  }
}

// A workgroup takes `chunk` Gaussians at a time (512), gathers those with
// records (a batch of a few slices reaches a small fraction of a large set)
// into LDS and gives them to its lanes, L per Gaussian, so that lanes do not
// idle on Gaussians without records.  Each Gaussian still has exactly one
// writer; the order in which a workgroup visits its Gaussians does not change
// any result.  512 rather than 2,048 at a time: four times the workgroups to
// hide the latency of each lane's chain over its records (measured 0.036 ->
// 0.034 ms on an 8-slice batch, 0.80 -> 0.56 ms on the 400-slice stack).
constexpr int kBwdChunk = 512;

// The workgroup's list of n Gaussians, L lanes each, in rounds of 256 / L
// (the bound is uniform over the workgroup, so every lane of a group reaches
// its exchanges).
template <int DT, bool POSED, int L>
__device__ __forceinline__ void backward_list(const BwdPreArgs& a, int n_groups, const int* list, int n) {
  for (int jb = 0; jb < n; jb += 256 / L) {
    const int jj = jb + (int)(threadIdx.x / L);
    const bool act = jj < n;
    backward_one<DT, POSED, L>(a, n_groups, act ? list[jj] : 0, act);
  }
}

template <int DT, bool POSED>
__global__ __launch_bounds__(256) void k_preprocess_bwd(BwdPreArgs a) {
  __shared__ int s_list[kBwdChunk];
  __shared__ int s_n;
  const int total = a.hdr->total_gauss;
  const int n_groups = a.hdr->n_groups;
  const int lane = threadIdx.x & 63;
  const int chunk = a.chunk;
  for (int base = blockIdx.x * chunk; base < total; base += gridDim.x * chunk) {
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    for (int i = 0; i < chunk / 256; ++i) {
      const int t = base + i * 256 + threadIdx.x;
      const bool active = t < total && a.g_nrec[t] > 0u;
      const uint64_t m = __ballot(active);
      int wbase = 0;
      if (lane == 0 && m) wbase = atomicAdd(&s_n, __popcll(m));
      wbase = __shfl(wbase, 0, 64);
      if (active) s_list[wbase + __popcll(m & ((1ull << lane) - 1ull))] = t;
    }
    __syncthreads();
    const int n = s_n;
    // as many lanes per Gaussian as fit the list in one round (n is uniform)
    if (n <= 32) backward_list<DT, POSED, 8>(a, n_groups, s_list, n);
    else if (n <= 64) backward_list<DT, POSED, 4>(a, n_groups, s_list, n);
    else if (n <= 128) backward_list<DT, POSED, 2>(a, n_groups, s_list, n);
    else backward_list<DT, POSED, 1>(a, n_groups, s_list, n);
    __syncthreads();   // s_list and s_n are rewritten by the next chunk
  }
}

template <bool POSED>
hipError_t launch_bwd_p(const BwdPreArgs& a, int attr_dtype, unsigned blocks, hipStream_t s) {
  switch (attr_dtype) {
    case GP_BF16: k_preprocess_bwd<GP_BF16, POSED><<<blocks, 256, 0, s>>>(a); break;
    case GP_F16: k_preprocess_bwd<GP_F16, POSED><<<blocks, 256, 0, s>>>(a); break;
    case GP_Q16: k_preprocess_bwd<GP_Q16, POSED><<<blocks, 256, 0, s>>>(a); break;
    default: k_preprocess_bwd<GP_F32, POSED><<<blocks, 256, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_preprocess_bwd(const RenderConst& rc, const Workspace& ws, float* grad,
                                 int64_t grad_stride, const LaunchDims& d, hipStream_t s) {
  if (d.gauss <= 0) return hipSuccess;
  BwdPreArgs a{rc,
               ws.d_hdr,
               ws.d_groups,
               ws.d_slices,
               ws.d_rec_pay,
               ws.d_rec_meta,
               ws.d_g_rbase,
               ws.d_g_nrec,
               ws.d_moments,
               grad,
               grad_stride,
               ws.st_grad_norm,
               ws.st_count,
               ws.st_max_radius,
               ws.st_n,
               ws.d_poses,
               kBwdChunk};
  int64_t blocks = (d.gauss + a.chunk - 1) / a.chunk;
  if (blocks > 16384) blocks = 16384;
  return d.posed ? launch_bwd_p<true>(a, rc.attr_dtype, (unsigned)blocks, s)
                 : launch_bwd_p<false>(a, rc.attr_dtype, (unsigned)blocks, s);
}

}  // namespace gp
