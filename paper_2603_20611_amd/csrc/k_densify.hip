// Densify and prune (Sec. 4.3, "Prune and densification": a densify-and-prune
// strategy driven by the footprint ("focus") radii of the Gaussians on the
// slices and by their intensity; thresholds from Sec. 5.1: gradient 5e-5,
// minimum intensity 0.02).  The paper gives the criteria, not the procedure;
// this follows the usual Gaussian-splatting control:
//   prune  alpha < min_alpha, or largest footprint radius > max_radius (px);
//   grow   mean projected-mean gradient (pixel units, per record) above
//          grad_threshold: clone (exact copy) if the largest scale is at most
//          split_scale, otherwise split into two children at mu + R diag(s) n_k
//          (n_k from the caller's noise) with log-scales reduced by
//          ln(split_factor);
//   Adam moments are carried over for kept Gaussians and zero for new ones.
// Three steps without atomics: mark (0, 1 or 2 outputs per Gaussian), an
// exclusive scan, emit in Gaussian order.
#include "gp_internal.h"
#include "gp_spec.h"

namespace gp {
namespace {

enum : uint32_t { kDrop = 0, kKeep = 1, kClone = 2, kSplit = 3 };

struct DensifyArgs {
  const float* p;
  const float* m;
  const float* v;
  int64_t n, stride;
  const float* grad_norm;
  const int32_t* count;
  const float* max_radius;
  const float* noise;     // [6][n]: two 3-vectors per Gaussian
  gp_densify_cfg cfg;
  uint32_t* action;
  uint32_t* outs;         // outputs per Gaussian, then (scanned) first output index
  float* p_out;
  float* m_out;
  float* v_out;
  int64_t stride_out;
};

__global__ __launch_bounds__(256) void k_densify_mark(DensifyArgs a) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= a.n) return;
  const float alpha = a.p[10 * a.stride + j];
  const float rad = a.max_radius[j];
  uint32_t act = kKeep;
  bool finite = true;
  for (int r = 0; r < 11; ++r) finite = finite && isfinite(a.p[r * a.stride + j]);
  if (!finite || !(alpha >= a.cfg.min_alpha) || rad > a.cfg.max_radius) {
    act = kDrop;
  } else if (a.count[j] > 0 && a.grad_norm[j] / (float)a.count[j] > a.cfg.grad_threshold) {
    const float lmax = fmaxf(a.p[3 * a.stride + j], fmaxf(a.p[4 * a.stride + j], a.p[5 * a.stride + j]));
    act = (expf(lmax) <= a.cfg.split_scale) ? kClone : kSplit;
  }
  a.action[j] = act;
  a.outs[j] = act == kDrop ? 0u : (act == kKeep ? 1u : 2u);
}

__global__ __launch_bounds__(256) void k_densify_emit(DensifyArgs a) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= a.n) return;
  const uint32_t act = a.action[j];
  if (act == kDrop) return;
  const int64_t o = a.outs[j];
  const int64_t so = a.stride_out, si = a.stride;
  float par[11];
  for (int r = 0; r < 11; ++r) par[r] = a.p[r * si + j];
  if (act == kSplit) {
    SpecCov c;
    spec_cov(par[3], par[4], par[5], par[6], par[7], par[8], par[9], 1.0f, c);
    const float s[3] = {c.s0, c.s1, c.s2};
    const float dl = logf(a.cfg.split_factor);
    for (int k = 0; k < 2; ++k) {
      float nk[3];
      for (int i = 0; i < 3; ++i) nk[i] = a.noise[(3 * k + i) * a.n + j];
      for (int i = 0; i < 3; ++i) {
        const float off = c.R[i][0] * s[0] * nk[0] + c.R[i][1] * s[1] * nk[1] + c.R[i][2] * s[2] * nk[2];
        a.p_out[i * so + o + k] = par[i] + off;
      }
      for (int r = 3; r < 6; ++r) a.p_out[r * so + o + k] = par[r] - dl;
      for (int r = 6; r < 11; ++r) a.p_out[r * so + o + k] = par[r];
      for (int r = 0; r < 11; ++r) {
        a.m_out[r * so + o + k] = 0.0f;
        a.v_out[r * so + o + k] = 0.0f;
      }
    }
    return;
  }
  for (int r = 0; r < 11; ++r) {
    a.p_out[r * so + o] = par[r];
    a.m_out[r * so + o] = a.m[r * si + j];
    a.v_out[r * so + o] = a.v[r * si + j];
  }
  if (act == kClone) {
    for (int r = 0; r < 11; ++r) {
      a.p_out[r * so + o + 1] = par[r];
      a.m_out[r * so + o + 1] = 0.0f;
      a.v_out[r * so + o + 1] = 0.0f;
    }
  }
}

}  // namespace

hipError_t launch_densify(const float* p, const float* m, const float* v, int64_t n, int64_t stride,
                          const float* grad_norm, const int32_t* count, const float* max_radius, const float* noise,
                          const gp_densify_cfg& cfg, uint32_t* action, uint32_t* outs, uint32_t* scan_part,
                          uint32_t* total, float* p_out, float* m_out, float* v_out, int64_t stride_out,
                          bool emit, hipStream_t s) {
  DensifyArgs a{p, m, v, n, stride, grad_norm, count, max_radius, noise, cfg, action, outs,
                p_out, m_out, v_out, stride_out};
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (!emit) {
    k_densify_mark<<<blocks, 256, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_scan_u32(outs, outs, nullptr, n, scan_part, total, s);
  }
  k_densify_emit<<<blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace gp
