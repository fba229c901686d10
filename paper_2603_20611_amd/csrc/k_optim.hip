// Fused Adam over the [11][stride] parameter planes (Kingma & Ba, Algorithm 1;
// the optimiser of Sec. 5.1 with one learning rate per parameter group) and
// the L1 term of the slice loss (Sec. 4.3, loss function).  Both are HBM-bound
// streams: Adam reads p, g, m, v and writes p, m, v (28 bytes per element),
// the L1 kernel reads two images and writes one.
#include "gp_internal.h"

namespace gp {
namespace {

struct AdamArgs {
  float* p;
  float* g;
  float* m;
  float* v;
  int64_t n, stride;
  float lr[4];
  float b1, b2, eps, inv_bc1, inv_bc2;
  uint32_t flags;
};

__device__ __forceinline__ int group_of_row(int r) { return r < 3 ? 0 : (r < 6 ? 1 : (r < 10 ? 2 : 3)); }

__device__ __forceinline__ float adam1(float& p, float g, float& m, float& v, float lr, const AdamArgs& a) {
  m = a.b1 * m + (1.0f - a.b1) * g;
  v = a.b2 * v + (1.0f - a.b2) * g * g;
  p -= lr * (m * a.inv_bc1) / (sqrtf(v * a.inv_bc2) + a.eps);
  return p;
}

// grid.y = parameter row; each thread updates two groups of four consecutive
// elements.
__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
  const int row = blockIdx.y;
  const float lr = a.lr[group_of_row(row)];
  const bool clamp = (a.flags & GP_ADAM_CLAMP_ALPHA) && row == 10;
  const bool zero = (a.flags & GP_ADAM_ZERO_GRAD) != 0;
  const int64_t base = (int64_t)row * a.stride;
  // a workgroup covers 2,048 elements: each thread two groups of four, 1,024
  // apart, loaded together when both are whole (eight loads in flight per
  // array); a tail group takes the single-group path
  const int64_t b0 = (int64_t)blockIdx.x * 2048 + threadIdx.x * 4;
  const int64_t b1 = b0 + 1024;
  const bool aligned = (a.stride & 3) == 0;
  if (aligned && b1 + 4 <= a.n) {
    float* __restrict__ P = a.p + base;
    float* __restrict__ Gr = a.g + base;
    float* __restrict__ M = a.m + base;
    float* __restrict__ V = a.v + base;
    float4 p[2] = {*reinterpret_cast<float4*>(P + b0), *reinterpret_cast<float4*>(P + b1)};
    const float4 g[2] = {*reinterpret_cast<const float4*>(Gr + b0), *reinterpret_cast<const float4*>(Gr + b1)};
    float4 m[2] = {*reinterpret_cast<float4*>(M + b0), *reinterpret_cast<float4*>(M + b1)};
    float4 v[2] = {*reinterpret_cast<float4*>(V + b0), *reinterpret_cast<float4*>(V + b1)};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      adam1(p[h].x, g[h].x, m[h].x, v[h].x, lr, a);
      adam1(p[h].y, g[h].y, m[h].y, v[h].y, lr, a);
      adam1(p[h].z, g[h].z, m[h].z, v[h].z, lr, a);
      adam1(p[h].w, g[h].w, m[h].w, v[h].w, lr, a);
      if (clamp) {
        p[h].x = fmaxf(p[h].x, 0.f); p[h].y = fmaxf(p[h].y, 0.f); p[h].z = fmaxf(p[h].z, 0.f); p[h].w = fmaxf(p[h].w, 0.f);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t i = h ? b1 : b0;
      *reinterpret_cast<float4*>(P + i) = p[h];
      *reinterpret_cast<float4*>(M + i) = m[h];
      *reinterpret_cast<float4*>(V + i) = v[h];
      if (zero) *reinterpret_cast<float4*>(Gr + i) = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    return;
  }
  for (int h = 0; h < 2; ++h) {
  const int64_t i0 = h ? b1 : b0;
  if (i0 >= a.n) return;
  const bool vec = (i0 + 4 <= a.n) && ((a.stride & 3) == 0);
  if (vec) {
    float4 p = *reinterpret_cast<float4*>(a.p + base + i0);
    float4 g = *reinterpret_cast<const float4*>(a.g + base + i0);
    float4 m = *reinterpret_cast<float4*>(a.m + base + i0);
    float4 v = *reinterpret_cast<float4*>(a.v + base + i0);
    adam1(p.x, g.x, m.x, v.x, lr, a);
    adam1(p.y, g.y, m.y, v.y, lr, a);
    adam1(p.z, g.z, m.z, v.z, lr, a);
    adam1(p.w, g.w, m.w, v.w, lr, a);
    if (clamp) {
      p.x = fmaxf(p.x, 0.f); p.y = fmaxf(p.y, 0.f); p.z = fmaxf(p.z, 0.f); p.w = fmaxf(p.w, 0.f);
    }
    *reinterpret_cast<float4*>(a.p + base + i0) = p;
    *reinterpret_cast<float4*>(a.m + base + i0) = m;
    *reinterpret_cast<float4*>(a.v + base + i0) = v;
    if (zero) *reinterpret_cast<float4*>(a.g + base + i0) = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    for (int64_t i = i0; i < a.n && i < i0 + 4; ++i) {
      float p = a.p[base + i], m = a.m[base + i], v = a.v[base + i];
      adam1(p, a.g[base + i], m, v, lr, a);
      if (clamp) p = fmaxf(p, 0.f);
      a.p[base + i] = p;
      a.m[base + i] = m;
      a.v[base + i] = v;
      if (zero) a.g[base + i] = 0.f;
    }
  }
  }
}

__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ img, const float* __restrict__ tgt,
                                            int64_t n, float scale, float* __restrict__ grad,
                                            float* __restrict__ loss) {
  __shared__ float red[4];
  float acc = 0.f;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const float d = img[i] - tgt[i];
    grad[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
    acc += fabsf(d);
  }
  if (loss == nullptr) return;
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, scale * (red[0] + red[1] + red[2] + red[3]));
}

}  // namespace

hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t n, int64_t stride,
                       const gp_adam_cfg& c, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  AdamArgs a;
  a.p = p; a.g = g; a.m = m; a.v = v; a.n = n; a.stride = stride;
  for (int i = 0; i < 4; ++i) a.lr[i] = c.lr[i];
  a.b1 = c.beta1; a.b2 = c.beta2; a.eps = c.eps;
  a.inv_bc1 = (float)(1.0 / (1.0 - std::pow((double)c.beta1, (double)c.step)));
  a.inv_bc2 = (float)(1.0 / (1.0 - std::pow((double)c.beta2, (double)c.step)));
  a.flags = c.flags;
  const int64_t per_block = 2048;
  dim3 grid((unsigned)((n + per_block - 1) / per_block), 11);
  k_adam<<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_l1(const float* img, const float* tgt, int64_t n, float scale, float* grad, float* loss,
                     hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_l1<<<(unsigned)blocks, 256, 0, s>>>(img, tgt, n, scale, grad, loss);
  return hipGetLastError();
}

}  // namespace gp
