// Slice loss L = mean |I - T| + lambda (1 - mean SSIM) and dL/dI (Sec. 4.3, loss
// function: an L1 term plus a D-SSIM term weighted by lambda; lambda = 0.2 in
// Sec. 5.1).  SSIM follows Wang et al. 2004: local means, variances and the
// covariance under an 11 x 11 Gaussian window (sigma 1.5, unit sum; zeros
// outside the slice), C1 = 0.01^2, C2 = 0.03^2.
//
// With A1 = 2 mx my + C1, A2 = 2 sxy + C2, B1 = mx^2 + my^2 + C1,
// B2 = sxx + syy + C2 and S = A1 A2 / (B1 B2), S at pixel q depends on the
// image only through the window sums mx, E[x^2] and E[xy] at q:
//   dS/dmx    = 2 my (A2 - A1) / (B1 B2) - 2 mx S (1/B1 - 1/B2)
//   dS/dE[x2] = -S / B2
//   dS/dE[xy] = 2 A1 / (B1 B2)
// so dL/dI(p) = sign(I - T)/n - lambda/n (W*c_mu + 2 I W*c_x2 + T W*c_xy)(p),
// where W* is the (symmetric) window filter of the three coefficient maps.
//
// Two stencil kernels, each over 32 x 16 output tiles with a 5-pixel halo in
// LDS and the 11-tap filter applied separably (columns, then rows: the column
// pass covers only the output rows, and the smaller LDS footprint lets four
// and six workgroups share a CU, so that a 256^2 x 8 batch runs in one round):
//   k_ssim_stats: five window sums -> S and the three coefficient maps;
//   k_ssim_grad:  window sums of the three maps -> dL/dI (its first workgroup
//                 also adds up the loss terms).
// Both compute in float64: the moments form of the variances (E[x^2] - mx^2)
// and the sum mx-term + 2 I x2-term cancel to a few bits in smooth regions,
// and the whole loss costs about 300 flops per pixel, far from any bound.
#include <mutex>

#include "gp_internal.h"

namespace gp {
namespace {

constexpr int kSW = 32, kSH = 16, kR = 5, kRW = kSW + 2 * kR, kRH = kSH + 2 * kR;

struct SsimArgs {
  const float* x;       // [S][H][W] rendered slices
  const float* y;       // [S][H][W] targets
  double* maps;         // [3][S][H][W] coefficient maps
  double* part;         // [2][blocks]: per-block sums of the two loss terms
  float* grad;          // [S][H][W] dL/dI (written)
  float* loss;          // [2]: += L1 term, += D-SSIM term
  int W, H;
  int64_t npix;         // S * H * W
  double inv_n, lam;
  double w[2 * kR + 1];
};

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < 4; ++i) t += sh[i];
  return t;
}

__global__ __launch_bounds__(256) void k_ssim_stats(SsimArgs a) {
  __shared__ float xs[kRH][kRW], ys[kRH][kRW];
  __shared__ double vs[5][kSH][kRW];   // column sums (36 KB in all: four workgroups per CU)
  __shared__ double red[4];
  const int s = blockIdx.z;
  const int ox = blockIdx.x * kSW, oy = blockIdx.y * kSH;
  const int64_t base = (int64_t)s * a.H * a.W;
  const float* X = a.x + base;
  const float* Y = a.y + base;
  for (int i = threadIdx.x; i < kRH * kRW; i += 256) {
    const int r = i / kRW, c = i % kRW;
    const int gx = ox - kR + c, gy = oy - kR + r;
    const bool in = gx >= 0 && gx < a.W && gy >= 0 && gy < a.H;
    xs[r][c] = in ? X[(int64_t)gy * a.W + gx] : 0.f;
    ys[r][c] = in ? Y[(int64_t)gy * a.W + gx] : 0.f;
  }
  __syncthreads();
  // the filter along columns first (the output rows over the halo's width),
  // then along rows
  for (int i = threadIdx.x; i < kSH * kRW; i += 256) {
    const int r = i / kRW, c = i % kRW;
    double sx = 0.0, sy = 0.0, sxx = 0.0, syy = 0.0, sxy = 0.0;
#pragma unroll
    for (int k = 0; k <= 2 * kR; ++k) {
      const double u = xs[r + k][c], v = ys[r + k][c], wk = a.w[k];
      sx += wk * u;
      sy += wk * v;
      sxx += wk * (u * u);
      syy += wk * (v * v);
      sxy += wk * (u * v);
    }
    vs[0][r][c] = sx;
    vs[1][r][c] = sy;
    vs[2][r][c] = sxx;
    vs[3][r][c] = syy;
    vs[4][r][c] = sxy;
  }
  __syncthreads();
  double part_l1 = 0.0, part_d = 0.0;
  for (int i = threadIdx.x; i < kSH * kSW; i += 256) {
    const int r = i / kSW, c = i % kSW;
    const int gx = ox + c, gy = oy + r;
    if (gx >= a.W || gy >= a.H) continue;
    double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k <= 2 * kR; ++k) {
      const double wk = a.w[k];
#pragma unroll
      for (int q = 0; q < 5; ++q) m[q] += wk * vs[q][r][c + k];
    }
    const double mx = m[0], my = m[1];
    const double vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
    const double A1 = 2.0 * mx * my + 1e-4, A2 = 2.0 * cxy + 9e-4;
    const double B1 = mx * mx + my * my + 1e-4, B2 = vx + vy + 9e-4;
    const double inv = 1.0 / (B1 * B2);
    const double S = A1 * A2 * inv;
    const double c_mu = 2.0 * my * (A2 - A1) * inv - 2.0 * mx * S * (1.0 / B1 - 1.0 / B2);
    const double c_x2 = -S / B2;
    const double c_xy = 2.0 * A1 * inv;
    const int64_t o = base + (int64_t)gy * a.W + gx;
    a.maps[o] = c_mu;
    a.maps[a.npix + o] = c_x2;
    a.maps[2 * a.npix + o] = c_xy;
    part_d += 1.0 - S;
    part_l1 += fabs((double)xs[r + kR][c + kR] - (double)ys[r + kR][c + kR]);
  }
  const double t1 = block_sum(part_l1, red);
  __syncthreads();
  const double t2 = block_sum(part_d, red);
  if (threadIdx.x == 0) {
    const int64_t bid = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    a.part[2 * bid] = t1;
    a.part[2 * bid + 1] = t2;
  }
}

// The two loss terms from the per-block sums of k_ssim_stats, in a fixed order
// (one writer: deterministic, and no contended atomics).  Run by the first
// workgroup of k_ssim_grad, which starts after every sum is written.
__device__ void ssim_loss_sum(const double* __restrict__ part, int64_t nblocks, double inv_n,
                              float* __restrict__ loss, double* red) {
  double s1 = 0.0, s2 = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += 256) {
    s1 += part[2 * b];
    s2 += part[2 * b + 1];
  }
  const double t1 = block_sum(s1, red);
  __syncthreads();
  const double t2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    loss[0] += (float)(t1 * inv_n);
    loss[1] += (float)(t2 * inv_n);
  }
}

__global__ __launch_bounds__(256) void k_ssim_grad(SsimArgs a) {
  // the three maps with their halo (26 KB: six workgroups per CU); after the
  // column pass its first kSH rows hold the column sums
  __shared__ double ms[3][kRH][kRW];
  const int s = blockIdx.z;
  const int ox = blockIdx.x * kSW, oy = blockIdx.y * kSH;
  const int64_t base = (int64_t)s * a.H * a.W;
  for (int i = threadIdx.x; i < kRH * kRW; i += 256) {
    const int r = i / kRW, c = i % kRW;
    const int gx = ox - kR + c, gy = oy - kR + r;
    const bool in = gx >= 0 && gx < a.W && gy >= 0 && gy < a.H;
    const int64_t o = base + (int64_t)gy * a.W + gx;
#pragma unroll
    for (int q = 0; q < 3; ++q) ms[q][r][c] = in ? a.maps[q * a.npix + o] : 0.0;
  }
  __syncthreads();
  constexpr int kCol = (kSH * kRW + 255) / 256;   // column sums per thread
  double t[kCol][3];
#pragma unroll
  for (int it = 0; it < kCol; ++it) {
    const int i = threadIdx.x + it * 256;
#pragma unroll
    for (int q = 0; q < 3; ++q) t[it][q] = 0.0;
    if (i < kSH * kRW) {
      const int r = i / kRW, c = i % kRW;
#pragma unroll
      for (int k = 0; k <= 2 * kR; ++k) {
        const double wk = a.w[k];
#pragma unroll
        for (int q = 0; q < 3; ++q) t[it][q] += wk * ms[q][r + k][c];
      }
    }
  }
  __syncthreads();   // every column sum read its inputs before any is stored
#pragma unroll
  for (int it = 0; it < kCol; ++it) {
    const int i = threadIdx.x + it * 256;
    if (i < kSH * kRW) {
      const int r = i / kRW, c = i % kRW;
#pragma unroll
      for (int q = 0; q < 3; ++q) ms[q][r][c] = t[it][q];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSH * kSW; i += 256) {
    const int r = i / kSW, c = i % kSW;
    const int gx = ox + c, gy = oy + r;
    if (gx >= a.W || gy >= a.H) continue;
    double u[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k <= 2 * kR; ++k) {
      const double wk = a.w[k];
#pragma unroll
      for (int q = 0; q < 3; ++q) u[q] += wk * ms[q][r][c + k];
    }
    const int64_t o = base + (int64_t)gy * a.W + gx;
    const double xv = a.x[o], yv = a.y[o];
    const double sg = xv > yv ? 1.0 : (xv < yv ? -1.0 : 0.0);
    const double dS = u[0] + 2.0 * xv * u[1] + yv * u[2];
    a.grad[o] = (float)(a.inv_n * (sg - a.lam * dS));
  }
  if (a.loss && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0) {
    __shared__ double red[4];
    ssim_loss_sum(a.part, (int64_t)gridDim.x * gridDim.y * gridDim.z, a.inv_n, a.loss, red);
  }
}

// Scratch of the allocation-free loss entry point: the coefficient maps of up to
// 2^21 pixels and the per-block sums, held by every GPU the library runs on
// until the process ends.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in): its device address is looked up once per
// device, with that device current, and that address is used instead.
constexpr int64_t kNoAllocScratchDoubles = 3ll * (1ll << 21) + (1ll << 17);
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

}  // namespace

int64_t ssim_noalloc_capacity() { return kNoAllocScratchDoubles; }

hipError_t ssim_noalloc_scratch(double** out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

int64_t ssim_scratch(int n_slices, int width, int height) {
  const int64_t blocks = (int64_t)((width + kSW - 1) / kSW) * ((height + kSH - 1) / kSH) * n_slices;
  return 3 * (int64_t)n_slices * width * height + 2 * blocks;
}

hipError_t launch_ssim_loss(const float* x, const float* y, int n_slices, int width, int height, double lam,
                            double* maps, float* grad, float* loss, hipStream_t s) {
  SsimArgs a{};
  a.x = x;
  a.y = y;
  a.maps = maps;
  a.part = maps + 3 * (int64_t)n_slices * width * height;
  a.grad = grad;
  a.loss = loss;
  a.W = width;
  a.H = height;
  a.npix = (int64_t)n_slices * width * height;
  a.inv_n = 1.0 / (double)a.npix;
  a.lam = lam;
  double sum = 0.0;
  for (int k = 0; k <= 2 * kR; ++k) {
    const double d = (double)(k - kR);
    a.w[k] = std::exp(-(d * d) / (2.0 * 1.5 * 1.5));
    sum += a.w[k];
  }
  for (int k = 0; k <= 2 * kR; ++k) a.w[k] /= sum;
  const dim3 grid((unsigned)((width + kSW - 1) / kSW), (unsigned)((height + kSH - 1) / kSH), (unsigned)n_slices);
  k_ssim_stats<<<grid, 256, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_ssim_grad<<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace gp
