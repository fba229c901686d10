// Differentiable voxeliser (Sec. 4.3, "Differentiable Voxelization"): the
// intensity volume sigma(x) = sum_i alpha_i exp(-1/2 (x - mu_i)^T Sigma_i^-1
// (x - mu_i)) of the world-space Gaussians (no focus re-parameterisation),
// accumulated over 8 x 8 x 8-voxel tiles that keep the Gaussians whose 3-sigma
// box reaches them, and its adjoint.
//
// Pipeline (one forward, no floating-point atomics anywhere):
//   k_vox_count   per Gaussian: activation, binary32 3-sigma tile box (the same
//                 operation sequence as the slice footprint: r = bbox sqrt(S_aa),
//                 floor(((mu -+ r - origin) / pitch) / 8)), the voxel-space record;
//   scan          instance slots in Gaussian order;
//   k_vox_emit    one (tile, Gaussian) pair per tile of each box;
//   radix sort    stable, by tile: every list ends in Gaussian order;
//   k_vox_fwd     one wavefront per tile pair (shared work counter); lane (x, y) of
//                 the 8 x 8 face owns the column of 8 voxels along z, so the
//                 x-y part of the quadratic form is shared by 8 voxels.
// Backward:
//   k_vox_bwd     one lane per list entry: ten moments of G e over the tile's
//                 512 voxels (sum, first and second moments of the offset),
//                 written at the entry's own instance slot;
//   k_vox_chain   per Gaussian: moments summed in slot order, then the chain
//                 rule to (mu, l, q, alpha), added into the gradient.
//
// Voxel-space record: with o the origin, h the pitch and d = (i + 1/2) - (mu -
// o)/h the offset of voxel i from the mean in voxel units, a contribution is
// w exp2(cxx dx^2 + cyy dy^2 + czz dz^2 + cxy dx dy + cxz dx dz + cyz dy dz),
// the coefficients carrying -1/2 log2(e), the precision matrix P = Sigma^-1 =
// R diag(1/s^2) R^T and the pitches.
#include "gp_internal.h"
#include "gp_spec.h"

#include <algorithm>
#include <cmath>

namespace gp {
namespace {

constexpr int kVT = 8;                       // tile edge in voxels
constexpr int kVTVox = kVT * kVT * kVT;      // voxels per tile
constexpr float kLog2e = 1.4426950408889634f;

struct VoxArgs {
  const float* means;
  const void* attrs;
  int64_t stride;
  int n;
  float x0, y0, z0, dx, dy, dz;
  int nx, ny, nz, ntx, nty, ntz, n_tiles;
  float bbox, scale_mod;
  uint32_t flags;
  float4* rec;            // [3][n]: (x, y, z, w), (cxx, cyy, czz, cxy), (cxz, cyz, -, -)
  uint32_t* box;          // [3][n]: t0 | t1 << 16 per axis (x, y, z)
  uint32_t* ninst;        // [n] tiles of the box (0 if culled)
  const uint32_t* ibase;  // [n] first instance slot (scanned)
  uint32_t* inst_key;
  uint32_t* inst_val;
  uint32_t inst_cap;
  const uint32_t* tile_lo;
  const uint32_t* tile_hi;
  const uint32_t* list;
  float* vol;
  const float* gvol;
  float4* mom;            // [3][inst]: (M0, Mx, My, Mz), (Mxx, Myy, Mzz, Mxy), (Mxz, Myz, -, -)
  uint32_t* work;
  float* grad;
  int64_t grad_stride;
  int tile_group;         // forward: consecutive tiles per work item
};

struct VoxGauss {
  float p[11];
  SpecCov c;
  bool ok;
};

template <int DT>
__device__ __forceinline__ void vox_load(const VoxArgs& a, int j, VoxGauss& g) {
  g.p[0] = a.means[j];
  g.p[1] = a.means[a.stride + j];
  g.p[2] = a.means[2 * a.stride + j];
#pragma unroll
  for (int r = 0; r < 8; ++r) g.p[3 + r] = load_attr<DT>(a.attrs, r, a.stride, j);
  bool finite = true;
#pragma unroll
  for (int r = 0; r < 11; ++r) finite = finite && isfinite(g.p[r]);
  spec_cov(g.p[3], g.p[4], g.p[5], g.p[6], g.p[7], g.p[8], g.p[9], a.scale_mod, g.c);
  g.ok = finite && g.c.n2 > 0.0f;
}

// Binary32 tile range of one axis; false if the box misses the grid.
__device__ __forceinline__ bool vox_axis(float mu, float saa, float o, float h, int nt, float bbox, int* t0,
                                         int* t1) {
#pragma clang fp contract(off)
  const float r = bbox * sqrtf(saa);
  const float lo = floorf((((mu - r) - o) / h) * 0.125f);
  const float hi = floorf((((mu + r) - o) / h) * 0.125f);
  const float fn = (float)(nt - 1);
  if (!(hi >= 0.0f) || !(lo <= fn)) return false;
  *t0 = (int)fmaxf(lo, 0.0f);
  *t1 = (int)fminf(hi, fn);
  return true;
}

// Records with a diagonal coefficient >= -4 (sigma >= 0.42 voxel along that
// axis) take the product recurrence along it.
constexpr float kVoxSmooth = -4.0f;

template <int DT>
__global__ __launch_bounds__(256) void k_vox_count(VoxArgs a) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= a.n) return;
  VoxGauss g;
  vox_load<DT>(a, j, g);
  int tx0 = 0, tx1 = -1, ty0 = 0, ty1 = -1, tz0 = 0, tz1 = -1;
  bool vis = g.ok;
  if (vis && (a.flags & GP_FLAG_EXACT)) {
    tx0 = 0; tx1 = a.ntx - 1; ty0 = 0; ty1 = a.nty - 1; tz0 = 0; tz1 = a.ntz - 1;
  } else if (vis) {
    vis = vox_axis(g.p[0], g.c.sxx, a.x0, a.dx, a.ntx, a.bbox, &tx0, &tx1) &&
          vox_axis(g.p[1], g.c.syy, a.y0, a.dy, a.nty, a.bbox, &ty0, &ty1) &&
          vox_axis(g.p[2], g.c.szz, a.z0, a.dz, a.ntz, a.bbox, &tz0, &tz1);
  }
  uint32_t cnt = 0u;
  if (vis) cnt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1) * (tz1 - tz0 + 1));
  a.ninst[j] = cnt;
  a.box[j] = (uint32_t)tx0 | ((uint32_t)(tx1 & 0xFFFF) << 16);
  a.box[a.n + j] = (uint32_t)ty0 | ((uint32_t)(ty1 & 0xFFFF) << 16);
  a.box[2 * a.n + j] = (uint32_t)tz0 | ((uint32_t)(tz1 & 0xFFFF) << 16);
  // voxel-space record (binary32 image arithmetic, not part of the membership)
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
  if (vis) {
    const SpecCov& c = g.c;
    const float i0 = 1.0f / (c.s0 * c.s0), i1 = 1.0f / (c.s1 * c.s1), i2 = 1.0f / (c.s2 * c.s2);
    float P[3][3];
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
      for (int v = 0; v < 3; ++v) P[u][v] = c.R[u][0] * c.R[v][0] * i0 + c.R[u][1] * c.R[v][1] * i1 + c.R[u][2] * c.R[v][2] * i2;
    const float k = -0.5f * kLog2e;
    r0 = make_float4((g.p[0] - a.x0) / a.dx - 0.5f, (g.p[1] - a.y0) / a.dy - 0.5f, (g.p[2] - a.z0) / a.dz - 0.5f,
                     g.p[10]);
    r1 = make_float4(k * P[0][0] * a.dx * a.dx, k * P[1][1] * a.dy * a.dy, k * P[2][2] * a.dz * a.dz,
                     2.0f * k * P[0][1] * a.dx * a.dy);
    // the per-voxel ratio's change along z (forward columns) and along x
    // (backward rows) for the product recurrence, -1 where it is not used
    const float czz = r1.z, cxx = r1.x;
    r2 = make_float4(2.0f * k * P[0][2] * a.dx * a.dz, 2.0f * k * P[1][2] * a.dy * a.dz,
                     czz >= kVoxSmooth ? exp2f(2.0f * czz) : -1.0f, cxx >= kVoxSmooth ? exp2f(2.0f * cxx) : -1.0f);
  }
  a.rec[j] = r0;
  a.rec[a.n + j] = r1;
  a.rec[2 * a.n + j] = r2;
}

__global__ __launch_bounds__(256) void k_vox_emit(VoxArgs a) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= a.n) return;
  const uint32_t cnt = a.ninst[j];
  if (cnt == 0u) return;
  uint32_t slot = a.ibase[j];
  if ((uint64_t)slot + cnt > a.inst_cap) return;   // sized from the count: cannot happen
  const uint32_t bx = a.box[j], by = a.box[a.n + j], bz = a.box[2 * a.n + j];
  for (int tz = (int)(bz & 0xFFFFu); tz <= (int)(bz >> 16); ++tz)
    for (int ty = (int)(by & 0xFFFFu); ty <= (int)(by >> 16); ++ty)
      for (int tx = (int)(bx & 0xFFFFu); tx <= (int)(bx >> 16); ++tx, ++slot) {
        a.inst_key[slot] = (uint32_t)((tz * a.nty + ty) * a.ntx + tx);
        a.inst_val[slot] = (uint32_t)j;
      }
}

__global__ __launch_bounds__(256) void k_vox_ranges(const uint32_t* __restrict__ key, uint32_t n, uint32_t n_tiles,
                                                    uint32_t* __restrict__ lo, uint32_t* __restrict__ hi) {
  for (uint32_t p = blockIdx.x * 256 + threadIdx.x; p < n; p += gridDim.x * 256) {
    const uint32_t b = key[p];
    if (b >= n_tiles) continue;
    if (p == 0 || key[p - 1] != b) lo[b] = p;
    if (p + 1 == n || key[p + 1] != b) hi[b] = p + 1;
  }
}

__device__ __forceinline__ void vox_tile_xyz(const VoxArgs& a, int tile, int* tx, int* ty, int* tz) {
  *tx = tile % a.ntx;
  *ty = (tile / a.ntx) % a.nty;
  *tz = tile / (a.ntx * a.nty);
}

// One wavefront per work item of tile_group consecutive tiles, rendered in
// turn; lane (lx, ly) owns the column of 8 voxels along z.  Each workgroup's
// first item is its own index; the shared counter hands out the rest (every
// workgroup taking a ticket at once serialised on it).
__global__ __launch_bounds__(64) void k_vox_fwd(VoxArgs a) {
  __shared__ float4 b0[64], b1[64], b2[64];
  const int lane = threadIdx.x;
  const int lx = lane & 7, ly = lane >> 3;
  uint32_t* counter = a.work + kWorkRasterFwd;
  const int G = a.tile_group;   // consecutive tiles per work item
  const uint32_t n_items = (uint32_t)((a.n_tiles + G - 1) / G);
  const uint32_t t0 = blockIdx.x;
  int left = 0;   // further tiles of the current item
  uint32_t ticket = 0u;
  for (int tile = t0 < n_items ? (int)t0 * G : -1; tile >= 0;) {
    if (left == 0) {
      ticket = wave_take(counter) + gridDim.x;   // resolved after this item
      left = min(G, a.n_tiles - tile);
    }
    --left;
    int tx, ty, tz;
    vox_tile_xyz(a, tile, &tx, &ty, &tz);
    const float fx = (float)(tx * kVT + lx), fy = (float)(ty * kVT + ly), fz0 = (float)(tz * kVT);
    const uint32_t start = a.tile_lo[tile], end = a.tile_hi[tile];
    float acc[kVT];
#pragma unroll
    for (int k = 0; k < kVT; ++k) acc[k] = 0.f;
    for (uint32_t base = start; base < end; base += 64) {
      if (base + lane < end) {
        const uint32_t j = a.list[base + lane];
        b0[lane] = a.rec[j];
        b1[lane] = a.rec[a.n + j];
        b2[lane] = a.rec[2 * a.n + j];
      }
      __syncthreads();
      const int cnt = __builtin_amdgcn_readfirstlane((int)min(64u, end - base));
      for (int e = 0; e < cnt; ++e) {
        const float4 r0 = b0[e], r1 = b1[e], r2 = b2[e];
        const float ddx = fx - r0.x, ddy = fy - r0.y;
        // q = cxx dx^2 + cxy dx dy + cyy dy^2 + dz (cxz dx + cyz dy + czz dz)
        const float pxy = fmaf(fmaf(r1.x, ddx, r1.w * ddy), ddx, r1.y * ddy * ddy);
        const float lz = fmaf(r2.x, ddx, r2.y * ddy);
        const float dz0 = fz0 - r0.z;
        if (r2.z > 0.0f) {
          // two four-voxel segments, each from an exact exp2 by the product
          // recurrence along z (the raster's reasoning with czz >= -4: a
          // ratio that overflows meets e = 0, and 0 * inf = 0)
#pragma unroll
          for (int h = 0; h < kVT; h += 4) {
            const float dz = dz0 + (float)h;
            float e = __builtin_amdgcn_exp2f(fmaf(fmaf(r1.z, dz, lz), dz, pxy));
            float r = __builtin_amdgcn_exp2f(fmaf(r1.z, fmaf(2.0f, dz, 1.0f), lz));
            acc[h] = fmaf(r0.w, e, acc[h]);
#pragma unroll
            for (int k = 1; k < 4; ++k) {
              e = mul0(e, r);
              r *= r2.z;
              acc[h + k] = fmaf(r0.w, e, acc[h + k]);
            }
          }
        } else {
#pragma unroll
          for (int k = 0; k < kVT; ++k) {
            const float dz = dz0 + (float)k;
            const float q = fmaf(fmaf(r1.z, dz, lz), dz, pxy);
            acc[k] = fmaf(r0.w, __builtin_amdgcn_exp2f(q), acc[k]);
          }
        }
      }
      __syncthreads();
    }
    const int ix = tx * kVT + lx, iy = ty * kVT + ly;
    if (ix < a.nx && iy < a.ny) {
#pragma unroll
      for (int k = 0; k < kVT; ++k) {
        const int iz = tz * kVT + k;
        if (iz < a.nz) a.vol[((int64_t)iz * a.ny + iy) * a.nx + ix] = acc[k];
      }
    }
    if (left > 0) ++tile;
    else tile = ticket < n_items ? (int)ticket * G : -1;
  }
}

// 256 lanes per tile, one list entry per lane.
__global__ __launch_bounds__(256) void k_vox_bwd(VoxArgs a) {
  __shared__ float G[kVTVox];
  __shared__ int s_item;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // the first tile is the workgroup's own index; the counter hands out the rest
  int tile = blockIdx.x < (unsigned)a.n_tiles ? (int)blockIdx.x : -1;
  while (tile >= 0) {
    uint32_t ticket = 0u;
    if (threadIdx.x == 0) ticket = atomicAdd(&a.work[kWorkRasterBwd], 1u) + gridDim.x;
    const uint32_t start = a.tile_lo[tile], end = a.tile_hi[tile];
    if (start != end) {
    int tx, ty, tz;
    vox_tile_xyz(a, tile, &tx, &ty, &tz);
    for (int v = threadIdx.x; v < kVTVox; v += 256) {
      const int ix = tx * kVT + (v & 7), iy = ty * kVT + ((v >> 3) & 7), iz = tz * kVT + (v >> 6);
      G[v] = (ix < a.nx && iy < a.ny && iz < a.nz) ? a.gvol[((int64_t)iz * a.ny + iy) * a.nx + ix] : 0.f;
    }
    __syncthreads();
    const float fx0 = (float)(tx * kVT), fy0 = (float)(ty * kVT), fz0 = (float)(tz * kVT);
    for (uint32_t cb = start + wave * 64; cb < end; cb += 256) {
      const uint32_t idx = cb + lane;
      if (idx >= end) continue;
      const uint32_t j = a.list[idx];
      const float4 r0 = a.rec[j], r1 = a.rec[a.n + j], r2 = a.rec[2 * a.n + j];
      float dxs[kVT];
#pragma unroll
      for (int c = 0; c < kVT; ++c) dxs[c] = (fx0 - r0.x) + (float)c;
      float M0 = 0.f, Mx = 0.f, My = 0.f, Mz = 0.f, Mxx = 0.f, Myy = 0.f, Mzz = 0.f, Mxy = 0.f, Mxz = 0.f,
            Myz = 0.f;
      for (int z = 0; z < kVT; ++z) {
        const float dz = (fz0 + (float)z) - r0.z;
        for (int y = 0; y < kVT; ++y) {
          const float dy = (fy0 + (float)y) - r0.y;
          // q = cxx dx^2 + dx (cxy dy + cxz dz) + (cyy dy^2 + cyz dy dz + czz dz^2)
          const float bx = fmaf(r1.w, dy, r2.x * dz);
          const float c0 = fmaf(fmaf(r1.y, dy, r2.y * dz), dy, r1.z * dz * dz);
          const float* grow = G + (z * kVT + y) * kVT;
          float s0 = 0.f, sx = 0.f, sxx = 0.f;
          float ev[kVT];
          if (r2.w > 0.0f) {
            // the product recurrence along x over two four-voxel segments
#pragma unroll
            for (int h = 0; h < kVT; h += 4) {
              const float d = dxs[h];
              ev[h] = __builtin_amdgcn_exp2f(fmaf(fmaf(r1.x, d, bx), d, c0));
              float r = __builtin_amdgcn_exp2f(fmaf(r1.x, fmaf(2.0f, d, 1.0f), bx));
#pragma unroll
              for (int k = 1; k < 4; ++k) {
                ev[h + k] = mul0(ev[h + k - 1], r);
                r *= r2.w;
              }
            }
          } else {
#pragma unroll
            for (int c = 0; c < kVT; ++c) {
              const float d = dxs[c];
              ev[c] = __builtin_amdgcn_exp2f(fmaf(fmaf(r1.x, d, bx), d, c0));
            }
          }
#pragma unroll
          for (int c = 0; c < kVT; ++c) {
            const float d = dxs[c];
            const float we = grow[c] * ev[c];
            const float wd = we * d;
            s0 += we;
            sx += wd;
            sxx = fmaf(wd, d, sxx);
          }
          M0 += s0;
          Mx += sx;
          Mxx += sxx;
          My = fmaf(dy, s0, My);
          Mz = fmaf(dz, s0, Mz);
          Myy = fmaf(dy * dy, s0, Myy);
          Mzz = fmaf(dz * dz, s0, Mzz);
          Mxy = fmaf(dy, sx, Mxy);
          Mxz = fmaf(dz, sx, Mxz);
          Myz = fmaf(dy * dz, s0, Myz);
        }
      }
      // the entry's instance slot: its tile's rank in the Gaussian's box (row-major z, y, x)
      const uint32_t bx_ = a.box[j], by_ = a.box[a.n + j], bz_ = a.box[2 * a.n + j];
      const uint32_t x0 = bx_ & 0xFFFFu, w = (bx_ >> 16) - x0 + 1u;
      const uint32_t y0 = by_ & 0xFFFFu, hgt = (by_ >> 16) - y0 + 1u;
      const uint32_t z0 = bz_ & 0xFFFFu;
      const uint32_t slot = a.ibase[j] + (((uint32_t)tz - z0) * hgt + ((uint32_t)ty - y0)) * w + ((uint32_t)tx - x0);
      const int64_t K = a.inst_cap;
      a.mom[slot] = make_float4(M0, Mx, My, Mz);
      a.mom[K + slot] = make_float4(Mxx, Myy, Mzz, Mxy);
      a.mom[2 * K + slot] = make_float4(Mxz, Myz, 0.f, 0.f);
    }
    __syncthreads();   // G[] is reused by the next tile
    }
    if (threadIdx.x == 0) s_item = ticket < (uint32_t)a.n_tiles ? (int)ticket : -1;
    __syncthreads();
    tile = s_item;
    __syncthreads();   // s_item is rewritten at the end of this tile
  }
}

// Chain rule per Gaussian.  With d_w = h * d_v the world offset (h the pitch),
// e = exp(-1/2 d_w^T P d_w) and P = R diag(1/s^2) R^T:
//   dL/dalpha = sum G e = M0
//   dL/dmu    = alpha P (h * m1)                  (m1 = sum G e d_v)
//   dL/dP     = -1/2 alpha (h h^T) * M2           (M2 = sum G e d_v d_v^T)
//   dL/dl_k   = -2 / s_k^2 r_k^T (dL/dP) r_k      (s_k = exp(l_k) mod)
//   dL/dR_ak  = 2 / s_k^2 (dL/dP r_k)_a
// then through R(q^) and the normalisation q^ = q / |q|.
template <int DT>
__global__ __launch_bounds__(256) void k_vox_chain(VoxArgs a) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= a.n) return;
  const uint32_t cnt = a.ninst[j];
  if (cnt == 0u) return;
  VoxGauss g;
  vox_load<DT>(a, j, g);
  const int64_t K = a.inst_cap;
  float M0 = 0.f, m1[3] = {0.f, 0.f, 0.f}, M2[3][3] = {};
  const uint32_t s0 = a.ibase[j];
  for (uint32_t s = s0; s < s0 + cnt; ++s) {
    const float4 u = a.mom[s], v = a.mom[K + s], w = a.mom[2 * K + s];
    M0 += u.x;
    m1[0] += u.y; m1[1] += u.z; m1[2] += u.w;
    M2[0][0] += v.x; M2[1][1] += v.y; M2[2][2] += v.z; M2[0][1] += v.w;
    M2[0][2] += w.x; M2[1][2] += w.y;
  }
  M2[1][0] = M2[0][1]; M2[2][0] = M2[0][2]; M2[2][1] = M2[1][2];
  const SpecCov& c = g.c;
  const float alpha = g.p[10];
  const float h[3] = {a.dx, a.dy, a.dz};
  const float is[3] = {1.0f / (c.s0 * c.s0), 1.0f / (c.s1 * c.s1), 1.0f / (c.s2 * c.s2)};
  float P[3][3];
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int v = 0; v < 3; ++v) P[u][v] = c.R[u][0] * c.R[v][0] * is[0] + c.R[u][1] * c.R[v][1] * is[1] + c.R[u][2] * c.R[v][2] * is[2];
  float gmu[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) gmu[u] = alpha * (P[u][0] * h[0] * m1[0] + P[u][1] * h[1] * m1[1] + P[u][2] * h[2] * m1[2]);
  float GP[3][3];
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int v = 0; v < 3; ++v) GP[u][v] = -0.5f * alpha * h[u] * h[v] * M2[u][v];
  float gl[3], GR[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float t[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) t[u] = GP[u][0] * c.R[0][k] + GP[u][1] * c.R[1][k] + GP[u][2] * c.R[2][k];
    gl[k] = -2.0f * is[k] * (c.R[0][k] * t[0] + c.R[1][k] * t[1] + c.R[2][k] * t[2]);
#pragma unroll
    for (int u = 0; u < 3; ++u) GR[u][k] = 2.0f * is[k] * t[u];
  }
  const float w = c.w, x = c.x, y = c.y, z = c.z;
  const float gw = 2.0f * (-z * GR[0][1] + y * GR[0][2] + z * GR[1][0] - x * GR[1][2] - y * GR[2][0] + x * GR[2][1]);
  const float gx = 2.0f * (y * GR[0][1] + z * GR[0][2] + y * GR[1][0] - 2.0f * x * GR[1][1] - w * GR[1][2] +
                           z * GR[2][0] + w * GR[2][1] - 2.0f * x * GR[2][2]);
  const float gy = 2.0f * (-2.0f * y * GR[0][0] + x * GR[0][1] + w * GR[0][2] + x * GR[1][0] + z * GR[1][2] -
                           w * GR[2][0] + z * GR[2][1] - 2.0f * y * GR[2][2]);
  const float gz = 2.0f * (-2.0f * z * GR[0][0] - w * GR[0][1] + x * GR[0][2] + w * GR[1][0] - 2.0f * z * GR[1][1] +
                           y * GR[1][2] + x * GR[2][0] + y * GR[2][1]);
  // through q^ = q / |q|
  const float rn = 1.0f / sqrtf(c.n2);
  const float dot = w * gw + x * gx + y * gy + z * gz;
  float* gp = a.grad + j;
  const int64_t gs = a.grad_stride;
  gp[0] += gmu[0];
  gp[gs] += gmu[1];
  gp[2 * gs] += gmu[2];
  gp[3 * gs] += gl[0];
  gp[4 * gs] += gl[1];
  gp[5 * gs] += gl[2];
  gp[6 * gs] += (gw - w * dot) * rn;
  gp[7 * gs] += (gx - x * dot) * rn;
  gp[8 * gs] += (gy - y * dot) * rn;
  gp[9 * gs] += (gz - z * dot) * rn;
  gp[10 * gs] += M0;
}

}  // namespace

VoxLaunch vox_prepare(const gp_gaussians* g, const gp_volume_grid* grid, const gp_render_opts* o) {
  VoxLaunch L{};
  L.n = (int)g->n;
  L.ntx = (grid->nx + kVT - 1) / kVT;
  L.nty = (grid->ny + kVT - 1) / kVT;
  L.ntz = (grid->nz + kVT - 1) / kVT;
  L.n_tiles = (int64_t)L.ntx * L.nty * L.ntz;
  (void)o;
  return L;
}

static VoxArgs vox_args(const Workspace& ws, const gp_gaussians* g, const gp_volume_grid* grid,
                        const gp_render_opts* o, const VoxLaunch& L) {
  VoxArgs a{};
  a.means = static_cast<const float*>(g->means);
  a.attrs = g->attrs;
  a.stride = g->stride;
  a.n = L.n;
  a.x0 = grid->x0; a.y0 = grid->y0; a.z0 = grid->z0;
  a.dx = grid->dx; a.dy = grid->dy; a.dz = grid->dz;
  a.nx = grid->nx; a.ny = grid->ny; a.nz = grid->nz;
  a.ntx = L.ntx; a.nty = L.nty; a.ntz = L.ntz;
  a.n_tiles = (int)L.n_tiles;
  a.bbox = o->bbox_sigmas;
  a.scale_mod = o->scale_mod;
  a.flags = o->flags;
  a.rec = ws.d_vox_rec;
  a.box = ws.d_vox_box;
  a.ninst = ws.d_g_ninst;
  a.ibase = ws.d_g_rbase;
  a.inst_key = ws.d_inst_key;
  a.inst_val = ws.d_inst_val;
  a.inst_cap = (uint32_t)ws.inst_cap;
  a.tile_lo = ws.d_bin_lo;
  a.tile_hi = ws.d_bin_hi;
  a.list = ws.d_list;
  a.mom = ws.d_vox_mom;
  a.work = ws.d_work;
  a.tile_group = 1;
  return a;
}

hipError_t launch_vox_count(const Workspace& ws, const gp_gaussians* g, const gp_volume_grid* grid,
                            const gp_render_opts* o, const VoxLaunch& L, hipStream_t s) {
  if (L.n <= 0) return hipSuccess;
  const VoxArgs a = vox_args(ws, g, grid, o, L);
  const unsigned blocks = (unsigned)((L.n + 255) / 256);
  switch (g->attr_dtype) {
    case GP_BF16: k_vox_count<GP_BF16><<<blocks, 256, 0, s>>>(a); break;
    case GP_F16: k_vox_count<GP_F16><<<blocks, 256, 0, s>>>(a); break;
    case GP_Q16: k_vox_count<GP_Q16><<<blocks, 256, 0, s>>>(a); break;
    default: k_vox_count<GP_F32><<<blocks, 256, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

hipError_t launch_vox_emit(const Workspace& ws, const gp_gaussians* g, const gp_volume_grid* grid,
                           const gp_render_opts* o, const VoxLaunch& L, hipStream_t s) {
  if (L.n <= 0) return hipSuccess;
  const VoxArgs a = vox_args(ws, g, grid, o, L);
  k_vox_emit<<<(unsigned)((L.n + 255) / 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_vox_ranges(const Workspace& ws, const VoxLaunch& L, uint32_t n_inst, hipStream_t s) {
  hipError_t e = launch_fill_u32(ws.d_bin_lo, 0u, L.n_tiles, s);
  if (e == hipSuccess) e = launch_fill_u32(ws.d_bin_hi, 0u, L.n_tiles, s);
  if (e != hipSuccess || n_inst == 0) return e;
  int64_t blocks = ((int64_t)n_inst + 255) / 256;
  blocks = blocks > 8192 ? 8192 : blocks;
  k_vox_ranges<<<(unsigned)blocks, 256, 0, s>>>(ws.d_list_key, n_inst, (uint32_t)L.n_tiles, ws.d_bin_lo,
                                                ws.d_bin_hi);
  return hipGetLastError();
}

hipError_t launch_vox_fwd(const Workspace& ws, const gp_gaussians* g, const gp_volume_grid* grid,
                          const gp_render_opts* o, const VoxLaunch& L, float* vol, hipStream_t s) {
  if (L.n_tiles <= 0) return hipSuccess;
  hipError_t e = launch_fill_u32(ws.d_work + kWorkRasterFwd, 0u, 1, s);
  if (e != hipSuccess) return e;
  VoxArgs a = vox_args(ws, g, grid, o, L);
  a.vol = vol;
  const int64_t blocks = L.n_tiles < 8192 ? L.n_tiles : 8192;
  // pairs of consecutive tiles (along x) per work item while there are still
  // two items per workgroup: the second tile's gathers find most of its
  // records in the cache (256 x 256 x 400 voxels: 0.79 -> 0.62 ms; four
  // tiles 0.62-0.64, eight 0.65-0.66)
  a.tile_group = L.n_tiles >= 2 * blocks ? 2 : 1;
  k_vox_fwd<<<(unsigned)blocks, 64, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_vox_bwd(const Workspace& ws, const gp_gaussians* g, const gp_volume_grid* grid,
                          const gp_render_opts* o, const VoxLaunch& L, const float* gvol, float* grad,
                          int64_t grad_stride, hipStream_t s) {
  if (L.n_tiles <= 0 || L.n <= 0) return hipSuccess;
  hipError_t e = launch_fill_u32(ws.d_work + kWorkRasterBwd, 0u, 1, s);
  if (e != hipSuccess) return e;
  VoxArgs a = vox_args(ws, g, grid, o, L);
  a.gvol = gvol;
  a.grad = grad;
  a.grad_stride = grad_stride;
  const int64_t blocks = L.n_tiles < 2048 ? L.n_tiles : 2048;
  k_vox_bwd<<<(unsigned)blocks, 256, 0, s>>>(a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned gb = (unsigned)((L.n + 255) / 256);
  switch (g->attr_dtype) {
    case GP_BF16: k_vox_chain<GP_BF16><<<gb, 256, 0, s>>>(a); break;
    case GP_F16: k_vox_chain<GP_F16><<<gb, 256, 0, s>>>(a); break;
    case GP_Q16: k_vox_chain<GP_Q16><<<gb, 256, 0, s>>>(a); break;
    default: k_vox_chain<GP_F32><<<gb, 256, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

}  // namespace gp
