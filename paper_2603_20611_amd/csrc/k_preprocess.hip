// Forward preprocess: per Gaussian, activation (s, q -> Sigma), then for every
// slice of its group the axial cull, Focus-Gaussian projection, normalised
// intensity and tile footprint (Sec. 4.2: axial re-parameterisation, opacity
// modulation, screen-space projection, intensity normalisation).
//
// One thread per Gaussian, looping over the slices of its group, so the
// covariance is built once per launch and reused by every slice.  For a stack
// of slices with non-decreasing z and one sigma_z, the kept slices of a
// Gaussian are a contiguous range (the binary32 axial test is monotone in |m|
// on either side of mu_z) found by binary search with the exact test, so the
// loop visits only those.  A first pass counts the Gaussian's visible records
// and footprint tiles; one atomic per wavefront (an inclusive scan across the
// lanes) then reserves contiguous record and instance slots, and a second
// pass writes them.  Every footprint tile takes a rank in its bin with an
// atomic increment; the bin scan turns (bin, rank) into a list position.
#include "gp_internal.h"
#include "gp_spec.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace gp {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

template <int DT>
__device__ __forceinline__ float load_attr(const void* base, int64_t idx) {
  if constexpr (DT == GP_F32) {
    return static_cast<const float*>(base)[idx];
  } else if constexpr (DT == GP_BF16) {
    return __bfloat162float(static_cast<const __hip_bfloat16*>(base)[idx]);
  } else {
    return __half2float(static_cast<const __half*>(base)[idx]);
  }
}

// Reserves n consecutive slots for every lane of a full wavefront; returns the
// lane's first slot.  All 64 lanes must call it together.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t* ctr, uint32_t n) {
  const int lane = __lane_id();
  uint32_t incl = n;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  uint32_t base = 0;
  if (total != 0) {
    if (lane == 63) base = atomicAdd(ctr, total);
    base = __shfl(base, 63, 64);
  }
  return base + incl - n;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = value;
}

// Zeroes the per-forward counters, the work queues and the bin counts of the
// batch described by the device header.
__global__ void k_reset(const BatchHdr* __restrict__ hdr, uint32_t* __restrict__ ctr, uint32_t* __restrict__ work,
                        uint32_t* __restrict__ bin_count, int clear_overflow) {
  const int64_t n = hdr->n_bins;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    ctr[kCtrRecords] = 0u;
    ctr[kCtrInstances] = 0u;
    if (clear_overflow) ctr[kCtrOverflow] = 0u;
    for (int i = 0; i < kWorkCount; ++i) work[i] = 0u;
  }
  for (int64_t i = t; i < n; i += stride) bin_count[i] = 0u;
}

struct PreArgs {
  RenderConst rc;
  const BatchHdr* hdr;
  const GroupDev* groups;
  const SliceDev* slices;
  uint32_t* ctr;
  uint32_t* bin_count;
  RecPay* rec_pay;
  RecMeta* rec_meta;
  uint32_t* g_rbase;
  uint32_t* g_nrec;
  uint32_t* inst_rank;
};

__device__ __forceinline__ bool kept_on(const PreArgs& a, float muz, float szz, int k) {
  const SpecAxial ax = spec_axial(muz, szz, a.slices[k].z, a.slices[k].sigma_z);
  return ax.q <= a.rc.q_cut;
}

// Kept slices [*kb, *ke) of a Gaussian in a z-sorted, single-sigma_z group.
__device__ __forceinline__ void kept_range(const PreArgs& a, const GroupDev& G, float muz, float szz, int* kb,
                                           int* ke) {
  // last slice with z <= mu_z (or k0 - 1)
  int lo = G.k0, hi = G.k1 - 1, ks = G.k0 - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    if (a.slices[mid].z <= muz) { ks = mid; lo = mid + 1; } else { hi = mid - 1; }
  }
  // the smallest q is at ks or ks + 1
  int kmin = -1;
  if (ks >= G.k0 && kept_on(a, muz, szz, ks)) kmin = ks;
  else if (ks + 1 < G.k1 && kept_on(a, muz, szz, ks + 1)) kmin = ks + 1;
  if (kmin < 0) { *kb = *ke = G.k0; return; }
  // first kept slice in [k0, kmin] (q non-increasing there)
  lo = G.k0; hi = kmin;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (kept_on(a, muz, szz, mid)) hi = mid; else lo = mid + 1;
  }
  *kb = lo;
  // last kept slice in [kmin, k1) (q non-decreasing there)
  lo = kmin; hi = G.k1 - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (kept_on(a, muz, szz, mid)) lo = mid; else hi = mid - 1;
  }
  *ke = lo + 1;
}

// One flattened Gaussian t (all 64 lanes of a wavefront call this together).
template <int DT>
__device__ __forceinline__ void preprocess_one(const PreArgs& a, int n_groups, int t) {
  const int wave0 = t & ~63;
  // group of this wavefront (groups start at multiples of 64)
  int g = 0;
  for (int jg = 1; jg < n_groups; ++jg)
    if (a.groups[jg].gbase <= wave0) g = jg;
  const GroupDev G = a.groups[g];
  const int j = t - G.gbase;
  const bool in_range = j < G.n;

  float p[11];
  if (in_range) {
    p[0] = G.means[j];
    p[1] = G.means[G.stride + j];
    p[2] = G.means[2 * G.stride + j];
#pragma unroll
    for (int r = 0; r < 8; ++r) p[3 + r] = load_attr<DT>(G.attrs, r * G.stride + j);
  } else {
#pragma unroll
    for (int r = 0; r < 11; ++r) p[r] = 0.0f;
  }
  bool finite = in_range;
#pragma unroll
  for (int r = 0; r < 11; ++r) finite = finite && isfinite(p[r]);

  SpecCov c;
  spec_cov(p[3], p[4], p[5], p[6], p[7], p[8], p[9], a.rc.scale_mod, c);
  const bool ok = finite && (c.n2 > 0.0f);
  const bool exact = (a.rc.flags & GP_FLAG_EXACT) != 0;

  // candidate slices
  int kb = G.k0, ke = G.k1;
  if (!ok) {
    ke = kb;
  } else if (!exact && (G.flags & kGroupSortedZ)) {
    kept_range(a, G, p[2], c.szz, &kb, &ke);
  }

  // pass 1: count visible records and their footprint tiles
  uint32_t nrec = 0, ninst = 0;
  for (int k = kb; k < ke; ++k) {
    const SliceDev& sl = a.slices[k];
    const SpecAxial ax = spec_axial(p[2], c.szz, sl.z, sl.sigma_z);
    if (!exact && !(ax.q <= a.rc.q_cut)) continue;
    SpecRect rect;
    if (exact) {
      rect.tx0 = 0; rect.tx1 = sl.ntx - 1; rect.ty0 = 0; rect.ty1 = sl.nty - 1;
    } else if (!spec_rect(c, p[0], p[1], ax, sl.x0, sl.y0, sl.dx, sl.dy, sl.ntx, sl.nty, a.rc.bbox, rect)) {
      continue;
    }
    nrec += 1u;
    ninst += (uint32_t)((rect.tx1 - rect.tx0 + 1) * (rect.ty1 - rect.ty0 + 1));
  }
  const uint32_t rbase = wave_reserve(&a.ctr[kCtrRecords], nrec);
  const uint32_t ibase = wave_reserve(&a.ctr[kCtrInstances], ninst);
  const bool fits = (uint64_t)rbase + nrec <= a.rc.rec_cap && (uint64_t)ibase + ninst <= a.rc.inst_cap;
  a.g_rbase[t] = rbase;
  a.g_nrec[t] = fits ? nrec : 0u;
  if (!fits) {
    // overflow: the reserved record slots inside the capacity stay unused and
    // are marked so that no later kernel reads them
    a.ctr[kCtrOverflow] = 1u;
    for (uint32_t r = rbase; r < rbase + nrec && r < a.rc.rec_cap; ++r) a.rec_meta[r].slice = kInvalidSlice;
    return;
  }
  if (nrec == 0) return;

  // pass 2: write the records and rank their tiles in the bins
  uint32_t rid = rbase, slot = ibase;
  for (int k = kb; k < ke; ++k) {
    const SliceDev sl = a.slices[k];
    const SpecAxial ax = spec_axial(p[2], c.szz, sl.z, sl.sigma_z);
    if (!exact && !(ax.q <= a.rc.q_cut)) continue;
    SpecRect rect;
    const bool vis = spec_rect(c, p[0], p[1], ax, sl.x0, sl.y0, sl.dx, sl.dy, sl.ntx, sl.nty, a.rc.bbox, rect);
    if (exact) {
      rect.tx0 = 0; rect.tx1 = sl.ntx - 1; rect.ty0 = 0; rect.ty1 = sl.nty - 1;
    } else if (!vis) {
      continue;
    }
    // image quantities (binary32; not part of the membership specification)
    RecPay pay;
    const float B = rect.w * c.sxy - c.a01 * rect.invD;
    const float det = rect.w * c.a22 + c.detS * rect.invD;
    const float rho = expf(-0.5f * ax.q);
    const float at = p[10] * rho / sqrtf(det);
    const float inv_det = 1.0f / det;
    const float ca = rect.C * inv_det, cb = -B * inv_det, cc = rect.A * inv_det;
    pay.x = (rect.mx - sl.x0) / sl.dx - 0.5f;
    pay.y = (rect.my - sl.y0) / sl.dy - 0.5f;
    pay.a = -0.5f * kLog2e * ca * sl.dx * sl.dx;
    pay.b = -kLog2e * cb * sl.dx * sl.dy;
    pay.c = -0.5f * kLog2e * cc * sl.dy * sl.dy;
    pay.w = at;
    const bool good = det > 0.0f && isfinite(at) && isfinite(pay.x) && isfinite(pay.y) && isfinite(pay.a) &&
                      isfinite(pay.b) && isfinite(pay.c);
    if (!good) pay.x = pay.y = pay.a = pay.b = pay.c = pay.w = 0.0f;
    pay.g = exp2f(2.0f * pay.a);
    pay.gid = (uint32_t)j;
    RecMeta meta;
    meta.ibase = slot;
    meta.rx = (uint32_t)rect.tx0 | ((uint32_t)rect.tx1 << 16);
    meta.ry = (uint32_t)rect.ty0 | ((uint32_t)rect.ty1 << 16);
    meta.slice = (uint32_t)k;
    a.rec_pay[rid] = pay;
    a.rec_meta[rid] = meta;
    ++rid;
    for (int ty = rect.ty0; ty <= rect.ty1; ++ty) {
      for (int tx = rect.tx0; tx <= rect.tx1; ++tx, ++slot) {
        const uint32_t bin = (uint32_t)(sl.tile_base + ty * sl.ntx + tx);
        a.inst_rank[slot] = atomicAdd(&a.bin_count[bin], 1u);
      }
    }
  }
}

// Grid-stride over whole wavefronts of flattened Gaussians, so that a launch
// sized for the workspace capacity serves any batch (sizes from the header).
template <int DT>
__global__ __launch_bounds__(256) void k_preprocess(PreArgs a) {
  const int total = a.hdr->total_gauss;
  const int n_groups = a.hdr->n_groups;
  const int stride = gridDim.x * 256;
  for (int t = blockIdx.x * 256 + threadIdx.x; (t & ~63) < total; t += stride) preprocess_one<DT>(a, n_groups, t);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  k_fill_u32<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(p, value, n);
  return hipGetLastError();
}

hipError_t launch_reset(const Workspace& ws, bool clear_overflow, const LaunchDims& d, hipStream_t s) {
  int64_t blocks = (d.bins + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  k_reset<<<(unsigned)blocks, 256, 0, s>>>(ws.d_hdr, ws.d_ctr, ws.d_work, ws.d_bin_count, clear_overflow ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_preprocess(const RenderConst& rc, const Workspace& ws, const LaunchDims& d, hipStream_t s) {
  PreArgs a{rc, ws.d_hdr, ws.d_groups, ws.d_slices, ws.d_ctr, ws.d_bin_count, ws.d_rec_pay, ws.d_rec_meta,
            ws.d_g_rbase, ws.d_g_nrec, ws.d_inst_rank};
  if (d.gauss <= 0) return hipSuccess;
  int64_t blocks = (d.gauss + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  switch (rc.attr_dtype) {
    case GP_BF16: k_preprocess<GP_BF16><<<(unsigned)blocks, 256, 0, s>>>(a); break;
    case GP_F16: k_preprocess<GP_F16><<<(unsigned)blocks, 256, 0, s>>>(a); break;
    default: k_preprocess<GP_F32><<<(unsigned)blocks, 256, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

}  // namespace gp
