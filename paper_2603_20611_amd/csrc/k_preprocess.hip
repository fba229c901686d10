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
// loop visits only those.
//
// Two kernels and a scan, no atomics: k_pre_count counts each Gaussian's
// visible records and footprint tiles (and sums them per wavefront); an
// exclusive scan of the wavefront sums gives every Gaussian contiguous record
// and instance slots in Gaussian order; k_pre_emit writes the records and one
// (bin, record) pair per footprint tile.  Slots are therefore identical from
// run to run.
#include <algorithm>

#include "gp_internal.h"
#include "gp_spec.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace gp {
namespace {



__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = value;
}

// Zeroes the per-forward counters, the work queues and the bin ranges of the
// batch described by the device header (run by every thread of a grid; the
// count does it on its way, the stand-alone kernel for a batch without
// Gaussians).
__device__ __forceinline__ void reset_forward(const BatchHdr* __restrict__ hdr, uint32_t* __restrict__ ctr,
                                              uint32_t* __restrict__ work, uint32_t* __restrict__ bin_lo,
                                              uint32_t* __restrict__ bin_hi, int clear_overflow) {
  const int64_t n = hdr->n_bins;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    ctr[kCtrRecords] = 0u;
    ctr[kCtrInstances] = 0u;
    ctr[kCtrSortEnd] = 0xFFFFFFFFu;
    if (clear_overflow) ctr[kCtrOverflow] = 0u;
  }
  for (int64_t i = t; i < kWorkCount; i += stride) work[i] = 0u;
  for (int64_t i = t; i < n; i += stride) {
    bin_lo[i] = 0u;
    bin_hi[i] = 0u;
  }
}

__global__ void k_reset(const BatchHdr* __restrict__ hdr, uint32_t* __restrict__ ctr, uint32_t* __restrict__ work,
                        uint32_t* __restrict__ bin_lo, uint32_t* __restrict__ bin_hi, int clear_overflow) {
  reset_forward(hdr, ctr, work, bin_lo, bin_hi, clear_overflow);
}

struct PreArgs {
  RenderConst rc;
  const BatchHdr* hdr;
  const GroupDev* groups;
  const SliceDev* slices;
  uint32_t* ctr;
  RecPay* rec_pay;
  RecMeta* rec_meta;
  uint32_t* g_rbase;
  uint32_t* g_nrec;
  uint32_t* g_ninst;
  uint32_t* g_krange;
  uint2* wave_cnt;      // per wavefront (records, instances), or their exclusive scan (scanned)
  uint32_t* inst_key;   // bin of every instance slot
  uint32_t* inst_val;   // record of every instance slot
  uint32_t sentinel_bin;
  const float* poses;   // [n_slices][12] of a posed batch
  int emit_chunk;       // Gaussians per workgroup round of the emit
  int scanned;          // wave_cnt already holds the scan (else the emit forms its bases and the totals)
  uint2* chunk_cnt;     // unscanned: the counts of 512-Gaussian chunks (compacting count), or null
  int count_lg;         // log2 of the lanes per near Gaussian in the compacting count
  // the count's own reset of the forward
  uint32_t* work;
  uint32_t* bin_lo;
  uint32_t* bin_hi;
  int clear_overflow;
};

// (z, sigma_z) of slice k: from the workgroup's LDS copy when there is one
__device__ __forceinline__ float2 slice_zs(const PreArgs& a, const float2* zs, int k) {
  return zs ? zs[k] : make_float2(a.slices[k].z, a.slices[k].sigma_z);
}
__device__ __forceinline__ bool kept_on(const PreArgs& a, const float2* zs, float muz, float szz, int k) {
  const float2 v = slice_zs(a, zs, k);
  const SpecAxial ax = spec_axial(muz, szz, v.x, v.y);
  return ax.q <= a.rc.q_cut;
}

// Kept slices [*kb, *ke) of a Gaussian in a z-sorted, single-sigma_z group.
__device__ __forceinline__ void kept_range(const PreArgs& a, const float2* zs, const GroupDev& G, float muz,
                                           float szz, int* kb, int* ke) {
  // last slice with z <= mu_z (or k0 - 1)
  int lo = G.k0, hi = G.k1 - 1, ks = G.k0 - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    if (slice_zs(a, zs, mid).x <= muz) { ks = mid; lo = mid + 1; } else { hi = mid - 1; }
  }
  // the smallest q is at ks or ks + 1
  int kmin = -1;
  if (ks >= G.k0 && kept_on(a, zs, muz, szz, ks)) kmin = ks;
  else if (ks + 1 < G.k1 && kept_on(a, zs, muz, szz, ks + 1)) kmin = ks + 1;
  if (kmin < 0) { *kb = *ke = G.k0; return; }
  // first kept slice in [k0, kmin] (q non-increasing there)
  lo = G.k0; hi = kmin;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (kept_on(a, zs, muz, szz, mid)) hi = mid; else lo = mid + 1;
  }
  *kb = lo;
  // last kept slice in [kmin, k1) (q non-decreasing there)
  lo = kmin; hi = G.k1 - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (kept_on(a, zs, muz, szz, mid)) lo = mid; else hi = mid - 1;
  }
  *ke = lo + 1;
}

// Parameters of coded Gaussian j (GP_QM): 11 uint16 code planes and the
// 9-float header (lo[3], hi[3], lmin, lmax, amax); the decoding of the codec, in
// binary32 without contraction.
__device__ __forceinline__ void decode_codes(const uint16_t* __restrict__ c, const float* __restrict__ h,
                                             int64_t stride, int64_t j, float* p) {
#pragma clang fp contract(off)
#pragma unroll
  for (int a = 0; a < 3; ++a) p[a] = h[a] + (float)c[a * stride + j] * ((h[3 + a] - h[a]) / 16383.0f);
#pragma unroll
  for (int a = 0; a < 3; ++a) p[3 + a] = h[6] + (float)c[(3 + a) * stride + j] * ((h[7] - h[6]) / 4095.0f);
#pragma unroll
  for (int r = 0; r < 4; ++r) p[6 + r] = (float)c[(6 + r) * stride + j] * (2.0f / 4095.0f) - 1.0f;
  p[10] = 0.0f + (float)c[10 * stride + j] * (h[8] / 4095.0f);
}

struct Loaded {
  GroupDev G;
  int j;
  float p[11];
  SpecCov c;
  bool ok;
};

// Parameters of flattened Gaussian t (L.ok: in range and all finite).
template <int DT>
__device__ __forceinline__ void load_params(const PreArgs& a, int n_groups, int t, Loaded& L) {
  const int wave0 = t & ~63;
  const int g = group_of(a.groups, n_groups, wave0);
  L.G = a.groups[g];
  L.j = t - L.G.gbase;
  const bool in_range = L.j < L.G.n;
  if (in_range) {
    if constexpr (DT == GP_QM) {
      decode_codes(reinterpret_cast<const uint16_t*>(L.G.means), static_cast<const float*>(L.G.attrs), L.G.stride,
                   L.j, L.p);
    } else {
      L.p[0] = L.G.means[L.j];
      L.p[1] = L.G.means[L.G.stride + L.j];
      L.p[2] = L.G.means[2 * L.G.stride + L.j];
#pragma unroll
      for (int r = 0; r < 8; ++r) L.p[3 + r] = load_attr<DT>(L.G.attrs, r, L.G.stride, L.j);
    }
  } else {
#pragma unroll
    for (int r = 0; r < 11; ++r) L.p[r] = 0.0f;
  }
  bool finite = in_range;
#pragma unroll
  for (int r = 0; r < 11; ++r) finite = finite && isfinite(L.p[r]);
  L.ok = finite;
}

__device__ __forceinline__ void activate(const PreArgs& a, Loaded& L) {
  spec_cov(L.p[3], L.p[4], L.p[5], L.p[6], L.p[7], L.p[8], L.p[9], a.rc.scale_mod, L.c);
  L.ok = L.ok && (L.c.n2 > 0.0f);
}

// Footprint of (Gaussian, slice k) from its camera-frame view (cv, mv); false
// if the pair is culled or off-grid.
__device__ __forceinline__ bool footprint(const PreArgs& a, const SpecCov& cv, const float* mv, int k,
                                          SpecAxial& ax, SpecRect& rect) {
  const SliceDev& sl = a.slices[k];
  const bool exact = (a.rc.flags & GP_FLAG_EXACT) != 0;
  ax = spec_axial(mv[2], cv.szz, sl.z, sl.sigma_z);
  if (!exact && !(ax.q <= a.rc.q_cut)) return false;
  const bool vis = spec_rect(cv, mv[0], mv[1], ax, sl.x0, sl.y0, sl.dx, sl.dy, sl.ntx, sl.nty, a.rc.bbox, rect);
  if (exact) {
    rect.tx0 = 0; rect.tx1 = sl.ntx - 1; rect.ty0 = 0; rect.ty1 = sl.nty - 1;
    return true;
  }
  return vis;
}

// The slice fields the footprint reads, loaded into registers.
struct SliceGeo {
  float z, sigma_z, x0, y0, dx, dy;
  int32_t ntx, nty;
};
__device__ __forceinline__ SliceGeo slice_geo(const SliceDev& sl) {
  return SliceGeo{sl.z, sl.sigma_z, sl.x0, sl.y0, sl.dx, sl.dy, sl.ntx, sl.nty};
}

// footprint() of an axial slice (the world-frame covariance c for every
// slice) with the sigma_z part reused from the previous slice of the same
// sigma_z (g, valid for the bits `key` of sigma_z^2 once `have`).
__device__ __forceinline__ bool footprint_axial(const PreArgs& a, const SpecCov& c, const float* mv,
                                                const SliceGeo& sl, SpecAxial& ax, SpecRect& rect, SpecSigma& g,
                                                uint32_t& key, bool& have) {
  const bool exact = (a.rc.flags & GP_FLAG_EXACT) != 0;
  ax = spec_axial(mv[2], c.szz, sl.z, sl.sigma_z);
  if (!exact && !(ax.q <= a.rc.q_cut)) return false;
  const uint32_t kb = __float_as_uint(ax.s2);
  if (!have || kb != key) {
    g = spec_sigma(c, ax, a.rc.bbox);
    key = kb;
    have = true;
  }
  const bool vis = spec_rect_from(g, mv[0], mv[1], ax, sl.x0, sl.y0, sl.dx, sl.dy, sl.ntx, sl.nty, rect);
  if (exact) {
    rect.tx0 = 0; rect.tx1 = sl.ntx - 1; rect.ty0 = 0; rect.ty1 = sl.nty - 1;
    return true;
  }
  return vis;
}

// Conservative axial pre-test on the raw parameters: true only if no slice of
// the group can keep the Gaussian.  Sigma_zz <= max_i s_i^2, so with d the
// distance of mu_z from the group's depth range, d^2 > q_cut (sigma_z,max^2 +
// max_i s_i^2) implies q_ax > q_cut on every slice; the 1e-3 margin covers
// the rounding of the specified binary32 test.  Saves the covariance of
// Gaussians far from every slice (most of them, for a few slices of a deep
// volume).
__device__ __forceinline__ bool far_from_group(const PreArgs& a, const GroupDev& G, const float* p) {
  if (a.rc.flags & GP_FLAG_EXACT) return false;
  const float lmax = fmaxf(p[3], fmaxf(p[4], p[5]));
  const float smax = exp_spec(lmax) * a.rc.scale_mod;
  const float d = fmaxf(fmaxf(G.zlo - p[2], p[2] - G.zhi), 0.0f);
  return d * d > a.rc.q_cut * (G.sz2max + smax * smax) * 1.001f;
}

// Whether flattened Gaussian t may have records on its group's slices: in
// range and not far_from_group(), from its depth and log-scales only (the
// compacting count's first look at every Gaussian; a near one is loaded whole
// and checked afterwards, so a non-finite parameter elsewhere still culls it).
template <int DT>
__device__ __forceinline__ bool maybe_near(const PreArgs& a, int n_groups, int t) {
  if constexpr (DT == GP_QM) {
    Loaded L;
    load_params<DT>(a, n_groups, t, L);
    return L.ok && !far_from_group(a, L.G, L.p);
  } else {
    const int wave0 = t & ~63;
    const int g = group_of(a.groups, n_groups, wave0);
    const GroupDev& G = a.groups[g];
    const int j = t - G.gbase;
    if (j >= G.n) return false;
    float p[6];
    p[2] = G.means[2 * G.stride + j];
    p[3] = load_attr<DT>(G.attrs, 0, G.stride, j);
    p[4] = load_attr<DT>(G.attrs, 1, G.stride, j);
    p[5] = load_attr<DT>(G.attrs, 2, G.stride, j);
    return !far_from_group(a, G, p);
  }
}

// far_from_group() for a group whose slices share one camera pose: the same
// test on the mean's depth in that camera frame (the operations of the
// specified pose transform, so the same bits as the per-slice view) against
// the group's camera-frame depth range; the camera-frame Sigma_zz is bounded by
// max_i s_i^2 as in the world frame (a rotation keeps the eigenvalues).
__device__ __forceinline__ bool far_from_pose(const PreArgs& a, const GroupDev& G, const float* p) {
#pragma clang fp contract(off)
  if (a.rc.flags & GP_FLAG_EXACT) return false;
  const float* P = a.poses + 12 * G.k0;
  const float mz = ((P[6] * p[0] + P[7] * p[1]) + P[8] * p[2]) + P[11];
  const float lmax = fmaxf(p[3], fmaxf(p[4], p[5]));
  const float smax = exp_spec(lmax) * a.rc.scale_mod;
  const float d = fmaxf(fmaxf(G.zlo - mz, mz - G.zhi), 0.0f);
  return d * d > a.rc.q_cut * (G.sz2max + smax * smax) * 1.001f;
}

// Records and list entries of Gaussian L on its slices (L loaded; L.ok false
// for a Gaussian culled on every slice); *kr receives its kept slice range.
template <bool POSED>
__device__ __forceinline__ void count_slices(const PreArgs& a, const float2* zs, Loaded& L, uint32_t* nrec_out,
                                             uint32_t* ninst_out, uint32_t* kr) {
  int kb = L.G.k0, ke = L.G.k1;
  if (!L.ok) {
    ke = kb;
  } else if (!POSED && !(a.rc.flags & GP_FLAG_EXACT) && (L.G.flags & kGroupSortedZ)) {
    kept_range(a, zs, L.G, L.p[2], L.c.szz, &kb, &ke);
  }
  uint32_t nrec = 0, ninst = 0;
  if constexpr (POSED) {
    if (L.G.flags & kGroupSharedPose) {
      // one camera frame for the group: its view once, and with sorted depths
      // the kept range by binary search, as for axial slices (the emit's view
      // of every slice is the same bits)
      SpecCov cv;
      float mv[3];
      spec_pose(L.c, L.p, a.poses + 12 * L.G.k0, cv, mv);
      if (kb < ke && !(a.rc.flags & GP_FLAG_EXACT) && (L.G.flags & kGroupSortedZ))
        kept_range(a, zs, L.G, mv[2], cv.szz, &kb, &ke);
      // the sigma_z part of the footprint once per sigma_z, as for axial slices
      SpecSigma sg;
      uint32_t sg_key = 0u;
      bool sg_have = false;
      for (int k = kb; k < ke; ++k) {
        SpecAxial ax;
        SpecRect rect;
        if (!footprint_axial(a, cv, mv, slice_geo(a.slices[k]), ax, rect, sg, sg_key, sg_have)) continue;
        nrec += 1u;
        ninst += (uint32_t)((rect.tx1 - rect.tx0 + 1) * (rect.ty1 - rect.ty0 + 1));
      }
    } else {
      for (int k = kb; k < ke; ++k) {
        // the Gaussian in the slice's camera frame
        SpecAxial ax;
        SpecRect rect;
        SpecCov cv;
        float mv[3];
        spec_pose(L.c, L.p, a.poses + 12 * k, cv, mv);
        if (!footprint(a, cv, mv, k, ax, rect)) continue;
        nrec += 1u;
        ninst += (uint32_t)((rect.tx1 - rect.tx0 + 1) * (rect.ty1 - rect.ty0 + 1));
      }
    }
  } else {
    // the next slice's fields are in flight while this slice is tested
    SpecSigma sg;
    uint32_t sg_key = 0u;
    bool sg_have = false;
    SliceGeo cur{};
    if (kb < ke) cur = slice_geo(a.slices[kb]);
    for (int k = kb; k < ke; ++k) {
      SliceGeo nxt = cur;
      if (k + 1 < ke) nxt = slice_geo(a.slices[k + 1]);
      SpecAxial ax;
      SpecRect rect;
      if (footprint_axial(a, L.c, L.p, cur, ax, rect, sg, sg_key, sg_have)) {
        nrec += 1u;
        ninst += (uint32_t)((rect.tx1 - rect.tx0 + 1) * (rect.ty1 - rect.ty0 + 1));
      }
      cur = nxt;
    }
  }
  *nrec_out = nrec;
  *ninst_out = ninst;
  *kr = (uint32_t)kb | ((uint32_t)ke << 16);
}

// count_slices() of an axial Gaussian by 2^lg lanes together: lane li of the
// group tests slices kb + li, kb + li + 2^lg, ...; the sums are formed across
// the group (every lane of the wavefront takes part, `active` false for lanes
// without a Gaussian).  Integer sums: the same values as one lane's loop.
__device__ __forceinline__ void count_slices_lanes(const PreArgs& a, const float2* zs, Loaded& L, bool active,
                                                   int lg, uint32_t* nrec_out, uint32_t* ninst_out, uint32_t* kr) {
  const int cl = 1 << lg, li = (int)(threadIdx.x & (cl - 1));
  int kb = L.G.k0, ke = L.G.k1;
  if (!active || !L.ok) {
    ke = kb;
  } else if (!(a.rc.flags & GP_FLAG_EXACT) && (L.G.flags & kGroupSortedZ)) {
    kept_range(a, zs, L.G, L.p[2], L.c.szz, &kb, &ke);
  }
  uint32_t nrec = 0, ninst = 0;
  SpecSigma sg;
  uint32_t sg_key = 0u;
  bool sg_have = false;
  for (int k = kb + li; k < ke; k += cl) {
    const SliceGeo geo = slice_geo(a.slices[k]);
    SpecAxial ax;
    SpecRect rect;
    if (footprint_axial(a, L.c, L.p, geo, ax, rect, sg, sg_key, sg_have)) {
      nrec += 1u;
      ninst += (uint32_t)((rect.tx1 - rect.tx0 + 1) * (rect.ty1 - rect.ty0 + 1));
    }
  }
  for (int o = 1; o < cl; o <<= 1) {
    nrec += __shfl_xor(nrec, o, 64);
    ninst += __shfl_xor(ninst, o, 64);
  }
  *nrec_out = nrec;
  *ninst_out = ninst;
  *kr = (uint32_t)kb | ((uint32_t)ke << 16);
}

// Per-Gaussian outputs of the count and the wavefront's sums (whole wavefronts).
__device__ __forceinline__ void count_store(const PreArgs& a, int t, uint32_t nrec, uint32_t ninst, uint32_t kr) {
  a.g_nrec[t] = nrec;
  a.g_ninst[t] = ninst;
  a.g_krange[t] = kr;
  uint32_t sr = nrec, si = ninst;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    sr += __shfl_xor(sr, o, 64);
    si += __shfl_xor(si, o, 64);
  }
  if ((t & 63) == 0) a.wave_cnt[t >> 6] = make_uint2(sr, si);
}

template <int DT, bool POSED>
__device__ __forceinline__ void count_one(const PreArgs& a, const float2* zs, int n_groups, int t) {
  Loaded L;
  load_params<DT>(a, n_groups, t, L);
  // the world-depth shortcuts hold for axial slices, and in the camera frame
  // for a group of slices sharing one pose
  bool far = false;
  if (L.ok) {
    if (!POSED) far = far_from_group(a, L.G, L.p);
    else if (L.G.flags & kGroupSharedPose) far = far_from_pose(a, L.G, L.p);
  }
  if (far) L.ok = false;   // culled on every slice
  else activate(a, L);
  uint32_t nrec, ninst, kr;
  count_slices<POSED>(a, zs, L, &nrec, &ninst, &kr);
  count_store(a, t, nrec, ninst, kr);
}

// Float64 covariance of a Gaussian from its binary32 parameters (rotation of
// the quaternion normalised in float64; the scales are the specification's
// binary32 exp, whose error moves an eigenvalue, not the conditioning), as
// Sigma = v1 I + (v0 - v1) r0 r0^T + (v2 - v1) r2 r2^T with r0, r2 the first
// and last columns of R.  out: xx, xy, xz, yy, yz, zz.
__device__ __forceinline__ void cov_f64(const float* p, float mod, double* out) {
#pragma clang fp contract(off)
  const double qw = p[6], qx = p[7], qy = p[8], qz = p[9];
  const double rn = 1.0 / sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
  const double w = qw * rn, x = qx * rn, y = qy * rn, z = qz * rn;
  const float s0 = exp_spec(p[3]) * mod, s1 = exp_spec(p[4]) * mod, s2 = exp_spec(p[5]) * mod;
  const double v0 = (double)s0 * (double)s0, v1 = (double)s1 * (double)s1, v2 = (double)s2 * (double)s2;
  const double r0[3] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y)};
  const double r2[3] = {2.0 * (x * z + w * y), 2.0 * (y * z - w * x), 1.0 - 2.0 * (x * x + y * y)};
  const double d0 = v0 - v1, d2 = v2 - v1;
  out[0] = (v1 + d0 * r0[0] * r0[0]) + d2 * r2[0] * r2[0];
  out[1] = d0 * r0[0] * r0[1] + d2 * r2[0] * r2[1];
  out[2] = d0 * r0[0] * r0[2] + d2 * r2[0] * r2[2];
  out[3] = (v1 + d0 * r0[1] * r0[1]) + d2 * r2[1] * r2[1];
  out[4] = d0 * r0[1] * r0[2] + d2 * r2[1] * r2[2];
  out[5] = (v1 + d0 * r0[2] * r0[2]) + d2 * r2[2] * r2[2];
}

// Image quantities of a kept (Gaussian, slice) pair, not part of the membership
// specification: computed in float64 from the Gaussian's float64 covariance
// and binary32 mean and intensity, rounded once.  A thin, elongated Gaussian
// makes Sigma_2d ill-conditioned, and its conic taken from binary32
// covariance entries would be off by ~1e-5 of the record's peak; the
// pixel-space mean at large pixel coordinates likewise.  Every operation runs
// in a fixed order (no contraction), so that equal inputs give equal records
// in every instantiation of the emit.
//
// RecSigma is the part that depends on the slice only through sigma_z (the
// conditioned 2D covariance, its determinant and the conic up to the pixel
// pitch): equal for every slice of one sigma_z, so the emit forms it once
// per Gaussian and reuses it on its slices.  sdet is sqrt(det) in binary32,
// NaN when det is not positive (the record is then zeroed, as any non-finite
// one); conv the exact convolution's factor.
struct RecSigma {
  double invD, u, v, ta, tb, tc;
  float sdet, conv;
};

// cov: xx, xy, xz, yy, yz, zz (in the slice's frame); sc0, sc1, sc2: the activated scales.
__device__ __forceinline__ RecSigma rec_sigma(const double* cov, float sc0, float sc1, float sc2, float sigma_z,
                                              uint32_t flags) {
#pragma clang fp contract(off)
  const double sxx = cov[0], sxy = cov[1], sxz = cov[2], syy = cov[3], syz = cov[4], szz = cov[5];
  const double s2 = (double)sigma_z * (double)sigma_z;
  RecSigma r;
  r.invD = 1.0 / (s2 + szz);          // 0 for sigma_z = inf
  r.u = sxz * r.invD;
  r.v = syz * r.invD;
  const double A = sxx - r.u * sxz, B = sxy - r.u * syz, C = syy - r.v * syz;
  const double det = A * C - B * B;
  const double inv_det = 1.0 / det;
  const double L2 = 1.4426950408889634;
  r.ta = -0.5 * L2 * C * inv_det;
  r.tb = L2 * B * inv_det;
  r.tc = -0.5 * L2 * A * inv_det;
  r.sdet = det > 0.0 ? sqrtf((float)det) : __builtin_nanf("");
  r.conv = 1.0f;
  // exact convolution integral: times sqrt(2 pi det Sigma_e), det Sigma_e = det Sigma w
  if (flags & GP_FLAG_CONV_EXACT) {
    const double v0 = (double)sc0 * (double)sc0, v1 = (double)sc1 * (double)sc1, v2 = (double)sc2 * (double)sc2;
    r.conv = sqrtf((float)(6.283185307179586 * ((v0 * v1) * v2) / (1.0 + szz / s2)));
  }
  return r;
}

// The record of a Gaussian with mean mu (slice frame) and intensity on slice sl.
__device__ __forceinline__ void rec_pay(const RecSigma& r, double mx, double my, double mz, float inten,
                                        const SliceDev& sl, uint32_t flags, RecPay& pay) {
#pragma clang fp contract(off)
  const double m = mz - (double)sl.z;
  const float rho = expf(-0.5f * (float)(m * m * r.invD));
  float at = inten * rho / r.sdet;
  if (flags & GP_FLAG_CONV_EXACT) at *= r.conv;
  // pixel-index mean as a binary32 anchor (nearest integer) plus remainder
  const double px = (((mx - r.u * m) - (double)sl.x0) / (double)sl.dx) - 0.5;
  const double py = (((my - r.v * m) - (double)sl.y0) / (double)sl.dy) - 0.5;
  pay.ax = (float)rint(px);
  pay.ay = (float)rint(py);
  pay.xr = (float)(px - (double)pay.ax);
  pay.yr = (float)(py - (double)pay.ay);
  pay.a = (float)(r.ta * (double)sl.dx * (double)sl.dx);
  pay.b = (float)(r.tb * (double)sl.dx * (double)sl.dy);
  pay.c = (float)(r.tc * (double)sl.dy * (double)sl.dy);
  pay.w = at;
  const bool good = isfinite(at) && isfinite(pay.ax) && isfinite(pay.ay) && isfinite(pay.xr) && isfinite(pay.yr) &&
                    isfinite(pay.a) && isfinite(pay.b) && isfinite(pay.c);
  if (!good) pay.xr = pay.yr = pay.ax = pay.ay = pay.a = pay.b = pay.c = pay.w = 0.0f;
}

__device__ __forceinline__ RecMeta rec_meta(uint32_t ibase, const SpecRect& rect, int k) {
  RecMeta meta;
  meta.ibase = ibase;
  meta.rx = (uint32_t)rect.tx0 | ((uint32_t)rect.tx1 << 16);
  meta.ry = (uint32_t)rect.ty0 | ((uint32_t)rect.ty1 << 16);
  meta.slice = (uint32_t)k;
  return meta;
}

// The record of (Gaussian, slice k) from its world covariance (cov), binary32
// parameters p and activated scales c.  pose: the slice's camera pose
// (Sigma_c = R_c Sigma R_c^T, mu_c = R_c mu + t) or nullptr.
__device__ __forceinline__ void make_record(const double* cov, const float* p, const SpecCov& c, const float* pose,
                                            const SliceDev& sl, uint32_t flags, RecPay& pay) {
#pragma clang fp contract(off)
  double mu[3] = {p[0], p[1], p[2]};
  double cv[6] = {cov[0], cov[1], cov[2], cov[3], cov[4], cov[5]};
  if (pose) {
    const double S[3][3] = {{cov[0], cov[1], cov[2]}, {cov[1], cov[3], cov[4]}, {cov[2], cov[4], cov[5]}};
    double T[3][3], mc[3];   // T = R_c Sigma
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int j = 0; j < 3; ++j)
        T[i][j] = ((double)pose[3 * i] * S[0][j] + (double)pose[3 * i + 1] * S[1][j]) + (double)pose[3 * i + 2] * S[2][j];
      mc[i] = (((double)pose[3 * i] * mu[0] + (double)pose[3 * i + 1] * mu[1]) + (double)pose[3 * i + 2] * mu[2]) +
              (double)pose[9 + i];
    }
    auto E = [&](int i, int j) {
      return (T[i][0] * (double)pose[3 * j] + T[i][1] * (double)pose[3 * j + 1]) + T[i][2] * (double)pose[3 * j + 2];
    };
    cv[0] = E(0, 0); cv[1] = E(0, 1); cv[2] = E(0, 2); cv[3] = E(1, 1); cv[4] = E(1, 2); cv[5] = E(2, 2);
    mu[0] = mc[0]; mu[1] = mc[1]; mu[2] = mc[2];
  }
  rec_pay(rec_sigma(cv, c.s0, c.s1, c.s2, sl.sigma_z, flags), mu[0], mu[1], mu[2], p[10], sl, flags, pay);
}

// Slots of the 64 consecutive Gaussians t0 .. t0 + 63 of one wavefront.
//
// Record and instance slots come from an exclusive scan over the wavefront
// (plus the wavefront's base), so the wavefront's output is one contiguous
// range of records and one of instances, in Gaussian order: g_rbase and
// g_ninst (overwritten with the instance base) receive them.  Gaussians that
// have records are appended to the workgroup's list in LDS (in any order:
// every output position is fixed by the scan).
__device__ __forceinline__ void slots_wave(const PreArgs& a, int t0, uint2 wb, int* list, int* n_list) {
  const int lane = threadIdx.x & 63;
  const int t = t0 + lane;
  uint32_t nrec = a.g_nrec[t];
  const uint32_t ninst = a.g_ninst[t];
  uint32_t pr = nrec, pi = ninst;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t ur = __shfl_up(pr, d, 64), ui = __shfl_up(pi, d, 64);
    if (lane >= d) { pr += ur; pi += ui; }
  }
  const uint32_t rbase = wb.x + pr - nrec, ibase = wb.y + pi - ninst;
  const bool fits = (uint64_t)rbase + nrec <= a.rc.rec_cap && (uint64_t)ibase + ninst <= a.rc.inst_cap;
  a.g_rbase[t] = rbase;
  a.g_ninst[t] = ibase;
  if (!fits) {
    // overflow: this Gaussian's slots inside the capacity stay unused and are
    // marked so that no later kernel reads them; the sort ends before the
    // first of them
    a.ctr[kCtrOverflow] = 1u;
    atomicMin(&a.ctr[kCtrSortEnd], ibase);
    a.g_nrec[t] = 0u;
    if (!(a.rc.flags & GP_FLAG_FORWARD_ONLY))
      for (uint32_t r = rbase; r < rbase + nrec && r < a.rc.rec_cap; ++r) a.rec_meta[r].slice = kInvalidSlice;
    for (uint32_t s = ibase; s < ibase + ninst && s < a.rc.inst_cap; ++s) a.inst_key[s] = a.sentinel_bin;
    nrec = 0u;
  }
  const uint64_t m = __ballot(nrec > 0u);
  int base = 0;
  if (lane == 0 && m) base = atomicAdd(n_list, __popcll(m));
  base = __shfl(base, 0, 64);
  if (nrec > 0u) list[base + __popcll(m & ((1ull << lane) - 1ull))] = t;
}

// Emit of 64 consecutive entries j0 .. j0 + 63 of the workgroup's list of
// Gaussians with records, by one wavefront: W lanes cooperate on one Gaussian.  Lane i of the group takes
// slices kb + i, kb + i + W, ... of its kept window, and the group's kept slices
// are compacted with a ballot, so consecutive lanes write consecutive records
// and adjacent instance runs.  (With one lane per Gaussian and many slices per
// Gaussian, every lane would stream to its own region and L2 would evict
// partly written lines.)  W = 1 is the one-lane form, used when each Gaussian
// has at most one slice.  Each lane first forms what the records of its own
// entry's Gaussian share into LDS, once for all of them: for axial slices the
// sigma_z parts of the footprint and of the record (RecSigma), for posed ones
// the float64 world covariance.
// What the emit needs of an activated Gaussian: the mean, the intensity, the
// scales and Sigma_zz, and the sigma_z part of its footprint (the u, v, rx, ry
// of SpecSigma) for the sigma_z of its first kept slice (key: the bits of that
// sigma_z).
struct EmitGauss {
  float mx, my, mz, inten, s0, s1, s2, szz;
  uint32_t key;
  float gu, gv, grx, gry;
};

// footprint() of an axial slice for the emit: the stored sigma_z part when the
// slice's sigma_z is the key's, else computed from the reloaded Gaussian t.
// With POSED, e holds the Gaussian in the camera frame its group's slices share
// (the reload takes the same view).
template <int DT, bool POSED>
__device__ __forceinline__ bool footprint_emit(const PreArgs& a, int n_groups, int t, const EmitGauss& e, int k,
                                               SpecAxial& ax, SpecRect& rect) {
  const SliceDev& sl = a.slices[k];
  const bool exact = (a.rc.flags & GP_FLAG_EXACT) != 0;
  ax = spec_axial(e.mz, e.szz, sl.z, sl.sigma_z);
  if (!exact && !(ax.q <= a.rc.q_cut)) return false;
  // (the rectangle reads only u, v, rx and ry)
  SpecSigma g{0.0f, 0.0f, 0.0f, 0.0f, e.gu, e.gv, e.grx, e.gry};
  if (__float_as_uint(sl.sigma_z) != e.key) {
    Loaded L;
    load_params<DT>(a, n_groups, t, L);
    activate(a, L);
    if constexpr (POSED) {
      SpecCov cv;
      float mv[3];
      spec_pose(L.c, L.p, a.poses + 12 * k, cv, mv);
      g = spec_sigma(cv, ax, a.rc.bbox);
    } else {
      g = spec_sigma(L.c, ax, a.rc.bbox);
    }
  }
  const bool vis = spec_rect_from(g, e.mx, e.my, ax, sl.x0, sl.y0, sl.dx, sl.dy, sl.ntx, sl.nty, rect);
  if (exact) {
    rect.tx0 = 0; rect.tx1 = sl.ntx - 1; rect.ty0 = 0; rect.ty1 = sl.nty - 1;
    return true;
  }
  return vis;
}

// Instances a group of W lanes stages in LDS per slice round before writing
// them out as one run (consecutive lanes, consecutive slots; each lane's own
// loop over its tiles left a wavefront's stores scattered over 64 places); a
// round with more goes out directly.  400-slice stack: emit 0.232 -> 0.224 ms.
constexpr int kStagePerLane = 4;

template <int DT, int W, bool POSED>
__device__ __forceinline__ void emit_wave(const PreArgs& a, int n_groups, const int* list, uint32_t j0,
                                          uint32_t n_active, double (*cov64)[6], RecSigma* rsg, EmitGauss* eg,
                                          float4* pw, uint2* stage) {
  const int lane = threadIdx.x & 63;
  const uint32_t j = j0 + (uint32_t)lane;
  const int t = j < n_active ? list[j] : 0;
  uint32_t rbase = 0u, ibase = 0u, krange = 0u;
  if (j < n_active) {
    rbase = a.g_rbase[t];
    ibase = a.g_ninst[t];
    krange = a.g_krange[t];
    Loaded Lq;
    load_params<DT>(a, n_groups, t, Lq);
    if (!POSED) {
      double cw[6];
      cov_f64(Lq.p, a.rc.scale_mod, cw);
      activate(a, Lq);
      const SpecCov& c = Lq.c;
      const SliceDev& s0 = a.slices[krange & 0xFFFFu];   // the first kept slice
      const SpecAxial ax0 = spec_axial(Lq.p[2], c.szz, s0.z, s0.sigma_z);
      const SpecSigma g0 = spec_sigma(c, ax0, a.rc.bbox);
      eg[lane] = EmitGauss{Lq.p[0], Lq.p[1], Lq.p[2], Lq.p[10], c.s0, c.s1, c.s2, c.szz,
                           __float_as_uint(s0.sigma_z), g0.u, g0.v, g0.rx, g0.ry};
      rsg[lane] = rec_sigma(cw, c.s0, c.s1, c.s2, s0.sigma_z, a.rc.flags);
    } else {
      cov_f64(Lq.p, a.rc.scale_mod, cov64[lane]);
      // slices sharing one pose: the Gaussian's view in that camera frame,
      // kept like an axial Gaussian's (the world mean for the record)
      const bool sh = (Lq.G.flags & kGroupSharedPose) != 0;
      pw[lane] = make_float4(Lq.p[0], Lq.p[1], Lq.p[2], sh ? 1.0f : 0.0f);
      if (sh) {
        activate(a, Lq);
        SpecCov cv;
        float mv[3];
        spec_pose(Lq.c, Lq.p, a.poses + 12 * Lq.G.k0, cv, mv);
        const SliceDev& s0 = a.slices[krange & 0xFFFFu];
        const SpecAxial ax0 = spec_axial(mv[2], cv.szz, s0.z, s0.sigma_z);
        const SpecSigma g0 = spec_sigma(cv, ax0, a.rc.bbox);
        eg[lane] = EmitGauss{mv[0], mv[1], mv[2], Lq.p[10], cv.s0, cv.s1, cv.s2, cv.szz,
                             __float_as_uint(s0.sigma_z), g0.u, g0.v, g0.rx, g0.ry};
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int sub = lane / W, li = lane % W;
  for (int it = 0; it < W; ++it) {
    // 64 / W groups per round, W rounds: entry gi of the 64.  Every lane takes
    // part in the exchanges; divergence starts after them.
    const int gi = it * (64 / W) + sub;
    const int tg = __shfl(t, gi, 64);
    const uint32_t g_rb = __shfl(rbase, gi, 64);
    const uint32_t g_ib = __shfl(ibase, gi, 64);
    const uint32_t g_kr = __shfl(krange, gi, 64);
    if (j0 + (uint32_t)gi >= n_active) continue;
    Loaded L;
    EmitGauss e{};
    bool shared_view = false;
    if constexpr (POSED) {
      const float4 w4 = pw[gi];
      shared_view = w4.w != 0.0f;
      if (shared_view) {
        // the camera-frame view its entry's lane formed; the record takes the
        // world mean, the intensity and the scales
        e = eg[gi];
#pragma unroll
        for (int r = 0; r < 11; ++r) L.p[r] = 0.0f;
        L.p[0] = w4.x;
        L.p[1] = w4.y;
        L.p[2] = w4.z;
        L.p[10] = e.inten;
        L.c = SpecCov{};
        L.c.s0 = e.s0;
        L.c.s1 = e.s1;
        L.c.s2 = e.s2;
      } else {
        load_params<DT>(a, n_groups, tg, L);
        activate(a, L);
      }
    } else {
      // the group's Gaussian as its entry's lane activated it (the same values)
      e = eg[gi];
    }
    const int kb = (int)(g_kr & 0xFFFFu), ke = (int)(g_kr >> 16);
    uint32_t rec_run = g_rb, inst_run = g_ib;
    for (int c0 = kb; c0 < ke; c0 += W) {
      const int k = c0 + li;
      SpecAxial ax;
      SpecRect rect;
      SpecCov cv;
      float mv[3];
      bool kept = false;
      if constexpr (POSED) {
        if (k < ke) {
          if (shared_view) {
            kept = footprint_emit<DT, true>(a, n_groups, tg, e, k, ax, rect);
          } else {
            spec_pose(L.c, L.p, a.poses + 12 * k, cv, mv);
            kept = footprint(a, cv, mv, k, ax, rect);
          }
        }
      } else {
        kept = k < ke && footprint_emit<DT, false>(a, n_groups, tg, e, k, ax, rect);
      }
      const uint32_t nt = kept ? (uint32_t)((rect.tx1 - rect.tx0 + 1) * (rect.ty1 - rect.ty0 + 1)) : 0u;
      uint32_t rpos = 0u, ipos = 0u, rtot = 1u, itot = nt;
      if (W > 1) {
        const uint64_t m = __ballot(kept);
        const uint32_t gm = (uint32_t)(m >> (sub * W)) & (uint32_t)((1ull << W) - 1ull);
        rpos = (uint32_t)__popc(gm & ((1u << li) - 1u));
        rtot = (uint32_t)__popc(gm);
        uint32_t inc = nt;
#pragma unroll
        for (int d = 1; d < W; d <<= 1) {
          const uint32_t u = __shfl_up(inc, d, W);
          if (li >= d) inc += u;
        }
        ipos = inc - nt;
        itot = __shfl(inc, W - 1, W);
      }
      // uniform over the group of W lanes
      const bool staged = W >= 8 && itot <= (uint32_t)(kStagePerLane * W);
      if (kept) {
        const SliceDev& sl = a.slices[k];
        const uint32_t rid = rec_run + rpos;
        uint32_t slot = inst_run + ipos;
        RecPay pay;
        if constexpr (POSED) {
          make_record(cov64[gi], L.p, L.c, a.poses + 12 * k, sl, a.rc.flags, pay);
        } else {
          RecSigma r;
          if (__float_as_uint(sl.sigma_z) == e.key) {
            r = rsg[gi];
          } else {
            // another sigma_z: the float64 covariance again, from the reloaded parameters
            Loaded Lr;
            load_params<DT>(a, n_groups, tg, Lr);
            double cw[6];
            cov_f64(Lr.p, a.rc.scale_mod, cw);
            r = rec_sigma(cw, e.s0, e.s1, e.s2, sl.sigma_z, a.rc.flags);
          }
          rec_pay(r, (double)e.mx, (double)e.my, (double)e.mz, e.inten, sl, a.rc.flags, pay);
        }
        a.rec_pay[rid] = pay;
        if (!(a.rc.flags & GP_FLAG_FORWARD_ONLY)) a.rec_meta[rid] = rec_meta(slot, rect, k);
        if (!staged) {
          for (int ty = rect.ty0; ty <= rect.ty1; ++ty) {
            for (int tx = rect.tx0; tx <= rect.tx1; ++tx, ++slot) {
              a.inst_key[slot] = (uint32_t)(sl.tile_base + ty * sl.ntx + tx);
              a.inst_val[slot] = rid;
            }
          }
        } else {
          uint2* st = stage + sub * (kStagePerLane * W) + ipos;
          for (int ty = rect.ty0; ty <= rect.ty1; ++ty)
            for (int tx = rect.tx0; tx <= rect.tx1; ++tx, ++st) *st = make_uint2((uint32_t)(sl.tile_base + ty * sl.ntx + tx), rid);
        }
      }
      if (staged) {
        // the group's instances of this round, consecutive lanes to consecutive slots
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint2* st = stage + sub * (kStagePerLane * W);
        for (uint32_t q = (uint32_t)li; q < itot; q += W) {
          const uint2 v = st[q];
          a.inst_key[inst_run + q] = v.x;
          a.inst_val[inst_run + q] = v.y;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      if (W > 1) {
        rec_run += rtot;
        inst_run += itot;
      } else if (kept) {
        rec_run += 1u;
        inst_run += nt;
      }
    }
  }
  // the wavefront's LDS slots are rewritten by its next round
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The (records, instances) counts cnt[0 .. n) added up by the workgroup's
// 256 threads (every thread gets the sum; integer sums, so the order does not
// matter).  With the counts unscanned, each workgroup of the emit forms its
// own bases this way from the compacting count's 512-Gaussian chunk totals
// (the scan kernel is one launch fewer; the totals are a few KB in L2).
// Not inlined: inlined, it raised the emit's registers past the four
// wavefronts per SIMD it runs at (127 -> 139 VGPRs).
__device__ __attribute__((noinline)) uint2 block_sum_u2(const uint2* __restrict__ cnt, int n, uint2* sh) {
  uint2 s = make_uint2(0u, 0u);
#pragma unroll 4
  for (int w = (int)threadIdx.x; w < n; w += 256) {
    const uint2 v = cnt[w];
    s.x += v.x;
    s.y += v.y;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    s.x += __shfl_xor(s.x, o, 64);
    s.y += __shfl_xor(s.y, o, 64);
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  const uint2 r = make_uint2((sh[0].x + sh[1].x) + (sh[2].x + sh[3].x), (sh[0].y + sh[1].y) + (sh[2].y + sh[3].y));
  __syncthreads();   // sh is rewritten by the next call
  return r;
}

// The first slots of the k-th wavefront of a chunk whose counts are not
// scanned: the workgroup's base for the chunk plus the counts of the chunk's
// wavefronts before it (wc: those counts, staged in LDS by one load each).
__device__ __forceinline__ uint2 wave_base(uint2 bb, const uint2* wc, int k) {
  for (int w = 0; w < k; ++w) {
    bb.x += wc[w].x;
    bb.y += wc[w].y;
  }
  return bb;
}

// Grid-stride over whole wavefronts of flattened Gaussians, so that a launch
// sized for the workspace capacity serves any batch (sizes from the header).
// The binary searches over slice depths read (z, sigma_z) from an LDS copy
// when the batch has at most kZsLds slices (a chain of dependent loads that
// otherwise goes to the cache hierarchy at every step).
constexpr int kZsLds = 2048;

// Gaussians per workgroup round of the compacting count.
constexpr int kCountChunk = 512;

// COMPACT (axial batches of few slices per group, where most Gaussians are far
// from every slice): a workgroup first tests a chunk of kCountChunk Gaussians
// against the group's depth range and lists the near ones in LDS, then gives
// one lane to each listed Gaussian for the covariance and footprints.  Without
// the list, the few near Gaussians of every wavefront kept the whole
// wavefront on the long path (the count of an 8-slice batch of 500k
// Gaussians was bound by that divergence).
template <int DT, bool POSED, bool COMPACT>
__global__ __launch_bounds__(256) void k_pre_count(PreArgs a) {
  __shared__ float2 zs_lds[POSED ? 1 : kZsLds];
  __shared__ int s_list[COMPACT ? kCountChunk : 1];
  __shared__ uint32_t s_nrec[COMPACT ? kCountChunk : 1], s_ninst[COMPACT ? kCountChunk : 1];
  __shared__ uint32_t s_kr[COMPACT ? kCountChunk : 1];
  __shared__ uint2 s_csum[4];
  __shared__ int s_n;
  const int total = a.hdr->total_gauss;
  const int n_groups = a.hdr->n_groups;
  const int n_slices = a.hdr->n_slices;
  reset_forward(a.hdr, a.ctr, a.work, a.bin_lo, a.bin_hi, a.clear_overflow);
  const float2* zs = nullptr;
  if (!POSED && n_slices <= kZsLds) {
    for (int i = threadIdx.x; i < n_slices; i += 256) zs_lds[i] = make_float2(a.slices[i].z, a.slices[i].sigma_z);
    __syncthreads();
    zs = zs_lds;
  }
  if constexpr (!COMPACT) {
    const int stride = gridDim.x * 256;
    for (int t = blockIdx.x * 256 + threadIdx.x; (t & ~63) < total; t += stride)
      count_one<DT, POSED>(a, zs, n_groups, t);
  } else {
    for (int base = blockIdx.x * kCountChunk; base < total; base += gridDim.x * kCountChunk) {
      if (threadIdx.x == 0) s_n = 0;
      __syncthreads();
      for (int i = threadIdx.x; i < kCountChunk; i += 256) {
        const int t = base + i;
        const bool near = t < total && maybe_near<DT>(a, n_groups, t);
        s_nrec[i] = 0u;
        s_ninst[i] = 0u;
        s_kr[i] = 0u;   // read only for Gaussians with records
        if (near) s_list[atomicAdd(&s_n, 1)] = i;
      }
      __syncthreads();
      const int n = s_n;
      // the near Gaussians, 2^count_lg lanes each (one slice per lane and
      // round): a narrow batch has few near Gaussians per chunk, and one lane
      // each would leave a single wavefront running long serial chains
      const int lg = a.count_lg;
      for (int jb = 0; jb < n; jb += (256 >> lg)) {
        const int j = jb + (int)(threadIdx.x >> lg);
        const bool active = j < n;
        const int i = active ? s_list[j] : 0;
        Loaded L;
        load_params<DT>(a, n_groups, base + i, L);
        activate(a, L);
        uint32_t nr, ni, kr;
        count_slices_lanes(a, zs, L, active, lg, &nr, &ni, &kr);
        if (active && (threadIdx.x & ((1u << lg) - 1u)) == 0u) {
          s_nrec[i] = nr;
          s_ninst[i] = ni;
          s_kr[i] = kr;
        }
      }
      __syncthreads();
      // whole wavefronts (chunk and base are multiples of 64; total is too)
      uint2 cs = make_uint2(0u, 0u);
      for (int i = threadIdx.x; i < kCountChunk; i += 256) {
        const int t = base + i;
        if ((t & ~63) < total) count_store(a, t, s_nrec[i], s_ninst[i], s_kr[i]);
        cs.x += s_nrec[i];
        cs.y += s_ninst[i];
      }
      if (a.chunk_cnt) {
        // the chunk's totals, from which the emit forms its bases
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
          cs.x += __shfl_xor(cs.x, o, 64);
          cs.y += __shfl_xor(cs.y, o, 64);
        }
        if ((threadIdx.x & 63) == 0) s_csum[threadIdx.x >> 6] = cs;
      }
      __syncthreads();   // the LDS arrays are rewritten by the next chunk
      if (a.chunk_cnt && threadIdx.x == 0)
        a.chunk_cnt[base / kCountChunk] = make_uint2((s_csum[0].x + s_csum[1].x) + (s_csum[2].x + s_csum[3].x),
                                                     (s_csum[0].y + s_csum[1].y) + (s_csum[2].y + s_csum[3].y));
    }
  }
}

// A workgroup takes `chunk` consecutive Gaussians at a time (a multiple of 256,
// at most kEmitChunk): their slots (wavefront scans), then the emit of those
// that have records, spread over the four wavefronts.  A batch of a few slices
// reaches a small fraction of a large set, and without the gathering most
// lanes would idle on Gaussians without records; 512 at a time gives a grid of
// about four workgroups per CU on 500k Gaussians (2,048 at a time left one per
// CU and took 0.028 ms per 8-slice emit against 0.018).  A deep stack reaches
// nearly all of them and takes 256 at a time (one wavefront's worth each, the
// most parallel form).
constexpr int kEmitChunk = 512;
// (the emit reads the compacting count's chunk totals chunk by chunk)
static_assert(kEmitChunk == kCountChunk, "emit and count chunks differ");

template <int DT, int W, bool POSED>
__global__ __launch_bounds__(256) void k_pre_emit(PreArgs a) {
  __shared__ int list[kEmitChunk];
  __shared__ int n_list;
  __shared__ double cov64[4][POSED ? 64 : 1][6];
  __shared__ RecSigma rsgs[4][POSED ? 1 : 64];
  __shared__ EmitGauss egs[4][64];
  __shared__ float4 pws[4][POSED ? 64 : 1];
  __shared__ uint2 stg[4][W >= 8 ? kStagePerLane * 64 : 1];
  const int total = a.hdr->total_gauss;
  const int n_groups = a.hdr->n_groups;
  __shared__ uint2 s_sum[4];
  __shared__ uint2 s_wc[kEmitChunk / 64];
  const int wave = threadIdx.x >> 6;
  const int chunk = a.emit_chunk;
  // unscanned counts come only with the compacting count, for groups of at
  // most 8 slices (the deep-stack instantiations leave the code out: it cost
  // them a wavefront per SIMD in registers)
  constexpr bool kMayForm = W <= 8;
  const bool form = kMayForm && !a.scanned;
  if (form && blockIdx.x == 0) {
    // the totals, which the sort and the host read
    const uint2 tot = block_sum_u2(a.chunk_cnt, (total + kCountChunk - 1) / kCountChunk, s_sum);
    if (threadIdx.x == 0) {
      a.ctr[kCtrRecords] = tot.x;
      a.ctr[kCtrInstances] = tot.y;
    }
  }
  if (chunk == 256) {
    // one wavefront's 64 Gaussians at a time, synchronised within the
    // wavefront only (deep stacks: the counts are always scanned)
    __shared__ int n_w[4];
    int* wl = list + wave * 64;
    const int lane = threadIdx.x & 63;
    for (int t0 = blockIdx.x * 256 + wave * 64; t0 < total; t0 += gridDim.x * 256) {
      if (lane == 0) n_w[wave] = 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      slots_wave(a, t0, a.wave_cnt[t0 >> 6], wl, &n_w[wave]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const uint32_t n = (uint32_t)__builtin_amdgcn_readfirstlane(n_w[wave]);
      if (n > 0u) emit_wave<DT, W, POSED>(a, n_groups, wl, 0u, n, cov64[wave], rsgs[wave], egs[wave], pws[wave],
                                          stg[wave]);
    }
    return;
  }
  for (int base = blockIdx.x * chunk; base < total; base += gridDim.x * chunk) {
    if (threadIdx.x == 0) n_list = 0;
    uint2 bb = make_uint2(0u, 0u);
    if (form) {
      bb = block_sum_u2(a.chunk_cnt, base / kCountChunk, s_sum);
      if (threadIdx.x < kEmitChunk / 64) {
        const int w = (base >> 6) + (int)threadIdx.x;
        s_wc[threadIdx.x] = w < a.hdr->n_waves ? a.wave_cnt[w] : make_uint2(0u, 0u);
      }
    }
    __syncthreads();
    for (int t0 = base + wave * 64; t0 < min(base + chunk, total); t0 += 256)
      slots_wave(a, t0, form ? wave_base(bb, s_wc, (t0 - base) >> 6) : a.wave_cnt[t0 >> 6], list, &n_list);
    __syncthreads();
    const uint32_t n = (uint32_t)n_list;
    // the list spread over the four wavefronts in whole rounds of 64 / W
    // entries: a short list (a narrow batch) in one wavefront would leave the
    // other three idle and take W serial rounds
    constexpr uint32_t kRound = 64u / (uint32_t)W;
    uint32_t q = ((n + 3u) / 4u + kRound - 1u) / kRound * kRound;
    q = q > 64u ? 64u : (q < kRound ? kRound : q);
    for (uint32_t j0 = (uint32_t)wave * q; j0 < n; j0 += 4u * q)
      emit_wave<DT, W, POSED>(a, n_groups, list, j0, j0 + q < n ? j0 + q : n, cov64[wave], rsgs[wave], egs[wave],
                              pws[wave], stg[wave]);
    __syncthreads();   // list and n_list are rewritten by the next chunk
  }
}

template <int DT, bool POSED>
hipError_t launch_emit_dt(const PreArgs& a, int width, unsigned blocks, hipStream_t s) {
  switch (width) {
    case 16: k_pre_emit<DT, 16, POSED><<<blocks, 256, 0, s>>>(a); break;
    case 8: k_pre_emit<DT, 8, POSED><<<blocks, 256, 0, s>>>(a); break;
    case 4: k_pre_emit<DT, 4, POSED><<<blocks, 256, 0, s>>>(a); break;
    case 2: k_pre_emit<DT, 2, POSED><<<blocks, 256, 0, s>>>(a); break;
    default: k_pre_emit<DT, 1, POSED><<<blocks, 256, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

template <bool POSED, bool COMPACT>
hipError_t launch_count_p(const PreArgs& a, int attr_dtype, unsigned blocks, hipStream_t s) {
  switch (attr_dtype) {
    case GP_BF16: k_pre_count<GP_BF16, POSED, COMPACT><<<blocks, 256, 0, s>>>(a); break;
    case GP_F16: k_pre_count<GP_F16, POSED, COMPACT><<<blocks, 256, 0, s>>>(a); break;
    case GP_Q16: k_pre_count<GP_Q16, POSED, COMPACT><<<blocks, 256, 0, s>>>(a); break;
    case GP_QM: k_pre_count<GP_QM, POSED, COMPACT><<<blocks, 256, 0, s>>>(a); break;
    default: k_pre_count<GP_F32, POSED, COMPACT><<<blocks, 256, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

template <bool POSED>
hipError_t launch_emit_p(const PreArgs& a, int attr_dtype, int width, unsigned blocks, hipStream_t s) {
  switch (attr_dtype) {
    case GP_BF16: return launch_emit_dt<GP_BF16, POSED>(a, width, blocks, s);
    case GP_F16: return launch_emit_dt<GP_F16, POSED>(a, width, blocks, s);
    case GP_Q16: return launch_emit_dt<GP_Q16, POSED>(a, width, blocks, s);
    case GP_QM: return launch_emit_dt<GP_QM, POSED>(a, width, blocks, s);
    default: return launch_emit_dt<GP_F32, POSED>(a, width, blocks, s);
  }
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
  k_reset<<<(unsigned)blocks, 256, 0, s>>>(ws.d_hdr, ws.d_ctr, ws.d_work, ws.d_bin_lo, ws.d_bin_hi,
                                          clear_overflow ? 1 : 0);
  return hipGetLastError();
}

static PreArgs pre_args(const RenderConst& rc, const Workspace& ws, uint32_t sentinel_bin) {
  return PreArgs{rc, ws.d_hdr, ws.d_groups, ws.d_slices, ws.d_ctr, ws.d_rec_pay, ws.d_rec_meta, ws.d_g_rbase,
                 ws.d_g_nrec, ws.d_g_ninst, ws.d_g_krange, ws.d_wave_cnt, ws.d_inst_key, ws.d_inst_val,
                 sentinel_bin, ws.d_poses, 256, 1, nullptr, 0, ws.d_work, ws.d_bin_lo, ws.d_bin_hi, 0};
}

hipError_t launch_pre_count(const RenderConst& rc, const Workspace& ws, const LaunchDims& d, bool clear_overflow,
                            bool scanned, hipStream_t s) {
  if (d.gauss <= 0) return launch_reset(ws, clear_overflow, d, s);
  PreArgs a = pre_args(rc, ws, 0u);
  a.clear_overflow = clear_overflow ? 1 : 0;
  a.scanned = scanned ? 1 : 0;
  if (!scanned) a.chunk_cnt = ws.d_wave_cnt + ws.wave_cap;
  // enough workgroups for the reset of the bin ranges too (16 bins per thread)
  const int64_t reset_blocks = (d.bins + 4095) / 4096;
  auto grid = [&](int64_t per_block) {
    int64_t blocks = std::max<int64_t>((d.gauss + per_block - 1) / per_block, reset_blocks);
    return (unsigned)(blocks > 16384 ? 16384 : blocks);
  };
  if (d.posed) return launch_count_p<true, false>(a, rc.attr_dtype, grid(256), s);
  // groups of at most 8 slices: most Gaussians are far from all of them
  if (d.emit_width <= 8) {
    while ((1 << a.count_lg) < d.emit_width) ++a.count_lg;   // one lane per slice of a group
    return launch_count_p<false, true>(a, rc.attr_dtype, grid(kCountChunk), s);
  }
  return launch_count_p<false, false>(a, rc.attr_dtype, grid(256), s);
}

hipError_t launch_pre_emit(const RenderConst& rc, const Workspace& ws, const LaunchDims& d, uint32_t sentinel_bin,
                           bool scanned, hipStream_t s) {
  if (d.gauss <= 0) return hipSuccess;
  PreArgs a = pre_args(rc, ws, sentinel_bin);
  a.scanned = scanned ? 1 : 0;
  if (!scanned) a.chunk_cnt = ws.d_wave_cnt + ws.wave_cap;
  // few slices per Gaussian set (narrow emit): most Gaussians have no record
  a.emit_chunk = d.emit_width >= 16 ? 256 : kEmitChunk;
  int64_t blocks = (d.gauss + a.emit_chunk - 1) / a.emit_chunk;
  if (blocks > 16384) blocks = 16384;
  return d.posed ? launch_emit_p<true>(a, rc.attr_dtype, d.emit_width, (unsigned)blocks, s)
                 : launch_emit_p<false>(a, rc.attr_dtype, d.emit_width, (unsigned)blocks, s);
}

}  // namespace gp
