// Forward preprocess: per Gaussian, activation (s, q -> Sigma), then for every
// slice of its group the axial cull, Focus-Gaussian projection, normalised
// intensity and tile footprint (Sec. 4.2: axial re-parameterisation, opacity
// modulation, screen-space projection, intensity normalisation).
//
// One thread per Gaussian, looping over the slices of its group, so the
// covariance is built once per launch and reused by every slice.  Records of a
// Gaussian are contiguous ([rbase, rbase + nrec)); record and instance slots
// are reserved with one atomic per wavefront (inclusive scan across lanes).
// Every tile of a record's footprint takes a rank in its bin with an atomic
// increment; the bin scan turns (bin, rank) into a list position.
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

struct PreArgs {
  RenderConst rc;
  const GroupDev* groups;
  const SliceDev* slices;
  uint32_t* ctr;
  uint32_t* bin_count;
  RecPay* rec_pay;
  RecMeta* rec_meta;
  uint32_t* g_rbase;
  uint32_t* g_nrec;
  uint32_t* inst_rank;
  uint32_t* inst_rid;
};

template <int DT>
__global__ __launch_bounds__(256) void k_preprocess(PreArgs a) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int wave0 = t & ~63;
  if (wave0 >= a.rc.total_gauss) return;  // whole wavefront out of range

  // group of this wavefront (groups start at multiples of 64)
  int g = 0;
  for (int j = 1; j < a.rc.n_groups; ++j)
    if (a.groups[j].gbase <= wave0) g = j;
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

  // pass 1: records of this Gaussian (axially kept slices)
  uint32_t nrec = 0;
  for (int k = G.k0; k < G.k1; ++k) {
    const SpecAxial ax = spec_axial(p[2], c.szz, a.slices[k].z, a.slices[k].sigma_z);
    nrec += (ok && (exact || ax.q <= a.rc.q_cut)) ? 1u : 0u;
  }
  const uint32_t rbase = wave_reserve(&a.ctr[kCtrRecords], nrec);
  a.g_rbase[t] = rbase;
  a.g_nrec[t] = nrec;
  if (rbase + nrec > a.rc.rec_cap && nrec) a.ctr[kCtrOverflow] = 1u;

  // pass 2: write the records and their tile instances
  uint32_t r = rbase;
  for (int k = G.k0; k < G.k1; ++k) {
    const SliceDev sl = a.slices[k];
    const SpecAxial ax = spec_axial(p[2], c.szz, sl.z, sl.sigma_z);
    const bool kept = ok && (exact || ax.q <= a.rc.q_cut);
    SpecRect rect;
    bool vis = false;
    if (kept) {
      vis = spec_rect(c, p[0], p[1], ax, sl.x0, sl.y0, sl.dx, sl.dy, sl.ntx, sl.nty, a.rc.bbox, rect);
      if (exact) {
        rect.tx0 = 0; rect.tx1 = sl.ntx - 1; rect.ty0 = 0; rect.ty1 = sl.nty - 1;
        vis = true;
      }
    }
    const uint32_t ntiles = vis ? (uint32_t)((rect.tx1 - rect.tx0 + 1) * (rect.ty1 - rect.ty0 + 1)) : 0u;
    const uint32_t ibase = wave_reserve(&a.ctr[kCtrInstances], ntiles);
    if (!kept) continue;
    const uint32_t rid = r++;
    if (rid >= a.rc.rec_cap) continue;
    const bool inst_ok = (uint64_t)ibase + ntiles <= a.rc.inst_cap;
    if (!inst_ok) a.ctr[kCtrOverflow] = 1u;

    // image quantities (binary32; not part of the membership specification)
    RecPay pay;
    RecMeta meta;
    meta.ibase = ibase;
    meta.ntiles = inst_ok ? ntiles : 0u;
    meta.rx = vis ? ((uint32_t)rect.tx0 | ((uint32_t)rect.tx1 << 16)) : 0u;
    meta.ry = vis ? ((uint32_t)rect.ty0 | ((uint32_t)rect.ty1 << 16)) : 0u;
    pay.gid = (uint32_t)j;
    pay.slice = (uint32_t)k;
    if (vis) {
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
      const bool good = det > 0.0f && isfinite(at) && isfinite(pay.x) && isfinite(pay.y) &&
                        isfinite(pay.a) && isfinite(pay.b) && isfinite(pay.c);
      if (!good) pay.x = pay.y = pay.a = pay.b = pay.c = pay.w = 0.0f;
    } else {
      pay.x = pay.y = pay.a = pay.b = pay.c = pay.w = 0.0f;
    }
    a.rec_pay[rid] = pay;
    a.rec_meta[rid] = meta;
    if (!inst_ok) continue;
    uint32_t slot = ibase;
    for (int ty = rect.ty0; ty <= rect.ty1 && vis; ++ty) {
      for (int tx = rect.tx0; tx <= rect.tx1; ++tx, ++slot) {
        const uint32_t bin = (uint32_t)(sl.tile_base + ty * sl.ntx + tx);
        a.inst_rank[slot] = atomicAdd(&a.bin_count[bin], 1u);
        a.inst_rid[slot] = rid;
      }
    }
  }
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  k_fill_u32<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(p, value, n);
  return hipGetLastError();
}

hipError_t launch_preprocess(const RenderConst& rc, const Workspace& ws, hipStream_t s) {
  PreArgs a{rc, ws.d_groups, ws.d_slices, ws.d_ctr, ws.d_bin_count, ws.d_rec_pay, ws.d_rec_meta,
            ws.d_g_rbase, ws.d_g_nrec, ws.d_inst_rank, ws.d_inst_rid};
  if (rc.total_gauss <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((rc.total_gauss + 255) / 256);
  // every group of a batch shares one attribute dtype (checked by the caller)
  switch (ws.h_groups[0].attr_dtype) {
    case GP_BF16: k_preprocess<GP_BF16><<<blocks, 256, 0, s>>>(a); break;
    case GP_F16: k_preprocess<GP_F16><<<blocks, 256, 0, s>>>(a); break;
    default: k_preprocess<GP_F32><<<blocks, 256, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

}  // namespace gp
