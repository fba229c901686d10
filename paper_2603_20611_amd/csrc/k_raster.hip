// Additive rasterisation of the tile lists (Sec. 4.2, additive rasterisation:
// I(p) = sum over N(p) of alpha~ exp(-1/2 d^T Sigma_2d^-1 d), no occlusion) and
// its adjoint (Sec. 4.3: dI/dalpha~ = exp(.), chain through mu_2d and the conic).
//
// Records arrive in pixel space: with dx, dy the offsets of the pixel index
// from the record's mean, a contribution is w * exp2(a dx^2 + b dx dy + c dy^2)
// (the exponent coefficients carry -1/2 log2(e) and the pixel pitch).  The mean
// is stored as an integer anchor plus a remainder; a tile forms each record's
// offset from its own origin once, as (origin - anchor) - remainder, which is
// exact up to one rounding of a number no larger than the footprint, so pixel
// offsets keep their precision on grids of any size.
//
// Forward: one 64-lane wavefront per 16x16 tile.  The two half-wavefronts
// take two records at a time, and lane m of a half owns the 2 x 4 pixels of
// rows 2 (m >> 2) + {0, 1}, columns 4 (m & 3) + 0..3, so the row terms b dy and
// c dy^2 are shared by four pixels, the column term by two rows, and eight
// pixel chains give the instruction stream the independent operations gfx950
// needs to issue VALU at full rate; the halves' partial sums are added at the
// end of the tile.  Records are staged 64 at a time in LDS and read back as
// broadcasts into VGPRs (operands held in SGPRs halve VALU issue on gfx950);
// each LDS read serves two records.
//
// Backward: one lane per list entry; the lane sweeps the tile's 256 pixels in
// row order with the upstream gradient staged in LDS, and accumulates six
// moments of G(p) e(p) (sum e, sum e dx, sum e dy, sum e dx^2, sum e dx dy,
// sum e dy^2).  The moments fully determine the entry's gradient with respect
// to its record, so no per-pixel reduction and no atomics are needed; they are
// written at the record's own instance slot of that tile and summed per record,
// in footprint order, later.
#include "gp_internal.h"

namespace gp {
namespace {

__device__ __forceinline__ int slice_of_bin(const SliceDev* __restrict__ slices, int n_slices, int bin) {
  int lo = 0, hi = n_slices - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (slices[mid].tile_base <= bin) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct FwdArgs {
  const BatchHdr* hdr;
  const SliceDev* slices;
  const uint32_t* bin_lo;
  const uint32_t* bin_hi;
  const uint32_t* list;
  const RecPay* rec_pay;
  uint32_t* work;
};

// Records with a >= kSmoothA (conditional x-sigma >= 0.42 px) and
// |b| <= kSmoothB are evaluated along each lane's four-pixel row segment by the
// exact product recurrence
//   e(d + 1) = e(d) 2^s(d),  2^s(d + 1) = 2^s(d) g,  s(d) = a (2d + 1) + b dy,  g = 2^(2a)
// which needs two exp2 per four pixels instead of four; the second row's first
// ratio is the first row's times h = 2^b.  Why this needs no clamping: with
// a >= -4 the exponent's x-slope is at most 4 sqrt(-exponent), so
//  * an underflow of e at the segment start leaves the rest of the segment
//    below 2^-27 of the record's peak;
//  * a ratio 2^s that overflows (s >= 128) forces e = 0 exactly at its own
//    row's segment start and, with |b| <= 16 (s >= 112 on the other row), at
//    the other row's too; the products use the multiply with 0 * inf = 0;
//  * a ratio that underflows leaves its row's remaining pixels below 2^-133.

// Work items: one tile position over a group of kSliceGroup consecutive slices
// of one grid, rendered in turn by one wavefront.  The records of a Gaussian
// on consecutive slices are adjacent in memory, so the gathers of a group's
// later slices mostly hit the lines its first slice brought into the cache.
// Used when the grouped items still outnumber the launch's workgroups several
// times over (a deep stack); smaller batches keep one tile per item.
constexpr int kSliceGroup = 3;
constexpr int kGroupMinBins = 3 * 8192;
// Otherwise an item is 4, 2 or 1 consecutive bins (the tile and those to its
// right, which share many records: their gathers then hit the cache), the
// most that still leaves at least one item per workgroup of the launch.
// Measured: a served batch of 63 requests over mixed 256^2-1024^2 grids
// (113k bins) 31k -> 45k -> 53k slices/s at 1, 2, 4 bins per item (8: 52k);
// 64 slices of 256^2 (16,384 bins) 0.373 / 0.362 / 0.387 ms at 1, 2, 4.
__device__ __forceinline__ int bin_group(int n_bins, int workgroups) {
  return n_bins >= 4 * workgroups ? 4 : (n_bins >= 2 * workgroups ? 2 : 1);
}

// A record as a tile's sweep reads it: the mean's offset from the tile origin
// (ox0, oy0), the exponent coefficients a, b, c and the intensity w, and for
// records inside the row recurrence's range g = 2^(2a), the change of the
// per-pixel ratio along a row, and h = 2^b, its change from one row to the
// next (g = -1, h = 0 mark the other records).  A zero record stages to w = 0.
__device__ __forceinline__ void stage_record(const float4 r0, const float4 r1, float ox0, float oy0, float4& s0,
                                             float4& s1) {
  const bool smooth = r0.z >= kSmoothA && fabsf(r0.w) <= kSmoothB;
  s0 = make_float4((ox0 - r1.z) - r0.x, (oy0 - r1.w) - r0.y, r0.z, r0.w);
  s1 = make_float4(r1.x, r1.y, smooth ? exp2f(2.0f * r0.z) : -1.0f, smooth ? exp2f(r0.w) : 0.0f);
}





// The forward's step keeps the same product written as inline asm: the
// compiler's own schedule of the step with the intrinsic measured 1 % slower
// on the 400-slice stack (0.686 -> 0.693 ms).  The compiler cannot see
// inside the asm, so the asm carries the wait state that gfx950 needs before
// a VALU instruction reads a transcendental's result (its operands are often
// fresh exp2 results).
__device__ __forceinline__ float mul0_asm(float x, float y) {
  float r;
  asm("s_nop 0\n\tv_mul_legacy_f32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(y));
  return r;
}

// One step of a half-wavefront: staged record (r0, r1) over the lane's 2 x 4
// pixels whose first pixel is (fx0, fy0) from the tile origin, added to acc
// (rows 0, 1 in acc[0..3], acc[4..7]).
__device__ __forceinline__ void raster_step(const float4 r0, const float4 r1, float fx0, float fy0,
                                            float (&acc)[8]) {
  const float d0 = fx0 + r0.x;
  const float dy0 = fy0 + r0.y;
  const float by0 = r0.w * dy0;
  const float cy0 = r1.x * dy0 * dy0;
  const float p00 = fmaf(fmaf(r0.z, d0, by0), d0, cy0);
  float e00, e01, e02, e03, e10, e11, e12, e13;
  // both records of the step must allow the row recurrence (uniform branch);
  // the record's g is negative where it does not
  if (__builtin_amdgcn_read_exec() == __builtin_amdgcn_ballot_w64(r1.z > 0.0f)) {
    // second row's exponent: p(d0, dy0 + 1) = p00 + b d0 + c (2 dy0 + 1)
    const float p10 = fmaf(r0.w, d0, fmaf(r1.x, fmaf(2.0f, dy0, 1.0f), p00));
    const float t = fmaf(d0, 2.0f, 1.0f);
    e00 = __builtin_amdgcn_exp2f(p00);
    e10 = __builtin_amdgcn_exp2f(p10);
    float q0 = __builtin_amdgcn_exp2f(fmaf(r0.z, t, by0));
    float q1 = q0 * r1.w;
    e01 = mul0_asm(e00, q0);
    e11 = mul0_asm(e10, q1);
    q0 *= r1.z;
    q1 *= r1.z;
    e02 = mul0_asm(e01, q0);
    e12 = mul0_asm(e11, q1);
    q0 *= r1.z;
    q1 *= r1.z;
    e03 = mul0_asm(e02, q0);
    e13 = mul0_asm(e12, q1);
  } else {
    const float dy1 = dy0 + 1.0f;
    const float by1 = r0.w * dy1, cy1 = r1.x * dy1 * dy1;
    const float d1 = d0 + 1.0f, d2 = d0 + 2.0f, d3 = d0 + 3.0f;
    e00 = __builtin_amdgcn_exp2f(p00);
    e01 = __builtin_amdgcn_exp2f(fmaf(fmaf(r0.z, d1, by0), d1, cy0));
    e02 = __builtin_amdgcn_exp2f(fmaf(fmaf(r0.z, d2, by0), d2, cy0));
    e03 = __builtin_amdgcn_exp2f(fmaf(fmaf(r0.z, d3, by0), d3, cy0));
    e10 = __builtin_amdgcn_exp2f(fmaf(fmaf(r0.z, d0, by1), d0, cy1));
    e11 = __builtin_amdgcn_exp2f(fmaf(fmaf(r0.z, d1, by1), d1, cy1));
    e12 = __builtin_amdgcn_exp2f(fmaf(fmaf(r0.z, d2, by1), d2, cy1));
    e13 = __builtin_amdgcn_exp2f(fmaf(fmaf(r0.z, d3, by1), d3, cy1));
  }
  const float w = r1.y;
  acc[0] = fmaf(w, e00, acc[0]);
  acc[1] = fmaf(w, e01, acc[1]);
  acc[2] = fmaf(w, e02, acc[2]);
  acc[3] = fmaf(w, e03, acc[3]);
  acc[4] = fmaf(w, e10, acc[4]);
  acc[5] = fmaf(w, e11, acc[5]);
  acc[6] = fmaf(w, e12, acc[6]);
  acc[7] = fmaf(w, e13, acc[7]);
}

// The two rows of a lane's pixels, clipped to the slice.
__device__ __forceinline__ void store_pixels(const SliceDev& sl, int px0, int py0, const float (&acc)[8]) {
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int py = py0 + r;
    if (py >= sl.height) continue;
    float* o = sl.out + (int64_t)py * sl.width;
    const float* v = acc + 4 * r;
    if (px0 + 3 < sl.width && (reinterpret_cast<uintptr_t>(o + px0) & 15) == 0) {
      *reinterpret_cast<float4*>(o + px0) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
      if (px0 < sl.width) o[px0] = v[0];
      if (px0 + 1 < sl.width) o[px0 + 1] = v[1];
      if (px0 + 2 < sl.width) o[px0 + 2] = v[2];
      if (px0 + 3 < sl.width) o[px0 + 3] = v[3];
    }
  }
}

__device__ __forceinline__ int slice_of(const FwdArgs& a, int n_slices, int tps, int bin) {
  return tps > 0 ? bin / tps : slice_of_bin(a.slices, n_slices, bin);
}

// One 64-lane workgroup per work item (a tile, or a tile position over a
// slice group), items taken from a shared counter; each workgroup's first two
// items are fixed (its index and index + grid size), since every workgroup
// taking its first tickets at once serialised on the counter (12 % of the
// kernel on the 400-slice stack).  Two software pipelines
// hide the memory latency: within a tile, record ids are
// loaded two batches ahead and records one batch ahead; across tiles, the next
// tile is fetched one step per batch of the current one (its queue ticket is
// resolved and its list range loaded after the first batch, its slice found
// and first ids loaded after the second, its first records gathered after the
// third), so a new tile rarely starts by waiting on memory.
//
// XQ (deep stacks on one grid whose tiles form whole 4 x 4-tile units, the
// units a multiple of 8): eight queues, one per XCD (workgroups are placed on
// the XCDs in turn, so workgroup w runs on XCD w mod 8).  Queue q serves the
// units q, q + 8, ... of every slice group, a unit's 16 tiles consecutively:
// the tiles that share a Gaussian's records mostly run on one XCD at about
// the same time and meet in its L2, while every XCD still works through the
// slice groups at the pace of the others.  A wavefront whose queue runs dry
// takes tickets from the next queues.
template <bool XQ>
__global__ __launch_bounds__(64) void k_raster_fwd(FwdArgs a) {
  __shared__ float4 buf0[64];   // x, y, a, b of the batch's records
  __shared__ float4 buf1[64];   // c, w, g, h
  const int n_bins = a.hdr->n_bins;
  const int n_slices = a.hdr->n_slices;
  const int tps = a.hdr->tiles_per_slice;
  const int lane = threadIdx.x;
  // the two half-wavefronts take two records at a time; within a half, lane m
  // owns the 2 x 4 pixels of rows 2 (m >> 2) + {0, 1}, columns 4 (m & 3) + 0..3
  const int half = lane >> 5, m = lane & 31;
  const int row0 = (m >> 2) * 2;
  const int col0 = (m & 3) * 4;
  const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const float fx0 = (float)col0, fy0 = (float)row0;
  // work items (queue tickets) -> first bin; rem = further bins of the item:
  // the same tile on the next slices of a slice group (step tps), or else the
  // next bins (step 1: the tiles to the right, which share many records)
  const int sg = (tps > 0 && n_bins >= kGroupMinBins) ? kSliceGroup : 1;
  const int bg = sg > 1 ? 1 : bin_group(n_bins, (int)gridDim.x);
  const int step = sg > 1 ? tps : 1;
  const int n_items = sg > 1 ? ((n_slices + sg - 1) / sg) * tps : (n_bins + bg - 1) / bg;
  // XQ: items per slice group and queue, the unit row length, this queue
  const int ipg = XQ ? tps >> 3 : 0;
  const int ntx4 = XQ ? a.slices[0].ntx >> 2 : 1;
  const uint32_t n_q = XQ ? (uint32_t)(((n_slices + sg - 1) / sg) * ipg) : 0u;
  int q = XQ ? (int)(blockIdx.x & 7u) : 0;
  uint32_t* counter = XQ ? a.work + kWorkXcd + 32 * q : a.work + kWorkRasterFwd;
  auto first_bin = [&](uint32_t t, int& rem) -> int {
    rem = 0;
    if constexpr (XQ) {
      if (t >= n_q) return -1;
      const int g = (int)t / ipg, r = (int)t - g * ipg;
      const int u = q + 8 * (r >> 4), j = r & 15;
      const int ux = u % ntx4, uy = u / ntx4;
      const int tt = ((uy << 2) + (j >> 2)) * (ntx4 << 2) + (ux << 2) + (j & 3);
      rem = min(sg, n_slices - g * sg) - 1;
      return g * sg * tps + tt;
    }
    if (t >= (uint32_t)n_items) return -1;
    if (sg == 1) {
      const int b0 = (int)t * bg;
      rem = min(bg, n_bins - b0) - 1;
      return b0;
    }
    const int g = (int)t / tps, tt = (int)t - g * tps;
    rem = min(sg, n_slices - g * sg) - 1;
    return g * sg * tps + tt;
  };

  // the first tile, fetched without overlap
  int rem = 0;
  // the first two items of every workgroup are fixed; the counter hands out the rest
  const uint32_t gq = XQ ? gridDim.x >> 3 : gridDim.x;   // workgroups per queue
  const uint32_t local = XQ ? blockIdx.x >> 3 : blockIdx.x;
  const uint32_t fixed = 2u * gq;
  int item = first_bin(local, rem);
  if (item < 0) return;
  uint32_t start = a.bin_lo[item], end = a.bin_hi[item];
  int k = slice_of(a, n_slices, tps, item);
  float4 n0 = zero4, n1 = zero4;
  if (start + lane < end) {
    const float4* src = reinterpret_cast<const float4*>(a.rec_pay + a.list[start + lane]);
    n0 = src[0];
    n1 = src[1];
  }
  uint32_t rid_next = (start + 64 + lane < end) ? a.list[start + 64 + lane] : 0u;
  uint32_t ticket = local + gq;

  while (item >= 0) {
    const int bin = item;
    const SliceDev sl = a.slices[k];
    const int tile = bin - sl.tile_base;
    const int tx = tile % sl.ntx, ty = tile / sl.ntx;
    const int px0 = tx * kTile + col0;
    const int py0 = ty * kTile + row0;
    const float ox0 = (float)(tx * kTile), oy0 = (float)(ty * kTile);
    float acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.f;

    // next tile, advanced one stage per batch
    int nitem = -1, nk = 0, stage = 0, nrem = 0;
    bool took = false;
    uint32_t ns = 0u, ne = 0u, nrid = 0u, nrid2 = 0u;
    float4 m0 = zero4, m1 = zero4;
    auto advance = [&]() {
      if (stage == 0) {
        if (rem > 0) {
          nitem = item + step;
          nrem = rem - 1;
        } else {
          nitem = first_bin(ticket, nrem);
          if constexpr (XQ) {
            // this queue is done: take from the next ones
            for (int k = 1; k < 8 && nitem < 0; ++k) {
              q = (q + 1) & 7;
              counter = a.work + kWorkXcd + 32 * q;
              ticket = wave_take(counter) + fixed;
              nitem = first_bin(ticket, nrem);
            }
          }
          took = true;
        }
        if (nitem >= 0) {
          ns = a.bin_lo[nitem];
          ne = a.bin_hi[nitem];
        }
      } else if (stage == 1) {
        if (nitem >= 0) {
          nk = slice_of(a, n_slices, tps, nitem);
          if (ns + lane < ne) nrid = a.list[ns + lane];
          if (ns + 64 + lane < ne) nrid2 = a.list[ns + 64 + lane];
        }
      } else if (stage == 2) {
        if (nitem >= 0 && ns + lane < ne) {
          const float4* src = reinterpret_cast<const float4*>(a.rec_pay + nrid);
          m0 = src[0];
          m1 = src[1];
        }
      }
      ++stage;
    };

    for (uint32_t base = start; base < end; base += 64) {
      {
        float4 s0, s1;
        stage_record(n0, n1, ox0, oy0, s0, s1);
        buf0[lane] = s0;
        buf1[lane] = s1;   // slots past the end hold zero records (w = 0)
      }
      __syncthreads();
      const int cnt = __builtin_amdgcn_readfirstlane((int)min(64u, end - base));
      const uint32_t nb = base + 64;
      n0 = zero4;
      n1 = zero4;
      if (nb + lane < end) {
        const float4* src = reinterpret_cast<const float4*>(a.rec_pay + rid_next);
        n0 = src[0];
        n1 = src[1];
      }
      if (nb + 64 + lane < end) rid_next = a.list[nb + 64 + lane];
      for (int j = 0; j < cnt; j += 2) {
        const float4 r0 = buf0[j + half];
        const float4 r1 = buf1[j + half];   // j + 1 may be a zero slot: w = 0
        asm volatile("" :: "v"(r1.z), "v"(r1.w));   // one 16-byte LDS read for r1
        raster_step(r0, r1, fx0, fy0, acc);
      }
      if (stage < 3) advance();
      __syncthreads();
    }
    while (stage < 3) advance();   // short tiles: finish fetching the next one

    // the two halves hold partial sums of the same pixels
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] += __shfl_xor(acc[i], 32, 64);
    if (half == 0) store_pixels(sl, px0, py0, acc);
    // the next tile becomes the current one
    item = nitem;
    rem = nrem;
    start = ns;
    end = ne;
    k = nk;
    n0 = m0;
    n1 = m1;
    rid_next = nrid2;
    if (item >= 0 && took) ticket = wave_take(counter) + fixed;
  }
}

// Small batches (at most kSplitMaxBins bins): one 256-lane workgroup per tile,
// its four wavefronts taking every fourth batch of the list, so that a batch of
// a few slices still fills the chip (a wavefront per tile would leave most
// SIMDs with one or two wavefronts to hide latency).  The four partial images
// are added in a fixed order through LDS (deterministic).
constexpr int kSplitMaxBins = 4096;

__global__ __launch_bounds__(256) void k_raster_fwd_split(FwdArgs a) {
  __shared__ float4 buf0[4][64];
  __shared__ float4 buf1[4][64];
  __shared__ float part[3][kTilePix];
  const int bin = blockIdx.x;
  if (bin >= a.hdr->n_bins) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int half = lane >> 5, m = lane & 31;
  const int row0 = (m >> 2) * 2, col0 = (m & 3) * 4;
  const int k = slice_of(a, a.hdr->n_slices, a.hdr->tiles_per_slice, bin);
  const SliceDev sl = a.slices[k];
  const int tile = bin - sl.tile_base;
  const int px0 = (tile % sl.ntx) * kTile + col0;
  const int py0 = (tile / sl.ntx) * kTile + row0;
  const float ox0 = (float)(px0 - col0), oy0 = (float)(py0 - row0);
  const float fx0 = (float)col0, fy0 = (float)row0;
  const uint32_t start = a.bin_lo[bin], end = a.bin_hi[bin];
  const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
  float acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = 0.f;
  // this wavefront's batches: start + 64 (wave + 4 i)
  uint32_t base = start + 64u * wave;
  float4 n0 = zero4, n1 = zero4;
  if (base + lane < end) {
    const float4* src = reinterpret_cast<const float4*>(a.rec_pay + a.list[base + lane]);
    n0 = src[0];
    n1 = src[1];
  }
  uint32_t rid_next = (base + 256 + lane < end) ? a.list[base + 256 + lane] : 0u;
  for (; base < end; base += 256) {
    {
      float4 s0, s1;
      stage_record(n0, n1, ox0, oy0, s0, s1);
      buf0[wave][lane] = s0;
      buf1[wave][lane] = s1;
    }
    // the wavefront's own LDS slots: ordering within the wavefront suffices
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int cnt = __builtin_amdgcn_readfirstlane((int)min(64u, end - base));
    const uint32_t nb = base + 256;
    n0 = zero4;
    n1 = zero4;
    if (nb + lane < end) {
      const float4* src = reinterpret_cast<const float4*>(a.rec_pay + rid_next);
      n0 = src[0];
      n1 = src[1];
    }
    if (nb + 256 + lane < end) rid_next = a.list[nb + 256 + lane];
    for (int j = 0; j < cnt; j += 2) {
      const float4 r0 = buf0[wave][j + half];
      const float4 r1 = buf1[wave][j + half];   // j + 1 may be a zero slot: w = 0
      asm volatile("" :: "v"(r1.z), "v"(r1.w));   // one 16-byte LDS read for r1
      raster_step(r0, r1, fx0, fy0, acc);
    }
    // all reads of this batch before the slots are overwritten
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] += __shfl_xor(acc[i], 32, 64);
  const int p0 = row0 * kTile + col0;
  if (wave > 0 && half == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      part[wave - 1][p0 + i] = acc[i];
      part[wave - 1][p0 + kTile + i] = acc[4 + i];
    }
  }
  __syncthreads();
  if (wave == 0 && half == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc[i] = ((acc[i] + part[0][p0 + i]) + part[1][p0 + i]) + part[2][p0 + i];
      acc[4 + i] = ((acc[4 + i] + part[0][p0 + kTile + i]) + part[1][p0 + kTile + i]) + part[2][p0 + kTile + i];
    }
    store_pixels(sl, px0, py0, acc);
  }
}

struct BwdArgs {
  const BatchHdr* hdr;
  const SliceDev* slices;
  const uint32_t* bin_lo;
  const uint32_t* bin_hi;
  const uint32_t* list;
  const RecPay* rec_pay;
  const RecMeta* rec_meta;
  const float* grad_out;
  float4* moments;
};

// 256 lanes per tile, tiles assigned round-robin (the tiles of a batch cost
// about the same, and every workgroup taking a ticket from one counter at the
// start of a small batch serialised on it: 30 % of this kernel); each lane sums
// the six moments of a list entry over a quarter of the tile's upstream
// gradient, staged in LDS.
__global__ __launch_bounds__(256) void k_raster_bwd(BwdArgs a) {
  __shared__ float G[kTilePix];
  const int n_bins = a.hdr->n_bins;
  const int n_slices = a.hdr->n_slices;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int item = blockIdx.x; item < n_bins; item += gridDim.x) {
    const int bin = item;
    const uint32_t start = a.bin_lo[bin], end = a.bin_hi[bin];
    if (start == end) continue;
    const int k = slice_of_bin(a.slices, n_slices, bin);
    const SliceDev sl = a.slices[k];
    const int tile = bin - sl.tile_base;
    const int tx = tile % sl.ntx, ty = tile / sl.ntx;
    {
      const int t = threadIdx.x;
      const int px = tx * kTile + (t & 15), py = ty * kTile + (t >> 4);
      G[t] = (px < sl.width && py < sl.height) ? a.grad_out[sl.out_off + (int64_t)py * sl.width + px] : 0.f;
    }
    __syncthreads();
    const float fx0 = (float)(tx * kTile), fy0 = (float)(ty * kTile);
    // work units: a list entry's four-row quarter of the tile (4 lanes per
    // entry), so that a tile with a few more entries than lanes costs a quarter
    // round more, not a whole round
    const uint32_t units = 4u * (end - start);
    for (uint32_t u0 = (uint32_t)wave * 64u; u0 < units; u0 += 256u) {
      const uint32_t u = u0 + (uint32_t)lane;
      const bool valid = u < units;
      const uint32_t e = u >> 2, rq = u & 3u;
      float M0 = 0.f, Mx = 0.f, My = 0.f, Mxx = 0.f, Mxy = 0.f, Myy = 0.f;
      uint32_t rid = 0u;
      if (valid) {
        rid = a.list[start + e];
        const float4* src = reinterpret_cast<const float4*>(a.rec_pay + rid);
        const float4 r0 = src[0];
        const float4 r1 = src[1];
        const float ca = r0.z, cb2 = r0.w, cc = r1.x;
        // offsets of the tile origin from the mean: (origin - anchor) - remainder
        const float ox = (fx0 - r1.z) - r0.x, oy = (fy0 - r1.w) - r0.y;
        float dx[kTile];
#pragma unroll
        for (int c = 0; c < kTile; ++c) dx[c] = ox + (float)c;
        // the forward's row recurrence over each four-pixel segment for the
        // records it allows (same conditions, same reasoning: no clamping)
        const bool smooth = ca >= kSmoothA && fabsf(cb2) <= kSmoothB;
        const float gx = smooth ? __builtin_amdgcn_exp2f(2.0f * ca) : 0.f;
        for (int rr = 0; rr < 4; ++rr) {
          const int row = 4 * (int)rq + rr;
          const float dy = oy + (float)row;
          const float by = cb2 * dy;
          const float cy = cc * dy * dy;
          const float4* grow = reinterpret_cast<const float4*>(G + row * kTile);
          float s0 = 0.f, sx = 0.f, sxx = 0.f;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float4 g4 = grow[q];
            const float gv[4] = {g4.x, g4.y, g4.z, g4.w};
            float ev[4];
            const float d0 = dx[4 * q];
            if (smooth) {
              // a ratio that overflows meets e = 0 (as in the forward), and
              // the products with 0 * inf = 0 give 0 there
              ev[0] = __builtin_amdgcn_exp2f(fmaf(fmaf(ca, d0, by), d0, cy));
              float r = __builtin_amdgcn_exp2f(fmaf(ca, fmaf(2.0f, d0, 1.0f), by));
              ev[1] = mul0(ev[0], r);
              r *= gx;
              ev[2] = mul0(ev[1], r);
              r *= gx;
              ev[3] = mul0(ev[2], r);
            } else {
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                const float d = dx[4 * q + c];
                ev[c] = __builtin_amdgcn_exp2f(fmaf(fmaf(ca, d, by), d, cy));
              }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const float d = dx[4 * q + c];
              const float we = gv[c] * ev[c];
              const float wd = we * d;
              s0 += we;
              sx += wd;
              sxx = fmaf(wd, d, sxx);
            }
          }
          M0 += s0;
          Mx += sx;
          Mxx += sxx;
          My = fmaf(dy, s0, My);
          Mxy = fmaf(dy, sx, Mxy);
          Myy = fmaf(dy * dy, s0, Myy);
        }
      }
      // the entry's four quarters, added in a fixed order
#pragma unroll
      for (int o = 1; o <= 2; o <<= 1) {
        M0 += __shfl_xor(M0, o, 64);
        Mx += __shfl_xor(Mx, o, 64);
        My += __shfl_xor(My, o, 64);
        Mxx += __shfl_xor(Mxx, o, 64);
        Mxy += __shfl_xor(Mxy, o, 64);
        Myy += __shfl_xor(Myy, o, 64);
      }
      if (valid && rq == 0u) {
        // the record's instance slot of this tile (footprint enumerated row-major)
        const RecMeta meta = a.rec_meta[rid];
        const uint32_t tx0 = meta.rx & 0xFFFFu, tx1 = meta.rx >> 16, ty0 = meta.ry & 0xFFFFu;
        const uint32_t slot = meta.ibase + ((uint32_t)ty - ty0) * (tx1 - tx0 + 1u) + ((uint32_t)tx - tx0);
        a.moments[2 * (size_t)slot] = make_float4(M0, Mx, My, Mxx);
        a.moments[2 * (size_t)slot + 1] = make_float4(Mxy, Myy, 0.f, 0.f);
      }
    }
    __syncthreads();   // G[] is reused by the next tile
  }
}

}  // namespace

hipError_t launch_raster_fwd(const RenderConst& rc, const Workspace& ws, const LaunchDims& d, hipStream_t s) {
  (void)rc;
  if (d.bins <= 0) return hipSuccess;
  FwdArgs a{ws.d_hdr, ws.d_slices, ws.d_bin_lo, ws.d_bin_hi, ws.d_list, ws.d_rec_pay, ws.d_work};
  if (d.bins <= kSplitMaxBins) {
    // d.bins bounds the batch's bins (the header holds the exact count)
    k_raster_fwd_split<<<(unsigned)d.bins, 256, 0, s>>>(a);
    return hipGetLastError();
  }
  const int64_t blocks = d.bins < 8192 ? d.bins : 8192;
  // per-XCD queues for a deep stack on one grid of whole 4 x 4-tile units (the
  // staged batch on the host tells; a capture for later batches does not)
  bool xq = false;
  if (d.host_batch && ws.h_hdr->n_slices > 0) {
    const int tps = ws.h_hdr->tiles_per_slice;
    const SliceDev& s0 = ws.h_slices[0];
    xq = tps > 0 && ws.h_hdr->n_bins >= kGroupMinBins && s0.ntx * s0.nty == tps && s0.ntx % 4 == 0 &&
         s0.nty % 4 == 0 && (tps / 16) % 8 == 0 && blocks >= 64;
  }
  if (xq) {
    k_raster_fwd<true><<<(unsigned)(blocks & ~7ll), 64, 0, s>>>(a);
  } else {
    k_raster_fwd<false><<<(unsigned)blocks, 64, 0, s>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_raster_bwd(const RenderConst& rc, const Workspace& ws, const float* grad_out,
                             const LaunchDims& d, hipStream_t s) {
  (void)rc;
  if (d.bins <= 0) return hipSuccess;
  BwdArgs a{ws.d_hdr, ws.d_slices, ws.d_bin_lo, ws.d_bin_hi, ws.d_list, ws.d_rec_pay, ws.d_rec_meta, grad_out,
            ws.d_moments};
  const int64_t blocks = d.bins < 2048 ? d.bins : 2048;
  k_raster_bwd<<<(unsigned)blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace gp
