// Tile lists: exclusive scan of the per-bin counts, scatter of every instance
// to (bin start + rank), then a per-bin sort by Gaussian index, which makes
// each list's order unique and independent of the order in which atomics
// handed out ranks.  A list holds record ids; the rasterisers gather the
// 32-byte records themselves.
//
// The paper sums over N(p), the Gaussians overlapping pixel p (Sec. 4.2); with
// purely additive accumulation the order of a list does not change the sum, so
// the Gaussian index is used as the tie-free ordering key.
#include "gp_internal.h"

namespace gp {
namespace {

constexpr int kScanThreads = 1024;

// Single-workgroup exclusive scan of n counts (n up to a few million).
__global__ __launch_bounds__(kScanThreads) void k_scan_bins(const BatchHdr* __restrict__ hdr,
                                                            const uint32_t* __restrict__ count,
                                                            uint32_t* __restrict__ start) {
  __shared__ uint32_t part[kScanThreads];
  const int n = hdr->n_bins;
  const int t = threadIdx.x;
  const int per = (n + kScanThreads - 1) / kScanThreads;
  const int b = t * per;
  const int e = min(n, b + per);
  uint32_t sum = 0;
  for (int i = b; i < e; ++i) sum += count[i];
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    const uint32_t v = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - sum;  // exclusive prefix of this chunk
  for (int i = b; i < e; ++i) {
    start[i] = run;
    run += count[i];
  }
  if (t == kScanThreads - 1) start[n] = part[t];
}

struct ScatterArgs {
  const RecPay* rec_pay;
  const RecMeta* rec_meta;
  const SliceDev* slices;
  const uint32_t* ctr;
  const uint32_t* bin_start;
  const uint32_t* inst_rank;
  uint64_t* sort_key;
  uint32_t rec_cap;
};

// One thread per record: every tile of its footprint goes to bin start + rank.
__global__ __launch_bounds__(256) void k_scatter(ScatterArgs a) {
  const uint32_t nrec = min(a.ctr[kCtrRecords], a.rec_cap);
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nrec; r += stride) {
    const RecMeta m = a.rec_meta[r];
    if (m.slice == kInvalidSlice) continue;
    const uint64_t key_hi = (uint64_t)a.rec_pay[r].gid << 32;
    const SliceDev& sl = a.slices[m.slice];
    const int tx0 = m.rx & 0xFFFF, tx1 = m.rx >> 16, ty0 = m.ry & 0xFFFF, ty1 = m.ry >> 16;
    uint32_t slot = m.ibase;
    for (int ty = ty0; ty <= ty1; ++ty) {
      for (int tx = tx0; tx <= tx1; ++tx, ++slot) {
        const uint32_t bin = (uint32_t)(sl.tile_base + ty * sl.ntx + tx);
        a.sort_key[a.bin_start[bin] + a.inst_rank[slot]] = key_hi | r;
      }
    }
  }
}

struct SortArgs {
  const BatchHdr* hdr;
  const uint32_t* bin_start;
  uint64_t* sort_key;
  uint32_t* list;
};

// Bitonic sorting network on [0, n) with every comparator ascending ("flip"
// form): positions >= n act as +infinity and are never touched.
template <typename Load, typename Store>
__device__ __forceinline__ void bitonic(int n, Load ld, Store st) {
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  const int half = n2 >> 1;
  for (int k = 2; k <= n2; k <<= 1) {
    const int hk = k >> 1;
    for (int i = threadIdx.x; i < half; i += blockDim.x) {
      const int blk = (i / hk) * k, off = i % hk;
      const int lo = blk + off, hi = blk + k - 1 - off;
      if (hi < n) {
        const uint64_t x = ld(lo), y = ld(hi);
        if (y < x) { st(lo, y); st(hi, x); }
      }
    }
    __syncthreads();
    for (int j = k >> 2; j >= 1; j >>= 1) {
      for (int i = threadIdx.x; i < half; i += blockDim.x) {
        const int lo = (i / j) * 2 * j + (i % j), hi = lo + j;
        if (hi < n) {
          const uint64_t x = ld(lo), y = ld(hi);
          if (y < x) { st(lo, y); st(hi, x); }
        }
      }
      __syncthreads();
    }
  }
}

// One workgroup per bin, grid-stride over the batch's bins.
__global__ __launch_bounds__(256) void k_bin_sort(SortArgs a) {
  __shared__ uint64_t keys[kBinSortCap];
  const int n_bins = a.hdr->n_bins;
  for (int bin = blockIdx.x; bin < n_bins; bin += gridDim.x) {
    const uint32_t start = a.bin_start[bin];
    const int n = (int)(a.bin_start[bin + 1] - start);
    if (n == 0) continue;
    uint64_t* gk = a.sort_key + start;
    if (n <= kBinSortCap) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) keys[i] = gk[i];
      __syncthreads();
      if (n > 1)
        bitonic(n, [&](int i) { return keys[i]; }, [&](int i, uint64_t v) { keys[i] = v; });
      for (int i = threadIdx.x; i < n; i += blockDim.x) a.list[start + i] = (uint32_t)keys[i];
    } else {
      // long list: the same network in global memory, this workgroup only
      bitonic(n, [&](int i) { return gk[i]; }, [&](int i, uint64_t v) { gk[i] = v; });
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += blockDim.x) a.list[start + i] = (uint32_t)gk[i];
    }
    __syncthreads();   // keys[] is reused by the next bin
  }
}

}  // namespace

hipError_t launch_scan_bins(const Workspace& ws, hipStream_t s) {
  k_scan_bins<<<1, kScanThreads, 0, s>>>(ws.d_hdr, ws.d_bin_count, ws.d_bin_start);
  return hipGetLastError();
}

hipError_t launch_scatter(const RenderConst& rc, const Workspace& ws, hipStream_t s) {
  ScatterArgs a{ws.d_rec_pay, ws.d_rec_meta, ws.d_slices, ws.d_ctr, ws.d_bin_start, ws.d_inst_rank,
                ws.d_sort_key, rc.rec_cap};
  int64_t blocks = ((int64_t)rc.rec_cap + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  k_scatter<<<(unsigned)blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_bin_sort(const RenderConst& rc, const Workspace& ws, const LaunchDims& d, hipStream_t s) {
  (void)rc;
  if (d.bins <= 0) return hipSuccess;
  SortArgs a{ws.d_hdr, ws.d_bin_start, ws.d_sort_key, ws.d_list};
  const int64_t blocks = d.bins < 8192 ? d.bins : 8192;
  k_bin_sort<<<(unsigned)blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace gp
