// Device-wide exclusive scan and stable LSD radix sort of (bin, record) pairs.
//
// The preprocess writes every (record, footprint tile) pair in Gaussian order
// (slots come from a scan, not from atomics).  A stable sort by bin therefore
// leaves each tile list in Gaussian-index order, the unique order the oracle
// also uses, without any per-list sort.  One pass of the sort:
//   hist:    each block counts the digits of its 4096-element tile (LDS atomics;
//            counts only, so their order does not matter);
//   scan:    exclusive scan of the digit-major [digit][block] count matrix;
//   scatter: each block re-reads its tile in 256-element chunks and gives every
//            element its stable rank among equal digits: within a wavefront by
//            matching digits bit by bit with ballots, across the block's four
//            wavefronts through per-digit counts in LDS.
// Element counts are read from the device, so launches sized for a capacity
// serve any batch (graph replay).
#include "gp_internal.h"

#include <algorithm>

namespace gp {
namespace {

constexpr int kScanItems = 8;                       // per thread
constexpr int kScanTile = 256 * kScanItems;         // per block

template <typename T>
__device__ __forceinline__ T zero_of() { return T{}; }

__device__ __forceinline__ uint2 add2(uint2 a, uint2 b) { return make_uint2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ uint32_t add2(uint32_t a, uint32_t b) { return a + b; }
__device__ __forceinline__ uint2 sub2(uint2 a, uint2 b) { return make_uint2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ uint32_t sub2(uint32_t a, uint32_t b) { return a - b; }

// Block-wide inclusive scan of one value per thread (256 threads).
template <typename T>
__device__ __forceinline__ T block_incl_scan(T v, T* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    T o = t >= d ? sh[t - d] : zero_of<T>();
    __syncthreads();
    if (t >= d) sh[t] = add2(sh[t], o);
    __syncthreads();
  }
  T r = sh[t];
  __syncthreads();
  return r;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_reduce(const T* __restrict__ in, const int32_t* __restrict__ n_ptr,
                                                     int64_t n_fixed, T* __restrict__ part) {
  __shared__ T sh[256];
  const int64_t n = n_ptr ? *n_ptr : n_fixed;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  T s = zero_of<T>();
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t j = base + (int64_t)i * 256 + threadIdx.x;
    if (j < n) s = add2(s, in[j]);
  }
  const T tot = block_incl_scan(s, sh);
  if (threadIdx.x == 255) part[blockIdx.x] = tot;
}

// Single-block exclusive scan of the block partials (any count).
template <typename T>
__global__ __launch_bounds__(256) void k_scan_parts(T* __restrict__ part, int nparts, T* __restrict__ total) {
  __shared__ T sh[256];
  __shared__ T chunk_total;
  T carry = zero_of<T>();
  for (int b0 = 0; b0 < nparts; b0 += 256) {
    const int j = b0 + threadIdx.x;
    const T v = j < nparts ? part[j] : zero_of<T>();
    const T inc = block_incl_scan(v, sh);
    if (j < nparts) part[j] = add2(carry, sub2(inc, v));
    if (threadIdx.x == 255) chunk_total = inc;
    __syncthreads();
    carry = add2(carry, chunk_total);
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_down(const T* __restrict__ in, const int32_t* __restrict__ n_ptr,
                                                   int64_t n_fixed, const T* __restrict__ part, T* __restrict__ out) {
  __shared__ T sh[256];
  const int64_t n = n_ptr ? *n_ptr : n_fixed;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = zero_of<T>();
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t j = base + i;
    v[i] = j < n ? in[j] : zero_of<T>();
    s = add2(s, v[i]);
  }
  const T inc = block_incl_scan(s, sh);
  T run = add2(part[blockIdx.x], sub2(inc, s));   // exclusive prefix of this thread
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t j = base + i;
    if (j < n) out[j] = run;
    run = add2(run, v[i]);
  }
}

}  // namespace

// Exclusive scan of n values (n on the host, or *d_n on the device when given;
// the launch covers max_n).  part must hold ceil(max_n / 2048) values.
template <typename T>
static hipError_t scan_impl(const T* in, T* out, const int32_t* d_n, int64_t max_n, T* part, T* total,
                            hipStream_t s) {
  const int64_t nb = (max_n + kScanTile - 1) / kScanTile;
  if (nb <= 0) return hipSuccess;
  k_scan_reduce<T><<<(unsigned)nb, 256, 0, s>>>(in, d_n, max_n, part);
  k_scan_parts<T><<<1, 256, 0, s>>>(part, (int)nb, total);
  k_scan_down<T><<<(unsigned)nb, 256, 0, s>>>(in, d_n, max_n, part, out);
  return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, const int32_t* d_n, int64_t max_n, uint32_t* part,
                           uint32_t* total, hipStream_t s) {
  return scan_impl<uint32_t>(in, out, d_n, max_n, part, total, s);
}

hipError_t launch_scan_u32x2(const uint2* in, uint2* out, const int32_t* d_n, int64_t max_n, uint2* part,
                             uint2* total, hipStream_t s) {
  return scan_impl<uint2>(in, out, d_n, max_n, part, total, s);
}

int64_t scan_parts_needed(int64_t max_n) { return (max_n + kScanTile - 1) / kScanTile + 1; }

// ---------------------------------------------------------------------------
// Radix sort
// ---------------------------------------------------------------------------
namespace {

constexpr int kSortTile = 4096;    // elements per block
constexpr int kSortChunk = 256;    // elements per block step (one per thread)
constexpr int kMaxDigitBits = 9;
constexpr int kMaxDigits = 1 << kMaxDigitBits;

struct RadixArgs {
  const uint32_t* key_in;
  const uint32_t* val_in;
  uint32_t* key_out;
  uint32_t* val_out;
  uint32_t* hist;         // [digits][nblocks]
  const uint32_t* count;  // element count (device)
  uint32_t cap;           // element capacity
  int nblocks, shift, bits;
};

__global__ __launch_bounds__(256) void k_radix_hist(RadixArgs a) {
  __shared__ uint32_t h[kMaxDigits];
  const int R = 1 << a.bits;
  for (int i = threadIdx.x; i < R; i += 256) h[i] = 0u;
  __syncthreads();
  const uint32_t n = min(*a.count, a.cap);
  const uint32_t tile = blockIdx.x;
  const uint32_t base = tile * kSortTile;
  // all loads first (independent, in flight together), then the counting
  constexpr int kPer = kSortTile / 256;
  uint32_t kv[kPer];
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const uint32_t j = base + c * 256 + threadIdx.x;
    kv[c] = j < n ? a.key_in[j] : 0u;
  }
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const uint32_t j = base + c * 256 + threadIdx.x;
    if (j < n) {
      const uint32_t d = (kv[c] >> a.shift) & (R - 1);
      // runs of equal digits are common (the high digit of consecutive pairs
      // is mostly the same slice): one atomic for a wavefront that agrees
      const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
      const uint64_t act = __builtin_amdgcn_read_exec();
      if (__builtin_amdgcn_ballot_w64(d == d0) == act) {
        if (__lane_id() == (uint32_t)__builtin_ctzll(act)) atomicAdd(&h[d0], (uint32_t)__popcll(act));
      } else {
        atomicAdd(&h[d], 1u);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += 256) a.hist[(size_t)i * a.nblocks + tile] = h[i];
}

// Scatter of one tile: the tile is first sorted stably by digit into LDS, then
// written out in that order, so consecutive threads store consecutive
// elements of each digit's run (coalesced) instead of every element landing
// on its own cache line.
//
// Wavefront w owns elements 1024 w .. 1024 w + 1023 of the tile (16 chunks of
// 64).  Each wavefront counts its digits; one block-wide scan turns the counts
// into the first local position of every (digit, wavefront); each wavefront
// then ranks its chunks on its own (lanes with equal digits matched by
// ballots, a per-wavefront running count per digit in LDS), with no
// workgroup barrier between chunks.
__global__ __launch_bounds__(256) void k_radix_scatter(RadixArgs a) {
  constexpr int kPerWave = kSortTile / 4;        // elements per wavefront
  constexpr int kChunks = kPerWave / 64;         // chunks per wavefront
  __shared__ uint32_t sk[kSortTile], sv[kSortTile];
  __shared__ uint32_t wrun[4][kMaxDigits];       // per-wavefront digit counts, then running positions
  __shared__ uint32_t loc[kMaxDigits];           // local run start of each digit (exclusive scan)
  __shared__ uint32_t glob[kMaxDigits];          // global start of this tile's run of each digit
  __shared__ uint32_t part[256];
  const int R = 1 << a.bits;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t n = min(*a.count, a.cap);
  const uint32_t tile = blockIdx.x;
  const uint32_t base = tile * kSortTile;
  if (base >= n) return;   // whole block past the end (uniform)
  const uint32_t tn = min((uint32_t)kSortTile, n - base);
  for (int i = threadIdx.x; i < R; i += 256) {
    glob[i] = a.hist[(size_t)i * a.nblocks + tile];
    wrun[0][i] = wrun[1][i] = wrun[2][i] = wrun[3][i] = 0u;
  }
  __syncthreads();
  // load (element 1024 w + 64 c + lane in register c) and count digits per wavefront
  uint32_t key[kChunks], val[kChunks];
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const uint32_t j = (uint32_t)(wave * kPerWave + c * 64 + lane);
    key[c] = j < tn ? a.key_in[base + j] : 0u;
    val[c] = j < tn ? a.val_in[base + j] : 0u;
  }
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const uint32_t j = (uint32_t)(wave * kPerWave + c * 64 + lane);
    if (j < tn) atomicAdd(&wrun[wave][(key[c] >> a.shift) & (R - 1)], 1u);
  }
  __syncthreads();
  // exclusive scan over digits of the tile's counts (two digits per thread),
  // then the first position of each (digit, wavefront)
  {
    const int i0 = 2 * threadIdx.x;
    uint32_t c0 = 0u, c1 = 0u;
    if (i0 < R) c0 = wrun[0][i0] + wrun[1][i0] + wrun[2][i0] + wrun[3][i0];
    if (i0 + 1 < R) c1 = wrun[0][i0 + 1] + wrun[1][i0 + 1] + wrun[2][i0 + 1] + wrun[3][i0 + 1];
    const uint32_t v = c0 + c1;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
      const uint32_t o = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0u;
      __syncthreads();
      part[threadIdx.x] += o;
      __syncthreads();
    }
    const uint32_t excl = part[threadIdx.x] - v;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = i0 + h;
      if (i >= R) continue;
      uint32_t p = h == 0 ? excl : excl + c0;
      loc[i] = p;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t cnt = wrun[w][i];
        wrun[w][i] = p;
        p += cnt;
      }
    }
  }
  __syncthreads();
  // stable ranks within each wavefront, chunk by chunk
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const bool valid = (uint32_t)(wave * kPerWave + c * 64 + lane) < tn;
    const uint32_t digit = valid ? (key[c] >> a.shift) & (R - 1) : 0u;
    uint64_t same = __ballot(valid);
    for (int b = 0; b < a.bits; ++b) {
      const uint64_t bb = __ballot((digit >> b) & 1u);
      same &= ((digit >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(same & lt_mask);
    uint32_t p = 0u;
    if (valid) {
      p = wrun[wave][digit] + rank;
      sk[p] = key[c];
      sv[p] = val[c];
    }
    // all lanes have read the running position before its leader advances it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) wrun[wave][digit] += (uint32_t)__popcll(same);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // write out in local order: runs of one digit go to consecutive addresses
  for (uint32_t p = threadIdx.x; p < tn; p += 256) {
    const uint32_t k = sk[p];
    const uint32_t d = (k >> a.shift) & (R - 1);
    const uint32_t dst = glob[d] + (p - loc[d]);
    a.key_out[dst] = k;
    a.val_out[dst] = sv[p];
  }
}

// Bin ranges from the sorted keys: [lo, hi) of every non-empty bin (the reset
// kernel zeroes both arrays first, so empty bins read as empty).
__global__ __launch_bounds__(256) void k_bin_ranges(const BatchHdr* __restrict__ hdr, const uint32_t* __restrict__ key,
                                                    const uint32_t* __restrict__ count, uint32_t cap,
                                                    uint32_t* __restrict__ lo, uint32_t* __restrict__ hi) {
  const uint32_t n = min(*count, cap);
  const uint32_t n_bins = (uint32_t)hdr->n_bins;
  // four consecutive keys per thread (one 16-byte load); the neighbours across
  // a thread boundary come from the adjacent lanes, across a wavefront
  // boundary from memory
  const uint32_t n4 = n / 4;
  const int lane = threadIdx.x & 63;
  for (uint32_t q0 = blockIdx.x * 256 + (threadIdx.x & ~63u); q0 < n4; q0 += gridDim.x * 256) {
    const uint32_t q = q0 + lane;
    uint4 k4 = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
    if (q < n4) k4 = reinterpret_cast<const uint4*>(key)[q];
    uint32_t prev = __shfl_up(k4.w, 1, 64), next = __shfl_down(k4.x, 1, 64);
    if (lane == 0) prev = q == 0 ? 0xFFFFFFFEu : key[4 * q - 1];
    if (lane == 63 || q + 1 >= n4) next = 4 * q + 4 < n ? key[4 * q + 4] : 0xFFFFFFFEu;
    if (q < n4) {
      const uint32_t kk[6] = {prev, k4.x, k4.y, k4.z, k4.w, next};
#pragma unroll
      for (int i = 1; i <= 4; ++i) {
        const uint32_t b = kk[i];
        if (b >= n_bins) continue;   // slots of an overflowed Gaussian (sorted last)
        if (kk[i - 1] != b) lo[b] = 4 * q + i - 1;
        if (kk[i + 1] != b) hi[b] = 4 * q + i;
      }
    }
  }
  // the last n % 4 keys
  if (blockIdx.x == 0 && threadIdx.x < (n & 3u)) {
    const uint32_t p = 4 * n4 + threadIdx.x;
    const uint32_t b = key[p];
    if (b < n_bins) {
      if (p == 0 || key[p - 1] != b) lo[b] = p;
      if (p + 1 == n || key[p + 1] != b) hi[b] = p + 1;
    }
  }
}

}  // namespace

int radix_passes(int bits) { return bits <= 0 ? 0 : (bits + kMaxDigitBits - 1) / kMaxDigitBits; }

int64_t radix_hist_entries(int bits, int64_t cap) {
  const int passes = radix_passes(bits);
  if (passes == 0) return 1;
  const int db = (bits + passes - 1) / passes;
  return ((int64_t)1 << db) * ((cap + kSortTile - 1) / kSortTile);
}

// Stable sort of `count` (device) pairs by the low `bits` bits of the key.
// Ping-pongs between (k0, v0) and (k1, v1); returns in *k_out / *v_out the
// buffers that hold the result.
hipError_t launch_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* d_count,
                             int64_t cap, int bits, uint32_t* hist, uint32_t* scan_part, hipStream_t s,
                             uint32_t** k_out, uint32_t** v_out) {
  const int passes = radix_passes(bits);
  *k_out = k0;
  *v_out = v0;
  if (passes == 0 || cap <= 0) return hipSuccess;
  const int db = (bits + passes - 1) / passes;
  const int nblocks = (int)((cap + kSortTile - 1) / kSortTile);
  uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * db;
    const int pb = std::min(db, bits - shift);
    RadixArgs a{ki, vi, ko, vo, hist, d_count, (uint32_t)cap, nblocks, shift, pb};
    k_radix_hist<<<nblocks, 256, 0, s>>>(a);
    hipError_t e = launch_scan_u32(hist, hist, nullptr, ((int64_t)1 << pb) * nblocks, scan_part, nullptr, s);
    if (e != hipSuccess) return e;
    k_radix_scatter<<<nblocks, 256, 0, s>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  *k_out = ki;
  *v_out = vi;
  return hipSuccess;
}

hipError_t launch_bin_ranges(const BatchHdr* hdr, const uint32_t* key, const uint32_t* d_count, int64_t cap,
                             uint32_t* lo, uint32_t* hi, hipStream_t s) {
  int64_t blocks = (cap + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 8192 ? 8192 : blocks);
  k_bin_ranges<<<(unsigned)blocks, 256, 0, s>>>(hdr, key, d_count, (uint32_t)cap, lo, hi);
  return hipGetLastError();
}

}  // namespace gp
