// Device-wide exclusive scan and stable LSD radix sort of (bin, record) pairs.
//
// The preprocess writes every (record, footprint tile) pair in Gaussian order
// (slots come from a scan, not from atomics).  A stable sort by bin therefore
// leaves each tile list in Gaussian-index order, the unique order the oracle
// also uses, without any per-list sort.  One pass of the sort:
//   hist:    each block counts the digits of its 8192-element tile (LDS atomics;
//            counts only, so their order does not matter);
//   scan:    exclusive scan of every digit's row of the [digit][block] count
//            matrix, and the rows' totals (the scatter scans those);
//   scatter: each block re-reads its tile and gives every element its stable
//            rank among equal digits: within a wavefront by matching digits
//            bit by bit with ballots, across the block's eight wavefronts
//            through per-digit counts in LDS.
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
__device__ __forceinline__ uint2 shfl_up2(uint2 v, int d) {
  return make_uint2(__shfl_up(v.x, d, 64), __shfl_up(v.y, d, 64));
}
__device__ __forceinline__ uint32_t shfl_up2(uint32_t v, int d) { return __shfl_up(v, d, 64); }

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
__global__ __launch_bounds__(256) void k_scan_down(const T* in, const int32_t* __restrict__ n_ptr, int64_t n_fixed,
                                                   const T* __restrict__ part, T* out) {
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

// Exclusive scan of up to kSmallScan values by one block: thread t takes 8
// consecutive values (one 64-byte run, so each wavefront's loads are
// contiguous), then a shuffle scan per wavefront and the wavefront totals.
// in and out may be the same array: every value is read before the barrier.
constexpr int kSmallScan = 8192;

template <typename T>
__global__ __launch_bounds__(1024) void k_scan_single(const T* in, const int32_t* __restrict__ n_ptr, int64_t n_fixed,
                                                      T* out, T* __restrict__ total) {
  constexpr int kPer = kSmallScan / 1024;
  __shared__ T wsum[16];
  const int64_t n = n_ptr ? *n_ptr : n_fixed;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j0 = (int64_t)threadIdx.x * kPer;
  T v[kPer];
  T sum = zero_of<T>();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    v[k] = j0 + k < n ? in[j0 + k] : zero_of<T>();
    sum = add2(sum, v[k]);
  }
  T inc = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T u = shfl_up2(inc, d);
    if (lane >= d) inc = add2(inc, u);
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  T run = sub2(inc, sum);
  for (int w = 0; w < wave; ++w) run = add2(run, wsum[w]);
  if (threadIdx.x == 1023 && total) *total = add2(run, sum);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (j0 + k < n) out[j0 + k] = run;
    run = add2(run, v[k]);
  }
}

}  // namespace

// Exclusive scan of n values (n on the host, or *d_n on the device when given;
// the launch covers max_n).  part must hold ceil(max_n / 2048) values (unused
// when max_n fits one block).
template <typename T>
static hipError_t scan_impl(const T* in, T* out, const int32_t* d_n, int64_t max_n, T* part, T* total,
                            hipStream_t s) {
  const int64_t nb = (max_n + kScanTile - 1) / kScanTile;
  if (nb <= 0) return hipSuccess;
  if (max_n <= kSmallScan) {
    k_scan_single<T><<<1, 1024, 0, s>>>(in, d_n, max_n, out, total);
    return hipGetLastError();
  }
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

constexpr int kSortThreads = 512;                         // threads per block
constexpr int kSortWaves = kSortThreads / 64;
// elements per wavefront: 1,024 (8,192 per block), or 256 (2,048 per block)
// for sorts of at most kSmallSort pairs, which would otherwise run on a few
// dozen blocks (a training batch's 0.5 M pairs: 59 tiles of 8,192)
constexpr int kPerWaveBig = 1024, kPerWaveSmall = 256;
constexpr int64_t kSmallSort = 1 << 21;
constexpr int kMaxDigitBits = 9;
constexpr int kMaxDigits = 1 << kMaxDigitBits;
constexpr int kDigPerThread = kMaxDigits / kSortThreads;  // 1 or 2

// LDS slot of a digit's counter: the low three bits are xor-ed with bits 6-8,
// so that digits 64 or 256 apart (the same tile on slices of the other
// parity, four tile rows down) fall in different banks.
__device__ __forceinline__ uint32_t dslot(uint32_t d) { return d ^ ((d >> 6) & 7u); }


struct RadixArgs {
  const uint32_t* key_in;
  const uint32_t* val_in;
  uint32_t* key_out;
  uint32_t* val_out;
  uint32_t* hist;         // [digits][nblocks]
  const uint32_t* rowtot; // [digits] row totals of hist
  const uint32_t* count;  // element count (device)
  const uint32_t* count2; // a second bound on it (device), or null
  uint32_t cap;           // element capacity
  int nblocks, shift, bits;
};

__device__ __forceinline__ uint32_t sort_count(const RadixArgs& a) {
  const uint32_t n = min(*a.count, a.cap);
  return a.count2 ? min(n, *a.count2) : n;
}

template <int PW>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(RadixArgs a) {
  constexpr int kSortTile = kSortWaves * PW;
  __shared__ uint32_t h[kMaxDigits];
  const int R = 1 << a.bits;
  for (int i = threadIdx.x; i < R; i += kSortThreads) h[i] = 0u;
  __syncthreads();
  const uint32_t n = sort_count(a);
  // consecutive tiles on one XCD (workgroups go to the eight XCDs in turn):
  // their counts share cache lines of the [digit][tile] matrix, which then
  // merge in that XCD's L2 instead of being written partially by eight
  const uint32_t per = (a.nblocks + 7) / 8;
  const uint32_t tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= (uint32_t)a.nblocks) return;
  const uint32_t base = tile * kSortTile;
  // all loads first (independent, in flight together), then the counting
  constexpr int kPer = kSortTile / kSortThreads;
  uint32_t kv[kPer];
  const bool full = base + kSortTile <= n;
  if (full) {
#pragma unroll
    for (int c = 0; c < kPer; ++c) kv[c] = a.key_in[base + c * kSortThreads + threadIdx.x];
  } else {
#pragma unroll
    for (int c = 0; c < kPer; ++c) {
      const uint32_t j = base + c * kSortThreads + threadIdx.x;
      kv[c] = j < n ? a.key_in[j] : 0u;
    }
  }
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const uint32_t j = base + c * kSortThreads + threadIdx.x;
    if (j < n) {
      const uint32_t d = (kv[c] >> a.shift) & (R - 1);
      // runs of equal digits are common (the high digit of consecutive pairs
      // is mostly the same slice): one atomic for a wavefront that agrees
      const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
      const uint64_t act = __builtin_amdgcn_read_exec();
      if (__builtin_amdgcn_ballot_w64(d == d0) == act) {
        if (__lane_id() == (uint32_t)__builtin_ctzll(act)) atomicAdd(&h[dslot(d0)], (uint32_t)__popcll(act));
      } else {
        atomicAdd(&h[dslot(d)], 1u);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += kSortThreads) a.hist[(size_t)i * a.nblocks + tile] = h[dslot(i)];
}

// Scatter of one tile: the tile is first sorted stably by digit into LDS, then
// written out in that order, so consecutive threads store consecutive
// elements of each digit's run (coalesced) instead of every element landing
// on its own cache line.
//
// Wavefront w owns elements 1024 w .. 1024 w + 1023 of the tile (16 chunks of
// 64).  Each wavefront matches the digits of each chunk (lanes with equal
// digits found bit by bit with ballots); the lowest lane of each distinct
// digit adds the chunk's count to the wavefront's counter in LDS and gets back
// the digit's count in the earlier chunks, so every element knows its offset
// within its (digit, wavefront) run.  One block-wide scan turns the counts
// into the first local position of every (digit, wavefront), and the elements
// go to their places with no further synchronisation.  Every global load
// (elements and the block's digit offsets) is issued before the first wait;
// the digit width is a template parameter so that the matching unrolls; LDS
// is 80 KB, two blocks per CU.
template <int BITS, int PW>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(RadixArgs a) {
  constexpr int kPerWave = PW, kSortTile = kSortWaves * PW;
  constexpr int kChunks = kPerWave / 64;         // chunks per wavefront
  constexpr int R = 1 << BITS;
  __shared__ uint32_t sk[kSortTile], sv[kSortTile];
  __shared__ uint32_t wrun[kSortWaves][kMaxDigits];   // per-wavefront digit counts, then running positions
  uint32_t* const wtot = sk;                     // the wavefront totals of the scan (before sk is used)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t n = sort_count(a);
  // consecutive tiles on one XCD, as in the histogram: a digit's runs of
  // adjacent tiles are adjacent in the output, and their shared lines then
  // merge in that XCD's L2
  const uint32_t per = (a.nblocks + 7) / 8;
  const uint32_t tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= (uint32_t)a.nblocks) return;
  const uint32_t base = tile * kSortTile;
  if (base >= n) return;   // whole block past the end (uniform)
  const uint32_t tn = min((uint32_t)kSortTile, n - base);
  const bool full = tn == (uint32_t)kSortTile;
  // every global load of the block is issued before anything waits on one
  uint32_t key[kChunks], val[kChunks];
  if (full) {
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      const uint32_t j = (uint32_t)(wave * kPerWave + c * 64 + lane);
      key[c] = a.key_in[base + j];
      val[c] = a.val_in[base + j];
    }
  } else {
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      const uint32_t j = (uint32_t)(wave * kPerWave + c * 64 + lane);
      key[c] = j < tn ? a.key_in[base + j] : 0u;
      val[c] = j < tn ? a.val_in[base + j] : 0u;
    }
  }
  // the digits' offsets for this tile and row totals wait in the tail of sk
  // (unused until the ranking) rather than in registers through the counting
  uint32_t* const sg = sk + kSortTile - 2 * kMaxDigits;
  uint32_t* const srt = sk + kSortTile - kMaxDigits;
#pragma unroll
  for (int h = 0; h < kDigPerThread; ++h) {
    const int i = kDigPerThread * threadIdx.x + h;
    sg[i] = i < R ? a.hist[(size_t)i * a.nblocks + tile] : 0u;
    srt[i] = i < R ? a.rowtot[i] : 0u;
  }
  for (int i = threadIdx.x; i < R; i += kSortThreads)
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) wrun[w][i] = 0u;
  __syncthreads();
  // lanes with the same digit: for every bit, the ballot of that bit, or its
  // complement where the lane's bit is 0.  The lowest lane of each distinct
  // digit of a chunk adds the chunk's count to the wavefront's counter; the
  // value it returns (the digit's count in the wavefront's earlier chunks)
  // plus a lane's rank among its equals is the lane's offset within the
  // wavefront's run of that digit (10 bits, three chunks per register).
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  constexpr int kPacked = (kChunks + 2) / 3;
  uint32_t pk[kPacked];
#pragma unroll
  for (int q = 0; q < kPacked; ++q) pk[q] = 0u;
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const bool valid = (uint32_t)(wave * kPerWave + c * 64 + lane) < tn;
    const uint32_t digit = valid ? (key[c] >> a.shift) & (R - 1) : 0u;
    const uint64_t vb = __ballot(valid);
    uint32_t same_lo = (uint32_t)vb, same_hi = (uint32_t)(vb >> 32);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const int32_t mt = (int32_t)(digit << (31 - b)) >> 31;   // -1 where the lane's bit is set
      const uint64_t bb = __builtin_amdgcn_ballot_w64(mt != 0);
      same_lo &= ~((uint32_t)bb ^ (uint32_t)mt);
      same_hi &= ~((uint32_t)(bb >> 32) ^ (uint32_t)mt);
    }
    const uint64_t same = ((uint64_t)same_hi << 32) | same_lo;
    const uint32_t rank = (uint32_t)__popcll(same & lt_mask);
    uint32_t old = 0u;
    if (valid && rank == 0u) old = atomicAdd(&wrun[wave][dslot(digit)], (uint32_t)__popcll(same));
    const int leader = valid ? __builtin_ctzll(same) : lane;
    const uint32_t off = __shfl(old, leader, 64) + rank;
    pk[c / 3] |= (off & 1023u) << (10 * (c % 3));
  }
  __syncthreads();
  // exclusive scans over digits of the tile's counts and of the digits' totals
  // (thread t owns digits kDigPerThread t ...): a shuffle scan within each
  // wavefront, then the totals of the wavefronts before it.  A digit's global
  // start for this tile is the total of the smaller digits plus the digit's
  // count in the earlier tiles (its row of the count matrix, scanned).
  uint32_t gofs[kDigPerThread];
  {
    uint32_t cw[kDigPerThread][kSortWaves], c[kDigPerThread];
    uint32_t v = 0u, vr = 0u, g[kDigPerThread], rt[kDigPerThread];
#pragma unroll
    for (int h = 0; h < kDigPerThread; ++h) {
      g[h] = sg[kDigPerThread * threadIdx.x + h];
      rt[h] = srt[kDigPerThread * threadIdx.x + h];
      vr += rt[h];
    }
#pragma unroll
    for (int h = 0; h < kDigPerThread; ++h) {
      const int i = kDigPerThread * threadIdx.x + h;
      c[h] = 0u;
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) {
        cw[h][w] = i < R ? wrun[w][dslot(i)] : 0u;
        c[h] += cw[h][w];
      }
      v += c[h];
    }
    uint32_t inc = v, incr = vr;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t u = __shfl_up(inc, d, 64), ur = __shfl_up(incr, d, 64);
      if (lane >= d) {
        inc += u;
        incr += ur;
      }
    }
    if (lane == 63) {
      wtot[wave] = inc;
      wtot[kSortWaves + wave] = incr;
    }
    __syncthreads();
    uint32_t p = inc - v, pr = incr - vr;
    for (int w = 0; w < wave; ++w) {
      p += wtot[w];
      pr += wtot[kSortWaves + w];
    }
#pragma unroll
    for (int h = 0; h < kDigPerThread; ++h) {
      const int i = kDigPerThread * threadIdx.x + h;
      gofs[h] = g[h] + pr - p;
      pr += rt[h];
      if (i < R) {
        uint32_t q = p;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
          wrun[w][dslot(i)] = q;
          q += cw[h][w];
        }
      }
      p += c[h];
    }
  }
  __syncthreads();
  // every element to its place in the tile's local order: the start of its
  // (digit, wavefront) run plus its offset in it
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const bool valid = (uint32_t)(wave * kPerWave + c * 64 + lane) < tn;
    if (valid) {
      const uint32_t slot = dslot((key[c] >> a.shift) & (R - 1));
      const uint32_t p = wrun[wave][slot] + ((pk[c / 3] >> (10 * (c % 3))) & 1023u);
      sk[p] = key[c];
      sv[p] = val[c];
    }
  }
  __syncthreads();
  // the running positions are done with: their first row now holds the offsets
  uint32_t* const go = wrun[0];
#pragma unroll
  for (int h = 0; h < kDigPerThread; ++h) {
    const int i = kDigPerThread * threadIdx.x + h;
    if (i < R) go[dslot(i)] = gofs[h];
  }
  __syncthreads();
  // write out in local order: runs of one digit go to consecutive addresses
#pragma unroll
  for (int c = 0; c < kSortTile / kSortThreads; ++c) {
    const uint32_t p = c * kSortThreads + threadIdx.x;
    if (p < tn) {
      const uint32_t k = sk[p];
      const uint32_t dst = go[dslot((k >> a.shift) & (R - 1))] + p;
      a.key_out[dst] = k;
      a.val_out[dst] = sv[p];
    }
  }
}

// Exclusive scan of every digit's row of the [digit][block] count matrix, in
// place, and the row's total (one block per digit).  The scatter adds the
// totals of the smaller digits itself.  The row passes through LDS in chunks
// of 4096 entries (unrolled, coalesced loads and stores); thread t scans
// entries 16 t .. 16 t + 15 of a chunk.
__global__ __launch_bounds__(256) void k_hist_rowscan(uint32_t* __restrict__ hist, int nblocks,
                                                      uint32_t* __restrict__ rowtot) {
  constexpr int kChunk = 4096, kPer = kChunk / 256;
  __shared__ uint32_t buf[kChunk];
  __shared__ uint32_t wsum[4];
  uint32_t* row = hist + (size_t)blockIdx.x * nblocks;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t carry = 0u;
  for (int c0 = 0; c0 < nblocks; c0 += kChunk) {
    const int m = min(kChunk, nblocks - c0);
    uint32_t ld[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int jj = k * 256 + (int)threadIdx.x;
      ld[k] = jj < m ? row[c0 + jj] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) buf[k * 256 + threadIdx.x] = ld[k];
    __syncthreads();
    uint32_t v[kPer], sum = 0u;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      v[k] = buf[kPer * threadIdx.x + k];
      sum += v[k];
    }
    uint32_t inc = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t u = __shfl_up(inc, d, 64);
      if (lane >= d) inc += u;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t run = carry + inc - sum;
    for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      buf[kPer * threadIdx.x + k] = run;
      run += v[k];
    }
    carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int jj = k * 256 + (int)threadIdx.x;
      if (jj < m) row[c0 + jj] = buf[jj];
    }
    __syncthreads();   // buf and wsum are rewritten by the next chunk
  }
  if (threadIdx.x == 0) rowtot[blockIdx.x] = carry;
}

// Bin ranges from the sorted keys: [lo, hi) of every non-empty bin (the reset
// kernel zeroes both arrays first, so empty bins read as empty).
__global__ __launch_bounds__(256) void k_bin_ranges(const BatchHdr* __restrict__ hdr, const uint32_t* __restrict__ key,
                                                    const uint32_t* __restrict__ count,
                                                    const uint32_t* __restrict__ count2, uint32_t cap,
                                                    uint32_t* __restrict__ lo, uint32_t* __restrict__ hi) {
  uint32_t n = min(*count, cap);
  if (count2) n = min(n, *count2);
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

static int64_t sort_tile(int64_t cap) { return kSortWaves * (cap <= kSmallSort ? kPerWaveSmall : kPerWaveBig); }

// Count-matrix entries for a sort of any extent up to `cap` (a smaller extent
// may take the small tiles and so more of them): the most tiles over both
// regimes, times the digits of a pass, plus the row totals.
int64_t radix_hist_entries(int bits, int64_t cap) {
  const int passes = radix_passes(bits);
  if (passes == 0) return 1;
  const int db = (bits + passes - 1) / passes;
  const int64_t small_tile = (int64_t)kSortWaves * kPerWaveSmall, big_tile = (int64_t)kSortWaves * kPerWaveBig;
  const int64_t small_tiles = (std::min(cap, kSmallSort) + small_tile - 1) / small_tile;
  const int64_t big_tiles = cap > kSmallSort ? (cap + big_tile - 1) / big_tile : 0;
  return ((int64_t)1 << db) * std::max(small_tiles, big_tiles) + kMaxDigits;   // matrix, row totals
}

template <int PW>
static void launch_scatter(int pb, unsigned grid, const RadixArgs& a, hipStream_t s) {
  switch (pb) {
    case 1: k_radix_scatter<1, PW><<<grid, kSortThreads, 0, s>>>(a); break;
    case 2: k_radix_scatter<2, PW><<<grid, kSortThreads, 0, s>>>(a); break;
    case 3: k_radix_scatter<3, PW><<<grid, kSortThreads, 0, s>>>(a); break;
    case 4: k_radix_scatter<4, PW><<<grid, kSortThreads, 0, s>>>(a); break;
    case 5: k_radix_scatter<5, PW><<<grid, kSortThreads, 0, s>>>(a); break;
    case 6: k_radix_scatter<6, PW><<<grid, kSortThreads, 0, s>>>(a); break;
    case 7: k_radix_scatter<7, PW><<<grid, kSortThreads, 0, s>>>(a); break;
    case 8: k_radix_scatter<8, PW><<<grid, kSortThreads, 0, s>>>(a); break;
    default: k_radix_scatter<9, PW><<<grid, kSortThreads, 0, s>>>(a); break;
  }
}

// Stable sort of min(*count, *count2, cap) pairs (count2 may be null) by the
// low `bits` bits of the key.
// Ping-pongs between (k0, v0) and (k1, v1); returns in *k_out / *v_out the
// buffers that hold the result.
hipError_t launch_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* d_count,
                             const uint32_t* d_count2, int64_t cap, int bits, uint32_t* hist, uint32_t* scan_part, hipStream_t s,
                             uint32_t** k_out, uint32_t** v_out) {
  const int passes = radix_passes(bits);
  *k_out = k0;
  *v_out = v0;
  if (passes == 0 || cap <= 0) return hipSuccess;
  const int db = (bits + passes - 1) / passes;
  const int64_t tile = sort_tile(cap);
  const bool small = tile < (int64_t)kSortWaves * kPerWaveBig;
  const int nblocks = (int)((cap + tile - 1) / tile);
  uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * db;
    const int pb = std::min(db, bits - shift);
    uint32_t* rowtot = hist + ((size_t)1 << db) * nblocks;
    RadixArgs a{ki, vi, ko, vo, hist, rowtot, d_count, d_count2, (uint32_t)cap, nblocks, shift, pb};
    const unsigned grid = 8u * (unsigned)((nblocks + 7) / 8);
    if (small) {
      k_radix_hist<kPerWaveSmall><<<grid, kSortThreads, 0, s>>>(a);
      k_hist_rowscan<<<1 << pb, 256, 0, s>>>(hist, nblocks, rowtot);
      launch_scatter<kPerWaveSmall>(pb, grid, a, s);
    } else {
      k_radix_hist<kPerWaveBig><<<grid, kSortThreads, 0, s>>>(a);
      k_hist_rowscan<<<1 << pb, 256, 0, s>>>(hist, nblocks, rowtot);
      launch_scatter<kPerWaveBig>(pb, grid, a, s);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  *k_out = ki;
  *v_out = vi;
  return hipSuccess;
}

hipError_t launch_bin_ranges(const BatchHdr* hdr, const uint32_t* key, const uint32_t* d_count,
                             const uint32_t* d_count2, int64_t cap, uint32_t* lo, uint32_t* hi, hipStream_t s) {
  int64_t blocks = (cap + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 8192 ? 8192 : blocks);
  k_bin_ranges<<<(unsigned)blocks, 256, 0, s>>>(hdr, key, d_count, d_count2, (uint32_t)cap, lo, hi);
  return hipGetLastError();
}

}  // namespace gp
