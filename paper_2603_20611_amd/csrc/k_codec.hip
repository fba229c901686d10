// Morton-ordered fixed-point codec of a Gaussian set (Sec. 4.3, "Quantization
// and compression": Gaussians sorted along the Morton curve; positions
// normalised to the bounding box with 14 bits per axis; intensity 12 bits on
// [0, 1]; log-scales 12 bits; quaternions on the positive half-sphere, 12 bits
// per component; intensities normalised to [0, 1] by their maximum).  The
// codes are stored as 11 uint16 planes and decoded in
// registers by the renderer (attribute type GP_QM), 22 bytes per Gaussian.
//
// Every decision that yields a code is a fixed binary32 sequence (contraction
// off): code = floor(((v - lo) / (hi - lo)) * (levels - 1) + 0.5), clamped;
// decoding is lo + code * ((hi - lo) / (levels - 1)).
//
// Encoding: bounds (order-independent min/max through ordered-integer
// atomics) -> codes and the 42-bit Morton key -> a stable LSD radix sort of
// (key, index) in two stages (the low 32 bits, then the high 10 bits of the
// keys gathered in that order) -> the code planes gathered in Morton order.
#include "gp_internal.h"

#include <algorithm>
#include <type_traits>
#include <vector>

namespace gp {
namespace {

constexpr float kPosLevels1 = 16383.0f;   // 2^14 - 1
constexpr float kAttrLevels1 = 4095.0f;   // 2^12 - 1

__device__ __forceinline__ uint32_t ordered(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unordered(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// Parameter row r (0..10) of Gaussian j: rows 0..2 from the means, 3..10 from
// the attributes.
__device__ __forceinline__ float prow(const float* m, const float* at, int64_t stride, int r, int64_t j) {
  return r < 3 ? m[r * stride + j] : at[(r - 3) * stride + j];
}

// bounds[0..2] = min mu, [3..5] = max mu, [6] = min l, [7] = max l, [8] = max
// intensity (ordered ints)
__global__ __launch_bounds__(256) void k_codec_bounds(const float* __restrict__ m, const float* __restrict__ at,
                                                      int64_t n, int64_t stride, uint32_t* __restrict__ bounds) {
  __shared__ uint32_t smin[4][5], smax[4][5];
  uint32_t mn[5] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[5] = {0u, 0u, 0u, 0u, 0u};
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float v = prow(m, at, stride, a, j);
      if (isfinite(v)) {
        mn[a] = min(mn[a], ordered(v));
        mx[a] = max(mx[a], ordered(v));
      }
    }
#pragma unroll
    for (int a = 3; a < 6; ++a) {
      const float v = prow(m, at, stride, a, j);
      if (isfinite(v)) {
        mn[3] = min(mn[3], ordered(v));
        mx[3] = max(mx[3], ordered(v));
      }
    }
    const float al = prow(m, at, stride, 10, j);
    if (isfinite(al)) mx[4] = max(mx[4], ordered(al));
  }
#pragma unroll
  for (int i = 0; i < 5; ++i)
    for (int o = 32; o > 0; o >>= 1) {
      mn[i] = min(mn[i], (uint32_t)__shfl_xor((int)mn[i], o));
      mx[i] = max(mx[i], (uint32_t)__shfl_xor((int)mx[i], o));
    }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int i = 0; i < 5; ++i) {
      smin[wave][i] = mn[i];
      smax[wave][i] = mx[i];
    }
  __syncthreads();
  if (threadIdx.x < 5) {
    const int i = threadIdx.x;
    uint32_t a = min(min(smin[0][i], smin[1][i]), min(smin[2][i], smin[3][i]));
    uint32_t b = max(max(smax[0][i], smax[1][i]), max(smax[2][i], smax[3][i]));
    if (i < 4) atomicMin(&bounds[i < 3 ? i : 6], a);
    atomicMax(&bounds[i < 3 ? 3 + i : (i == 3 ? 7 : 8)], b);
  }
}

__global__ void k_codec_header(const uint32_t* __restrict__ bounds, float* __restrict__ hdr) {
  const int i = threadIdx.x;
  if (i >= 9) return;
  const bool is_min = (i < 3) || i == 6;
  const uint32_t k = bounds[i];
  // no finite value: the min stays at all-ones, the max at zero
  const bool empty = is_min ? (k == 0xFFFFFFFFu) : (k == 0u);
  float v = empty ? 0.0f : unordered(k);
  if (i == 8) v = fmaxf(v, 0.0f);   // intensities are coded on [0, amax]
  hdr[i] = v;
}

__device__ __forceinline__ uint32_t code_of(float v, float lo, float hi, float levels1) {
#pragma clang fp contract(off)
  if (!(hi > lo)) return 0u;
  const float c = floorf(((v - lo) / (hi - lo)) * levels1 + 0.5f);
  if (!isfinite(c)) return 0u;
  return (uint32_t)fminf(fmaxf(c, 0.0f), levels1);
}

__device__ __forceinline__ uint64_t spread3_64(uint32_t v) {
  uint64_t x = v & 0x3FFFu;
  x = (x | (x << 16)) & 0x0000FF0000FFull;
  x = (x | (x << 8)) & 0x00F00F00F00Full;
  x = (x | (x << 4)) & 0x0C30C30C30C3ull;
  x = (x | (x << 2)) & 0x249249249249ull;
  return x;
}

__global__ __launch_bounds__(256) void k_codec_codes(const float* __restrict__ m, const float* __restrict__ at,
                                                     int64_t n, int64_t stride,
                                                     const float* __restrict__ hdr, uint16_t* __restrict__ codes,
                                                     uint32_t* __restrict__ key_lo, uint32_t* __restrict__ key_hi,
                                                     uint32_t* __restrict__ idx) {
#pragma clang fp contract(off)
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  uint32_t c[11];
#pragma unroll
  for (int a = 0; a < 3; ++a) c[a] = code_of(prow(m, at, stride, a, j), hdr[a], hdr[3 + a], kPosLevels1);
#pragma unroll
  for (int a = 0; a < 3; ++a) c[3 + a] = code_of(prow(m, at, stride, 3 + a, j), hdr[6], hdr[7], kAttrLevels1);
  float q[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) q[r] = prow(m, at, stride, 6 + r, j);
  const float n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
  const float rn = sqrtf(n2);
  float qn[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) qn[r] = q[r] / rn;
  const bool flip = qn[0] < 0.0f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float v = flip ? -qn[r] : qn[r];
    const float cc = floorf(((v + 1.0f) * 0.5f) * kAttrLevels1 + 0.5f);
    c[6 + r] = isfinite(cc) ? (uint32_t)fminf(fmaxf(cc, 0.0f), kAttrLevels1) : 0u;
  }
  c[10] = code_of(fmaxf(prow(m, at, stride, 10, j), 0.0f), 0.0f, hdr[8], kAttrLevels1);
#pragma unroll
  for (int r = 0; r < 11; ++r) codes[r * n + j] = (uint16_t)c[r];
  const uint64_t key = spread3_64(c[0]) | (spread3_64(c[1]) << 1) | (spread3_64(c[2]) << 2);
  key_lo[j] = (uint32_t)key;
  key_hi[j] = (uint32_t)(key >> 32);
  idx[j] = (uint32_t)j;
}

__global__ __launch_bounds__(256) void k_codec_gather_u32(const uint32_t* __restrict__ src,
                                                          const uint32_t* __restrict__ perm, int64_t n,
                                                          uint32_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

__global__ __launch_bounds__(256) void k_codec_gather_codes(const uint16_t* __restrict__ src,
                                                            const uint32_t* __restrict__ perm, int64_t n,
                                                            int64_t stride_out, uint16_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = perm[i];
#pragma unroll
  for (int r = 0; r < 11; ++r) dst[r * stride_out + i] = src[r * n + j];
}

__global__ void k_codec_init_bounds(uint32_t* b) {
  const int i = threadIdx.x;
  if (i < 9) b[i] = ((i < 3) || i == 6) ? 0xFFFFFFFFu : 0u;
}

}  // namespace

hipError_t launch_encode(const float* means, const float* attrs, int64_t n, int64_t stride, uint16_t* codes_out,
                         int64_t stride_out, uint32_t* perm_out, float* d_hdr, const CodecScratch& t, hipStream_t s) {
  k_codec_init_bounds<<<1, 64, 0, s>>>(t.bounds);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) {
    if (e == hipSuccess) k_codec_header<<<1, 64, 0, s>>>(t.bounds, d_hdr);
    return e == hipSuccess ? hipGetLastError() : e;
  }
  const unsigned blocks = (unsigned)((n + 255) / 256);
  e = launch_fill_u32(t.count, (uint32_t)n, 1, s);
  if (e != hipSuccess) return e;
  k_codec_bounds<<<std::min(blocks, 2048u), 256, 0, s>>>(means, attrs, n, stride, t.bounds);
  k_codec_header<<<1, 64, 0, s>>>(t.bounds, d_hdr);
  k_codec_codes<<<blocks, 256, 0, s>>>(means, attrs, n, stride, d_hdr, t.codes, t.key_lo, t.key_hi, t.idx);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // stable sort by the low 32 key bits, then by the high 10 (keys gathered in that order)
  uint32_t *k_sorted = nullptr, *i_sorted = nullptr;
  e = launch_radix_sort(t.key_lo, t.idx, t.key2, t.val2, t.count, nullptr, n, 32, t.hist, t.scan_part, s, &k_sorted, &i_sorted);
  if (e != hipSuccess) return e;
  uint32_t* hi_perm = (k_sorted == t.key_lo) ? t.key2 : t.key_lo;   // the buffer the sort left free
  k_codec_gather_u32<<<blocks, 256, 0, s>>>(t.key_hi, i_sorted, n, hi_perm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  uint32_t* i_free = (i_sorted == t.idx) ? t.val2 : t.idx;
  uint32_t* v_alt = (hi_perm == t.key_lo) ? t.key2 : t.key_lo;
  uint32_t *k2 = nullptr, *perm = nullptr;
  e = launch_radix_sort(hi_perm, i_sorted, v_alt, i_free, t.count, nullptr, n, 10, t.hist, t.scan_part, s, &k2, &perm);
  if (e != hipSuccess) return e;
  k_codec_gather_codes<<<blocks, 256, 0, s>>>(t.codes, perm, n, stride_out, codes_out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (perm_out) e = hipMemcpyAsync(perm_out, perm, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
  return e;
}

}  // namespace gp

namespace gp {

// Allocates the codec's scratch, encodes, synchronises and frees.
gp_status encode_volume(const float* means, const float* attrs, int64_t n, int64_t stride, uint16_t* codes_out,
                        int64_t stride_out, uint32_t* perm_out, float* d_hdr, hipStream_t s) {
  CodecScratch t{};
  const int64_t nn = std::max<int64_t>(n, 1);
  const int64_t hist = radix_hist_entries(32, nn);
  const int64_t part = scan_parts_needed(hist);
  std::vector<void*> owned;
  auto alloc = [&](auto** p, int64_t count) {
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, sizeof(**p) * (size_t)count);
    *p = static_cast<std::remove_reference_t<decltype(*p)>>(q);
    if (e == hipSuccess) owned.push_back(q);
    return e;
  };
  hipError_t e = alloc(&t.bounds, 9);
  if (e == hipSuccess) e = alloc(&t.count, 1);
  if (e == hipSuccess) e = alloc(&t.codes, 11 * nn);
  if (e == hipSuccess) e = alloc(&t.key_lo, nn);
  if (e == hipSuccess) e = alloc(&t.key_hi, nn);
  if (e == hipSuccess) e = alloc(&t.idx, nn);
  if (e == hipSuccess) e = alloc(&t.key2, nn);
  if (e == hipSuccess) e = alloc(&t.val2, nn);
  if (e == hipSuccess) e = alloc(&t.hist, hist);
  if (e == hipSuccess) e = alloc(&t.scan_part, 2 * part);
  gp_status st = GP_OK;
  if (e != hipSuccess) {
    set_error("encode: out of device memory");
    st = GP_ENOMEM;
  } else {
    e = launch_encode(means, attrs, n, stride, codes_out, stride_out, perm_out, d_hdr, t, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "encode");
  }
  for (void* q : owned) (void)hipFree(q);
  return st;
}

}  // namespace gp
