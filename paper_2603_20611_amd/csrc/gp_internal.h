// Internal declarations shared by the HIP translation units of libgaussianpile.
// Device-side layouts, the workspace object and the kernel launch wrappers.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gaussianpile.h"

// The amdgcn legacy multiply intrinsic, declared by its LLVM name.
extern "C" __device__ float gp_fmul_legacy(float, float) __asm("llvm.amdgcn.fmul.legacy");

namespace gp {

// Product with 0 * anything = 0 (also 0 * inf): v_mul_legacy_f32 through the
// compiler's own intrinsic, so that it schedules the product like any other
// and inserts the wait state gfx950 requires between a transcendental
// (v_exp_f32) and a VALU instruction reading its result only where one is
// needed.  (Written as inline asm, the product is opaque to the hazard
// recognizer: a variant that multiplied an exp2 result at once read stale
// values, so an asm form must carry a wait state of its own.)
__device__ __forceinline__ float mul0(float x, float y) { return gp_fmul_legacy(x, y); }

// Attribute row r (0..7: l_x, l_y, l_z, q_w, q_x, q_y, q_z, alpha) of Gaussian
// j, converted to float32.
template <int DT>
__device__ __forceinline__ float load_attr(const void* base, int r, int64_t stride, int64_t j) {
  const int64_t i = r * stride + j;
  if constexpr (DT == GP_F32) {
    return static_cast<const float*>(base)[i];
  } else if constexpr (DT == GP_BF16) {
    return __bfloat162float(static_cast<const __hip_bfloat16*>(base)[i]);
  } else if constexpr (DT == GP_F16) {
    return __half2float(static_cast<const __half*>(base)[i]);
  } else {   // GP_Q16
    if (r >= 3 && r <= 6) return (float)static_cast<const int16_t*>(base)[i] / 32767.0f;
    return __half2float(static_cast<const __half*>(base)[i]);
  }
}

constexpr int kTile = 16;            // tile edge in pixels (16 x 16 tiles)
constexpr int kTilePix = kTile * kTile;

// Per-slice constants on the device (one entry per slice of a batch).
struct SliceDev {
  float z, sigma_z, x0, y0, dx, dy;
  int32_t width, height, ntx, nty;
  int32_t tile_base;   // index of the slice's first bin
  int32_t group;       // which Gaussian set the slice samples
  int64_t out_off;     // offset of the slice's image in a packed batch
  float* out;          // where the forward writes the slice's image
  int64_t pad;
};
// Camera poses of a posed batch live in their own array ([n_slices][12]: R_c
// row-major, then t), so the slice descriptors stay small (they are read for
// every (Gaussian, slice) pair and should stay in the L1 cache).

// Sizes of one batch, read by the kernels from device memory so that a launch
// sequence can be captured once and replayed for batches of any size up to the
// workspace capacity.
struct BatchHdr {
  int32_t n_groups, n_slices, n_bins, total_gauss;
  int32_t n_waves;     // total_gauss / 64
  int32_t tiles_per_slice;   // the common tile count of every slice, or 0 if they differ
  int32_t pad[2];
};

// Rasteriser work counters, handed out by atomics (reset at the start of every
// forward): one shared queue, and eight per-XCD queues on cache lines of their
// own (kWorkXcd + 32 q) for the deep-stack raster.  (One queue per XCD, each
// draining a contiguous eighth of the tiles, was measured 35 % slower than one
// queue shared by all: with every XCD on the same slices at once, records one
// XCD brings in are still cached for the others.  The per-XCD queues of the
// deep-stack raster interleave 4 x 4-tile units instead, so that every XCD
// works on every slice group.)
enum { kWorkRasterFwd = 0, kWorkRasterBwd = 1, kWorkXcd = 32, kWorkCount = kWorkXcd + 8 * 32 };

__device__ __forceinline__ uint32_t wave_take(uint32_t* counter) {
  uint32_t v = 0;
  if (__lane_id() == 0) v = atomicAdd(counter, 1u);
  return __builtin_amdgcn_readfirstlane(v);
}


// One Gaussian set and the contiguous range of slices that sample it.
struct GroupDev {
  const float* means;  // [3][stride] float32
  const void* attrs;   // [8][stride] attr_dtype
  int64_t stride;
  int32_t n;
  int32_t attr_dtype;
  int32_t k0, k1;      // slices [k0, k1) of the batch
  int32_t gbase;       // first flattened Gaussian index (multiple of 64)
  int32_t flags;       // kGroupSortedZ, kGroupSharedPose
  float zlo, zhi;      // depth range of the group's slices
  float sz2max;        // largest sigma_z^2 of the group's slices (+inf if any is infinite)
  float pad;
};

// Group of flattened Gaussian index wave0 (a multiple of 64; groups start at
// multiples of 64 in ascending order): the last group whose base is at most
// wave0, by binary search (uniform over a wavefront, so scalar loads).
__device__ __forceinline__ int group_of(const GroupDev* groups, int n_groups, int wave0) {
  int lo = 0, hi = n_groups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (groups[mid].gbase <= wave0) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Rendering constants of one call (sizes that vary per batch live in BatchHdr).
struct RenderConst {
  float q_cut, bbox, scale_mod;
  uint32_t flags;
  uint32_t rec_cap, inst_cap;
  int32_t attr_dtype;
  int32_t pad;
};

// Grid sizes of a launch sequence: exact for one known batch, or the
// workspace capacity when the sequence is captured for replay.
struct LaunchDims {
  int64_t gauss;        // flattened Gaussians to cover (multiple of 64)
  int64_t bins;         // bins to cover (also fixes the sort's key width)
  int32_t emit_width = 1;   // lanes per Gaussian in the emit (1, 2, 4, 8 or 16)
  int32_t posed = 0;        // the slices carry camera poses
  int32_t host_batch = 0;   // the host staging holds this batch (not a capture for later batches)
  // the most bins of one group (0: `bins`).  The emit writes a batch's list
  // entries group after group and a group's bins are one contiguous run of
  // keys, so a stable sort by the low bits that tell one group's bins apart
  // leaves every bin's entries contiguous and in Gaussian order.
  int64_t sort_bins = 0;
};
// Emit width for groups of at most `slices` slices each.
inline int32_t emit_width_for(int64_t slices) {
  int32_t w = 1;
  while (w < 16 && w < slices) w <<= 1;
  return w;
}

// Counters written by the preprocess.
// (records and instances are adjacent: the wavefront scan writes both as one uint2)
// kCtrSortEnd: the first instance slot of an overflowed Gaussian (every later
// slot is one too: slots are a scan in Gaussian order), all ones if none; the
// sort and the bin ranges stop there.
enum { kCtrRecords = 0, kCtrInstances = 1, kCtrOverflow = 2, kCtrSortEnd = 3, kCtrCount = 4 };

// Record payload in pixel space, 32 bytes, gathered by the rasterisers:
//   the mean in pixel-index units as ax + xr, ay + yr, with the anchors ax, ay
//   the nearest integers (exact in binary32) and xr, yr the remainders
//   (|xr|, |yr| <= 1/2), so that the rasterisers form offsets from a tile
//   origin as (origin - anchor) - remainder without the rounding a binary32
//   mean of a large coordinate would carry; a, b, c = exponent coefficients of
//   exp2(a dx^2 + b dx dy + c dy^2); w = alpha~.
struct alignas(16) RecPay {
  float xr, yr, a, b;
  float c, w, ax, ay;
};
// Records with a >= kSmoothA and |b| <= kSmoothB take the forward raster's row
// recurrence.
constexpr float kSmoothA = -4.0f;
constexpr float kSmoothB = 16.0f;

// Record bookkeeping, 16 bytes.  Records are the visible (Gaussian, slice)
// pairs; the instance slots [ibase, ibase + ntiles) enumerate the footprint
// row-major.
struct alignas(16) RecMeta {
  uint32_t ibase;   // first instance slot
  uint32_t rx;      // tx0 | tx1 << 16
  uint32_t ry;      // ty0 | ty1 << 16
  uint32_t slice;   // slice index within the batch
};

constexpr uint32_t kInvalidSlice = 0xFFFFFFFFu;   // RecMeta.slice of an unused record slot

__host__ __device__ inline uint32_t rec_ntiles(const RecMeta& m) {
  return ((m.rx >> 16) - (m.rx & 0xFFFFu) + 1u) * ((m.ry >> 16) - (m.ry & 0xFFFFu) + 1u);
}

// GroupDev.flags: the group's slices have non-decreasing z and one sigma_z, so
// each Gaussian's kept slices form a range found by binary search.
constexpr int32_t kGroupSortedZ = 1;
// GroupDev.flags: every slice of a posed group has the same camera pose (bit
// for bit), so the group is an axial stack in that camera frame: the
// Gaussian's camera-frame view is computed once and, with kGroupSortedZ, its
// kept slices are found by binary search on the camera-frame depths.
constexpr int32_t kGroupSharedPose = 2;

// The workspace: library-owned device buffers, sized by capacity.
struct Workspace {
  int device = 0;
  bool auto_size = true;
  bool overflow_per_forward = false;  // clear the overflow flag at every forward
  bool overflowed = false;
  void* last_stream = nullptr;

  // capacities (elements)
  int64_t rec_cap = 0, inst_cap = 0, bin_cap = 0, slice_cap = 0, group_cap = 0, gauss_cap = 0;

  // batch descriptors: header, slices, groups and poses in one block (device
  // and pinned host copies of the same layout), so that a batch is uploaded by
  // one copy; the pointers below point into it
  void* d_desc = nullptr;
  void* h_desc = nullptr;
  size_t desc_off_groups = 0, desc_off_poses = 0;

  // device buffers
  SliceDev* d_slices = nullptr;
  float* d_poses = nullptr;         // [slice_cap][12]
  GroupDev* d_groups = nullptr;
  BatchHdr* d_hdr = nullptr;
  uint32_t* d_work = nullptr;       // kWorkCount work counters
  uint32_t* d_ctr = nullptr;        // kCtrCount counters
  uint32_t* d_bin_lo = nullptr;     // [bin_cap] list range [lo, hi) of each bin
  uint32_t* d_bin_hi = nullptr;     // [bin_cap]
  RecPay* d_rec_pay = nullptr;      // [rec_cap]
  RecMeta* d_rec_meta = nullptr;    // [rec_cap]
  uint32_t* d_g_rbase = nullptr;    // [gauss_cap]
  uint32_t* d_g_nrec = nullptr;     // [gauss_cap]
  uint32_t* d_g_ninst = nullptr;    // [gauss_cap]
  uint32_t* d_g_krange = nullptr;   // [gauss_cap] kept slices kb | ke << 16
  uint2* d_wave_cnt = nullptr;      // [wave_cap] per-wavefront counts, then bases
  uint32_t* d_inst_key = nullptr;   // [inst_cap] bin of each instance slot
  uint32_t* d_inst_val = nullptr;   // [inst_cap] record of each instance slot
  uint32_t* d_key2 = nullptr;       // [inst_cap] sort ping-pong
  uint32_t* d_val2 = nullptr;       // [inst_cap]
  uint32_t* d_list = nullptr;       // record ids in list order (one of the above)
  uint32_t* d_list_key = nullptr;   // their bins
  uint32_t* d_hist = nullptr;       // [hist_cap] radix digit counts
  uint2* d_scan_part = nullptr;     // [part_cap] scan partials
  float4* d_moments = nullptr;      // [2 * inst_cap] backward moments per instance slot
  double* d_ssim = nullptr;         // [ssim_cap] coefficient maps of the D-SSIM gradient
  int64_t ssim_cap = 0;
  // voxeliser: records and tile boxes per Gaussian, moments per instance
  float4* d_vox_rec = nullptr;      // [3 * vox_gcap]
  uint32_t* d_vox_box = nullptr;    // [3 * vox_gcap]
  float4* d_vox_mom = nullptr;      // [3 * vox_icap]
  int64_t vox_gcap = 0, vox_icap = 0;
  bool vox_have = false;            // holds the lists of a voxelisation
  const void* vox_means = nullptr;
  const void* vox_attrs = nullptr;
  int64_t vox_n = 0, vox_stride = 0, vox_ntiles = 0, vox_ninst = 0;
  uint64_t vox_hash = 0;
  int64_t hist_cap = 0, part_cap = 0, wave_cap = 0;

  // pinned staging for uploads / readbacks
  SliceDev* h_slices = nullptr;
  float* h_poses = nullptr;
  GroupDev* h_groups = nullptr;
  BatchHdr* h_hdr = nullptr;
  uint32_t* h_ctr = nullptr;
  hipEvent_t upload_done = nullptr;

  // state of the last forward (checked by the backward)
  bool have_forward = false;
  bool fwd_forward_only = false;    // rendered with GP_FLAG_FORWARD_ONLY: no backward
  const void* fwd_means = nullptr;
  const void* fwd_attrs = nullptr;
  int64_t fwd_n = 0, fwd_stride = 0;
  int32_t fwd_nslices = 0, fwd_nbins = 0;
  int32_t fwd_posed = 0;
  int64_t fwd_gauss = 0;
  uint64_t fwd_slice_hash = 0;
  RenderConst fwd_rc{};
  int64_t last_records = 0, last_instances = 0;

  // optional densification statistics, accumulated by the backward
  float* st_grad_norm = nullptr;
  int32_t* st_count = nullptr;
  float* st_max_radius = nullptr;
  int64_t st_n = 0;

  // optional per-stage timing (events recorded around the stages whose bit is set)
  uint32_t timing = 0;
  struct TimedLaunch { int stage; hipEvent_t start, stop; };
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> event_pool;
  double stage_ms[GP_N_STAGES] = {};
  int64_t stage_n[GP_N_STAGES] = {};
};

// ---- error plumbing (gp_api.hip) ----
void set_error(const std::string& msg);
gp_status hip_fail(hipError_t e, const char* what);
#define GP_HIP(call)                                   \
  do {                                                 \
    hipError_t _e = (call);                            \
    if (_e != hipSuccess) return gp::hip_fail(_e, #call); \
  } while (0)

// ---- batches (gp_api.hip) ----
struct GroupIn {
  const gp_gaussians* g;
  int32_t k0, k1;   // its slices [k0, k1) of the batch
};
struct BatchPlan {
  int32_t ns, ng;
  int64_t nbins, total_gauss, npix;
  int64_t max_group_bins;   // the most bins of one group
  int32_t attr_dtype;
  int32_t posed;
};
hipError_t wait_ws(Workspace* ws);
gp_status reserve_small(Workspace* ws, int64_t n_slices, int64_t n_groups, int64_t n_bins, int64_t n_gauss);
gp_status reserve_lists(Workspace* ws, int64_t rec_cap, int64_t inst_cap);
gp_status reserve_sort(Workspace* ws, int bits);
gp_status stage_batch(Workspace* ws, const GroupIn* groups, int ng, const gp_slice* hs, int ns, float* out_base,
                      float* const* outs, BatchPlan* plan, const float* poses = nullptr);
gp_status upload_batch(Workspace* ws, const BatchPlan& p, hipStream_t s);
RenderConst make_render_const(const gp_render_opts* o, int attr_dtype, const Workspace* ws);
gp_status enqueue_forward(Workspace* ws, RenderConst rc, const LaunchDims& d, hipStream_t s, int64_t rec_limit = 0,
                          int64_t inst_limit = 0);
gp_status check_gaussians_pub(const gp_gaussians* g);
gp_status check_slice_pub(const gp_slice& sl, int k);
gp_status check_opts_pub(const gp_render_opts* o);
gp_status workspace_new(Workspace** out, int64_t max_records, int64_t max_instances);
void workspace_free(Workspace* ws);

// ---- launch wrappers (one per kernel file) ----
// k_preprocess.hip
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s);
hipError_t launch_reset(const Workspace& ws, bool clear_overflow, const LaunchDims& d, hipStream_t s);
// Count of the forward, which also resets its counters, work queues and bin
// ranges (one launch fewer per forward).
// scanned: the wavefront counts will be scanned by the scan kernel (else the
// compacting count also writes 512-Gaussian chunk totals for the emit).
hipError_t launch_pre_count(const RenderConst& rc, const Workspace& ws, const LaunchDims& d, bool clear_overflow,
                            bool scanned, hipStream_t s);
// scanned: the wavefront counts were scanned (else the emit forms the bases
// and writes the totals itself).
hipError_t launch_pre_emit(const RenderConst& rc, const Workspace& ws, const LaunchDims& d, uint32_t sentinel_bin,
                           bool scanned, hipStream_t s);
// k_sort.hip
hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, const int32_t* d_n, int64_t max_n, uint32_t* part,
                           uint32_t* total, hipStream_t s);
hipError_t launch_scan_u32x2(const uint2* in, uint2* out, const int32_t* d_n, int64_t max_n, uint2* part,
                             uint2* total, hipStream_t s);
int64_t scan_parts_needed(int64_t max_n);
int radix_passes(int bits);
int64_t radix_hist_entries(int bits, int64_t cap);
hipError_t launch_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* d_count,
                             const uint32_t* d_count2,
                             int64_t cap, int bits, uint32_t* hist, uint32_t* scan_part, hipStream_t s,
                             uint32_t** k_out, uint32_t** v_out);
hipError_t launch_bin_ranges(const BatchHdr* hdr, const uint32_t* key, const uint32_t* d_count,
                             const uint32_t* d_count2, int64_t cap,
                             uint32_t* lo, uint32_t* hi, hipStream_t s);
inline int key_bits(int64_t n_bins) {
  int b = 0;
  while (b < 31 && ((int64_t)1 << b) <= n_bins) ++b;
  return b;   // 2^b > n_bins, so n_bins itself (the overflow sentinel) fits
}
// k_raster.hip
hipError_t launch_raster_fwd(const RenderConst& rc, const Workspace& ws, const LaunchDims& d, hipStream_t s);
hipError_t launch_raster_bwd(const RenderConst& rc, const Workspace& ws, const float* grad_out,
                             const LaunchDims& d, hipStream_t s);
// k_backward.hip
hipError_t launch_preprocess_bwd(const RenderConst& rc, const Workspace& ws, float* grad,
                                 int64_t grad_stride, const LaunchDims& d, hipStream_t s);
// k_codec.hip
struct CodecScratch {
  uint32_t* bounds;     // [8]
  uint32_t* count;      // [1]
  uint16_t* codes;      // [11][n] in the original order
  uint32_t *key_lo, *key_hi, *idx, *key2, *val2;   // [n] each
  uint32_t* hist;       // radix_hist_entries(32, n)
  uint32_t* scan_part;  // scan_parts_needed of the histogram
};
hipError_t launch_encode(const float* means, const float* attrs, int64_t n, int64_t stride, uint16_t* codes_out,
                         int64_t stride_out, uint32_t* perm_out, float* d_hdr, const CodecScratch& t, hipStream_t s);
gp_status encode_volume(const float* means, const float* attrs, int64_t n, int64_t stride, uint16_t* codes_out,
                        int64_t stride_out, uint32_t* perm_out, float* d_hdr, hipStream_t s);
// k_voxel.hip
struct VoxLaunch {
  int n;
  int ntx, nty, ntz;
  int64_t n_tiles;
};
VoxLaunch vox_prepare(const gp_gaussians* g, const gp_volume_grid* grid, const gp_render_opts* o);
hipError_t launch_vox_count(const Workspace& ws, const gp_gaussians* g, const gp_volume_grid* grid,
                            const gp_render_opts* o, const VoxLaunch& L, hipStream_t s);
hipError_t launch_vox_emit(const Workspace& ws, const gp_gaussians* g, const gp_volume_grid* grid,
                           const gp_render_opts* o, const VoxLaunch& L, hipStream_t s);
hipError_t launch_vox_ranges(const Workspace& ws, const VoxLaunch& L, uint32_t n_inst, hipStream_t s);
hipError_t launch_vox_fwd(const Workspace& ws, const gp_gaussians* g, const gp_volume_grid* grid,
                          const gp_render_opts* o, const VoxLaunch& L, float* vol, hipStream_t s);
hipError_t launch_vox_bwd(const Workspace& ws, const gp_gaussians* g, const gp_volume_grid* grid,
                          const gp_render_opts* o, const VoxLaunch& L, const float* gvol, float* grad,
                          int64_t grad_stride, hipStream_t s);
// k_densify.hip
hipError_t launch_densify(const float* p, const float* m, const float* v, int64_t n, int64_t stride,
                          const float* grad_norm, const int32_t* count, const float* max_radius, const float* noise,
                          const gp_densify_cfg& cfg, uint32_t* action, uint32_t* outs, uint32_t* scan_part,
                          uint32_t* total, float* p_out, float* m_out, float* v_out, int64_t stride_out,
                          bool emit, hipStream_t s);
// k_optim.hip
hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t n, int64_t stride,
                       const gp_adam_cfg& c, hipStream_t s);
// Scratch (float64 elements) of launch_ssim_loss: coefficient maps and per-block sums.
// ssim_noalloc_scratch: the device address, on the current device, of the
// library's static scratch of ssim_noalloc_capacity() elements (looked up once per device).
int64_t ssim_noalloc_capacity();
hipError_t ssim_noalloc_scratch(double** out);
int64_t ssim_scratch(int n_slices, int width, int height);
hipError_t launch_ssim_loss(const float* x, const float* y, int n_slices, int width, int height, double lam,
                            double* maps, float* grad, float* loss, hipStream_t s);
hipError_t launch_l1(const float* img, const float* tgt, int64_t n, float scale, float* grad,
                     float* loss, hipStream_t s);

}  // namespace gp
