// Internal declarations shared by the HIP translation units of libgaussianpile.
// Device-side layouts, the workspace object and the kernel launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gaussianpile.h"

namespace gp {

constexpr int kTile = 16;            // tile edge in pixels (16 x 16 tiles)
constexpr int kTilePix = kTile * kTile;
constexpr int kBinSortCap = 4096;    // tile lists up to this length are sorted in LDS

// Per-slice constants on the device (one entry per slice of a batch).
struct SliceDev {
  float z, sigma_z, x0, y0, dx, dy;
  int32_t width, height, ntx, nty;
  int32_t tile_base;   // index of the slice's first bin
  int32_t group;       // which Gaussian set the slice samples
  int64_t out_off;     // offset of the slice's image in the packed output
};

// One Gaussian set and the contiguous range of slices that sample it.
struct GroupDev {
  const float* means;  // [3][stride] float32
  const void* attrs;   // [8][stride] attr_dtype
  int64_t stride;
  int32_t n;
  int32_t attr_dtype;
  int32_t k0, k1;      // slices [k0, k1) of the batch
  int32_t gbase;       // first flattened Gaussian index (multiple of 64)
  int32_t pad;
};

// Rendering constants of one call.
struct RenderConst {
  float q_cut, bbox, scale_mod;
  uint32_t flags;
  int32_t n_groups, n_slices, n_bins;
  int32_t total_gauss;   // flattened Gaussian count (groups padded to 64)
  uint32_t rec_cap, inst_cap;
};

// Counters written by the preprocess.
enum { kCtrRecords = 0, kCtrInstances = 1, kCtrOverflow = 2, kCtrCount = 4 };

// Record payload in pixel space (what the rasteriser streams), 32 bytes:
//   x = mean x in pixel-index units, y = mean y, a/b/c = exponent coefficients
//   of exp2(a dx^2 + b dx dy + c dy^2), w = alpha~, gid = Gaussian index,
//   slice = slice index within the batch.
struct alignas(16) RecPay {
  float x, y, a, b;
  float c, w;
  uint32_t gid, slice;
};

// Record bookkeeping, 16 bytes.
struct alignas(16) RecMeta {
  uint32_t ibase;   // first instance slot
  uint32_t rx;      // tx0 | tx1 << 16
  uint32_t ry;      // ty0 | ty1 << 16
  uint32_t ntiles;
};

// The workspace: library-owned device buffers, sized by capacity.
struct Workspace {
  int device = 0;
  bool auto_size = true;
  bool overflowed = false;
  void* last_stream = nullptr;

  // capacities (elements)
  int64_t rec_cap = 0, inst_cap = 0, bin_cap = 0, slice_cap = 0, group_cap = 0, gauss_cap = 0;

  // device buffers
  SliceDev* d_slices = nullptr;
  GroupDev* d_groups = nullptr;
  uint32_t* d_ctr = nullptr;        // kCtrCount counters
  uint32_t* d_bin_count = nullptr;  // [bin_cap]
  uint32_t* d_bin_start = nullptr;  // [bin_cap + 1]
  RecPay* d_rec_pay = nullptr;      // [rec_cap]
  RecMeta* d_rec_meta = nullptr;    // [rec_cap]
  uint32_t* d_g_rbase = nullptr;    // [gauss_cap]
  uint32_t* d_g_nrec = nullptr;     // [gauss_cap]
  uint32_t* d_inst_rank = nullptr;  // [inst_cap]
  uint32_t* d_inst_rid = nullptr;   // [inst_cap]
  uint64_t* d_sort_key = nullptr;   // [inst_cap]
  RecPay* d_pay = nullptr;          // [inst_cap] payload in list order
  uint32_t* d_inst_pos = nullptr;   // [inst_cap] instance slot -> list position
  float4* d_moments = nullptr;      // [2 * inst_cap] backward moments per list entry

  // pinned staging for uploads / readbacks
  SliceDev* h_slices = nullptr;
  GroupDev* h_groups = nullptr;
  uint32_t* h_ctr = nullptr;
  hipEvent_t upload_done = nullptr;

  // state of the last forward (checked by the backward)
  bool have_forward = false;
  const void* fwd_means = nullptr;
  const void* fwd_attrs = nullptr;
  int64_t fwd_n = 0, fwd_stride = 0;
  int32_t fwd_nslices = 0, fwd_nbins = 0;
  uint64_t fwd_slice_hash = 0;
  RenderConst fwd_rc{};
  int64_t last_records = 0, last_instances = 0;

  // optional per-stage timing (events recorded around each stage)
  bool timing = false;
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

// ---- launch wrappers (one per kernel file) ----
// k_preprocess.hip
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s);
hipError_t launch_preprocess(const RenderConst& rc, const Workspace& ws, hipStream_t s);
// k_bins.hip
hipError_t launch_scan_bins(const Workspace& ws, int32_t n_bins, hipStream_t s);
hipError_t launch_scatter(const RenderConst& rc, const Workspace& ws, hipStream_t s);
hipError_t launch_bin_sort(const RenderConst& rc, const Workspace& ws, hipStream_t s);
// k_raster.hip
hipError_t launch_raster_fwd(const RenderConst& rc, const Workspace& ws, float* out, hipStream_t s);
hipError_t launch_raster_bwd(const RenderConst& rc, const Workspace& ws, const float* grad_out,
                             hipStream_t s);
// k_backward.hip
hipError_t launch_preprocess_bwd(const RenderConst& rc, const Workspace& ws, float* grad,
                                 int64_t grad_stride, hipStream_t s);
// k_optim.hip
hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t n, int64_t stride,
                       const gp_adam_cfg& c, hipStream_t s);
hipError_t launch_l1(const float* img, const float* tgt, int64_t n, float scale, float* grad,
                     float* loss, hipStream_t s);

}  // namespace gp
