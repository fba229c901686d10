// Host side of the C-ABI: argument validation, the workspace, and the launch
// sequence of a render (preprocess -> bin scan -> scatter -> per-bin sort ->
// rasterise), its backward, Adam and the L1 loss.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gp_internal.h"

namespace gp {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

gp_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return GP_EHIP;
}

static gp_status einval(const std::string& msg) {
  set_error(msg);
  return GP_EINVAL;
}

template <typename T>
static hipError_t dev_alloc(T** p, int64_t count) {
  if (*p) {
    hipError_t e = hipFree(*p);
    *p = nullptr;
    if (e != hipSuccess) return e;
  }
  if (count <= 0) return hipSuccess;
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)count);
}

template <typename T>
static hipError_t host_alloc(T** p, int64_t count) {
  if (*p) {
    hipError_t e = hipHostFree(*p);
    *p = nullptr;
    if (e != hipSuccess) return e;
  }
  return hipHostMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)(count > 0 ? count : 1),
                       hipHostMallocDefault);
}

hipError_t wait_ws(Workspace* ws) {
  if (ws->upload_done) {
    hipError_t e = hipEventSynchronize(ws->upload_done);
    if (e != hipSuccess) return e;
  }
  return hipStreamSynchronize(static_cast<hipStream_t>(ws->last_stream));
}

// The descriptor block for slice_cap slices and group_cap groups: header at 0,
// then slices, groups, poses (256-byte aligned parts).
static hipError_t layout_desc(Workspace* ws, int64_t slice_cap, int64_t group_cap) {
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t off_s = up(sizeof(BatchHdr));
  const size_t off_g = off_s + up(sizeof(SliceDev) * (size_t)slice_cap);
  const size_t off_p = off_g + up(sizeof(GroupDev) * (size_t)group_cap);
  const size_t bytes = off_p + up(sizeof(float) * 12 * (size_t)slice_cap);
  if (ws->d_desc) {
    hipError_t e = hipFree(ws->d_desc);
    ws->d_desc = nullptr;
    if (e != hipSuccess) return e;
  }
  if (ws->h_desc) {
    hipError_t e = hipHostFree(ws->h_desc);
    ws->h_desc = nullptr;
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipMalloc(&ws->d_desc, bytes);
  if (e == hipSuccess) e = hipHostMalloc(&ws->h_desc, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return e;
  std::memset(ws->h_desc, 0, bytes);
  char* d = static_cast<char*>(ws->d_desc);
  char* h = static_cast<char*>(ws->h_desc);
  ws->d_hdr = reinterpret_cast<BatchHdr*>(d);
  ws->h_hdr = reinterpret_cast<BatchHdr*>(h);
  ws->d_slices = reinterpret_cast<SliceDev*>(d + off_s);
  ws->h_slices = reinterpret_cast<SliceDev*>(h + off_s);
  ws->d_groups = reinterpret_cast<GroupDev*>(d + off_g);
  ws->h_groups = reinterpret_cast<GroupDev*>(h + off_g);
  ws->d_poses = reinterpret_cast<float*>(d + off_p);
  ws->h_poses = reinterpret_cast<float*>(h + off_p);
  ws->desc_off_groups = off_g;
  ws->desc_off_poses = off_p;
  ws->slice_cap = slice_cap;
  ws->group_cap = group_cap;
  return hipSuccess;
}

gp_status reserve_small(Workspace* ws, int64_t n_slices, int64_t n_groups, int64_t n_bins,
                               int64_t n_gauss) {
  if (n_slices > ws->slice_cap || n_groups > ws->group_cap) {
    GP_HIP(wait_ws(ws));
    GP_HIP(layout_desc(ws, std::max<int64_t>(ws->slice_cap, n_slices > ws->slice_cap ? n_slices + 64 : 0),
                       std::max<int64_t>(ws->group_cap, n_groups > ws->group_cap ? n_groups + 8 : 0)));
  }
  if (n_bins > ws->bin_cap) {
    GP_HIP(wait_ws(ws));
    const int64_t cap = n_bins + n_bins / 4 + 256;
    GP_HIP(dev_alloc(&ws->d_bin_lo, cap));
    GP_HIP(dev_alloc(&ws->d_bin_hi, cap));
    ws->bin_cap = cap;
  }
  if (n_gauss > ws->gauss_cap) {
    GP_HIP(wait_ws(ws));
    const int64_t cap = (n_gauss + n_gauss / 8 + 256 + 63) / 64 * 64;
    GP_HIP(dev_alloc(&ws->d_g_rbase, cap));
    GP_HIP(dev_alloc(&ws->d_g_nrec, cap));
    GP_HIP(dev_alloc(&ws->d_g_ninst, cap));
    GP_HIP(dev_alloc(&ws->d_g_krange, cap));
    // the wavefront counts, then the counts of 512-Gaussian chunks
    GP_HIP(dev_alloc(&ws->d_wave_cnt, cap / 64 + 1 + cap / 512 + 1));
    ws->gauss_cap = cap;
    ws->wave_cap = cap / 64 + 1;
  }
  return GP_OK;
}

// Radix-sort scratch for keys of `bits` bits over the instance capacity, and
// scan partials for both the digit counts and the wavefront counts.
gp_status reserve_sort(Workspace* ws, int bits) {
  const int64_t hist = radix_hist_entries(bits, ws->inst_cap);
  const int64_t part = std::max(scan_parts_needed(hist), scan_parts_needed(ws->wave_cap));
  if (hist > ws->hist_cap) {
    GP_HIP(wait_ws(ws));
    GP_HIP(dev_alloc(&ws->d_hist, hist));
    ws->hist_cap = hist;
  }
  if (part > ws->part_cap) {
    GP_HIP(wait_ws(ws));
    GP_HIP(dev_alloc(&ws->d_scan_part, part));
    ws->part_cap = part;
  }
  return GP_OK;
}

gp_status reserve_lists(Workspace* ws, int64_t rec_cap, int64_t inst_cap) {
  if (rec_cap > 0xFFFFFFF0ll || inst_cap > 0xFFFFFFF0ll) return einval("capacity exceeds 2^32 entries");
  if (rec_cap > ws->rec_cap) {
    GP_HIP(wait_ws(ws));
    if (dev_alloc(&ws->d_rec_pay, rec_cap) != hipSuccess || dev_alloc(&ws->d_rec_meta, rec_cap) != hipSuccess) {
      ws->rec_cap = 0;
      set_error("record buffers: out of device memory");
      return GP_ENOMEM;
    }
    ws->rec_cap = rec_cap;
  }
  if (inst_cap > ws->inst_cap) {
    GP_HIP(wait_ws(ws));
    if (dev_alloc(&ws->d_inst_key, inst_cap) != hipSuccess || dev_alloc(&ws->d_inst_val, inst_cap) != hipSuccess ||
        dev_alloc(&ws->d_key2, inst_cap) != hipSuccess || dev_alloc(&ws->d_val2, inst_cap) != hipSuccess ||
        dev_alloc(&ws->d_moments, 2 * inst_cap) != hipSuccess) {
      ws->inst_cap = 0;
      set_error("tile-list buffers: out of device memory");
      return GP_ENOMEM;
    }
    ws->inst_cap = inst_cap;
  }
  return GP_OK;
}

static uint64_t hash_bytes(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

static hipEvent_t take_event(Workspace* ws) {
  if (!ws->event_pool.empty()) {
    hipEvent_t e = ws->event_pool.back();
    ws->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs f (which enqueues one stage on s); with the stage's timing bit set,
// brackets it by events.
template <typename F>
static hipError_t timed(Workspace* ws, int stage, hipStream_t s, F&& f) {
  if (!((ws->timing >> stage) & 1u)) return f();
  hipEvent_t a = take_event(ws), b = take_event(ws);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = f();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  if (e != hipSuccess) return e;
  ws->pending.push_back({stage, a, b});
  return hipSuccess;
}

static hipError_t resolve_timings(Workspace* ws) {
  for (auto& t : ws->pending) {
    hipError_t e = hipEventSynchronize(t.stop);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, t.start, t.stop);
    if (e != hipSuccess) return e;
    ws->stage_ms[t.stage] += ms;
    ws->stage_n[t.stage] += 1;
    ws->event_pool.push_back(t.start);
    ws->event_pool.push_back(t.stop);
  }
  ws->pending.clear();
  return hipSuccess;
}

static gp_status check_gaussians(const gp_gaussians* g) {
  if (!g) return einval("gaussians: NULL");
  if (g->n < 0 || g->n >= (1ll << 31)) return einval("gaussians: n out of range");
  if (g->stride < g->n) return einval("gaussians: stride < n");
  if (g->n > 0 && (!g->means || !g->attrs)) return einval("gaussians: NULL means/attrs");
  if ((g->mean_dtype == GP_QM) != (g->attr_dtype == GP_QM)) return einval("gaussians: GP_QM is for both or neither");
  if (g->mean_dtype != GP_F32 && g->mean_dtype != GP_QM) return einval("gaussians: means must be GP_F32 or GP_QM");
  if (g->attr_dtype != GP_F32 && g->attr_dtype != GP_BF16 && g->attr_dtype != GP_F16 && g->attr_dtype != GP_Q16 &&
      g->attr_dtype != GP_QM)
    return einval("gaussians: unknown attr_dtype");
  return GP_OK;
}

static gp_status check_slice(const gp_slice& s, int k) {
  char buf[128];
  if (!(s.width >= 1 && s.width <= 16384 && s.height >= 1 && s.height <= 16384)) {
    snprintf(buf, sizeof buf, "slice %d: width/height out of range", k);
    return einval(buf);
  }
  if (!(s.dx > 0.f) || !(s.dy > 0.f) || !std::isfinite(s.dx) || !std::isfinite(s.dy)) {
    snprintf(buf, sizeof buf, "slice %d: pixel pitch must be finite and > 0", k);
    return einval(buf);
  }
  if (!std::isfinite(s.z) || !std::isfinite(s.x0) || !std::isfinite(s.y0) || !(s.sigma_z >= 0.f)) {
    snprintf(buf, sizeof buf, "slice %d: z, x0, y0 must be finite and sigma_z >= 0", k);
    return einval(buf);
  }
  return GP_OK;
}

static gp_status check_opts(const gp_render_opts* o) {
  if (!o) return einval("opts: NULL");
  if (!(o->q_cut >= 0.f) || !(o->bbox_sigmas > 0.f) || !(o->scale_mod > 0.f))
    return einval("opts: q_cut >= 0, bbox_sigmas > 0 and scale_mod > 0 required");
  if (o->flags & ~(GP_FLAG_EXACT | GP_FLAG_CONV_EXACT | GP_FLAG_FORWARD_ONLY)) return einval("opts: unknown flag");
  return GP_OK;
}

// Host descriptors of a batch (groups of slices sampling one Gaussian set
// each) into the workspace's pinned staging.  outs[k] (if given) is where slice
// k's image goes; otherwise images are packed back to back from out_base.
gp_status stage_batch(Workspace* ws, const GroupIn* groups, int ng, const gp_slice* hs, int ns, float* out_base,
                      float* const* outs, BatchPlan* plan, const float* poses) {
  int64_t nbins = 0, total_gauss = 0;
  for (int k = 0; k < ns; ++k)
    nbins += (int64_t)((hs[k].width + kTile - 1) / kTile) * ((hs[k].height + kTile - 1) / kTile);
  for (int g = 0; g < ng; ++g) total_gauss += (groups[g].g->n + 63) / 64 * 64;
  if (nbins >= (1ll << 30) || total_gauss >= (1ll << 31)) return einval("batch too large");
  if (ns > 65535) return einval("at most 65535 slices per batch");
  gp_status st = reserve_small(ws, ns, ng, nbins, total_gauss);
  if (st != GP_OK) return st;
  // the previous batch's upload must have been consumed before staging is reused
  if (ws->upload_done) GP_HIP(hipEventSynchronize(ws->upload_done));
  int64_t tb = 0, off = 0;
  for (int k = 0; k < ns; ++k) {
    SliceDev& d = ws->h_slices[k];
    d.z = hs[k].z; d.sigma_z = hs[k].sigma_z; d.x0 = hs[k].x0; d.y0 = hs[k].y0;
    d.dx = hs[k].dx; d.dy = hs[k].dy; d.width = hs[k].width; d.height = hs[k].height;
    d.ntx = (hs[k].width + kTile - 1) / kTile; d.nty = (hs[k].height + kTile - 1) / kTile;
    d.tile_base = (int32_t)tb; d.group = 0; d.out_off = off;
    d.out = outs ? outs[k] : out_base + off;
    d.pad = 0;
    tb += (int64_t)d.ntx * d.nty;
    off += (int64_t)hs[k].width * hs[k].height;
  }
  int64_t gb = 0, max_group_bins = 0;
  for (int g = 0; g < ng; ++g) {
    GroupDev& G = ws->h_groups[g];
    G.means = static_cast<const float*>(groups[g].g->means);
    G.attrs = groups[g].g->attrs;
    G.stride = groups[g].g->stride;
    G.n = (int32_t)groups[g].g->n;
    G.attr_dtype = groups[g].g->attr_dtype;
    G.k0 = groups[g].k0; G.k1 = groups[g].k1;
    G.gbase = (int32_t)gb;
    // non-decreasing z and one sigma_z: kept slices form a range (binary search)
    bool sorted = true;
    for (int k = G.k0 + 1; k < G.k1 && sorted; ++k)
      sorted = hs[k].z >= hs[k - 1].z && hs[k].sigma_z == hs[G.k0].sigma_z;
    // one camera pose for the whole group (bitwise): an axial stack in that frame
    bool shared = poses != nullptr;
    for (int k = G.k0 + 1; k < G.k1 && shared; ++k)
      shared = std::memcmp(poses + 12 * (size_t)k, poses + 12 * (size_t)G.k0, 12 * sizeof(float)) == 0;
    G.flags = (sorted && (!poses || shared) ? kGroupSortedZ : 0) | (shared ? kGroupSharedPose : 0);
    G.zlo = INFINITY; G.zhi = -INFINITY; G.sz2max = 0.f; G.pad = 0.f;
    for (int k = G.k0; k < G.k1; ++k) {
      G.zlo = std::min(G.zlo, hs[k].z);
      G.zhi = std::max(G.zhi, hs[k].z);
      G.sz2max = std::max(G.sz2max, hs[k].sigma_z * hs[k].sigma_z);
    }
    if (poses && !shared) {   // depths are in each slice's own frame: no world-depth shortcut
      G.zlo = -INFINITY;
      G.zhi = INFINITY;
    }
    for (int k = G.k0; k < G.k1; ++k) ws->h_slices[k].group = g;
    if (G.k1 > G.k0) {
      const int64_t first = ws->h_slices[G.k0].tile_base;
      const SliceDev& last = ws->h_slices[G.k1 - 1];
      max_group_bins = std::max<int64_t>(max_group_bins, (int64_t)last.tile_base + (int64_t)last.ntx * last.nty - first);
    }
    gb += (groups[g].g->n + 63) / 64 * 64;
  }
  ws->h_hdr->n_groups = ng;
  ws->h_hdr->n_slices = ns;
  ws->h_hdr->n_bins = (int32_t)nbins;
  ws->h_hdr->total_gauss = (int32_t)total_gauss;
  ws->h_hdr->n_waves = (int32_t)(total_gauss / 64);
  int32_t tps = ns > 0 ? ws->h_slices[0].ntx * ws->h_slices[0].nty : 0;
  for (int k = 1; k < ns && tps > 0; ++k)
    if (ws->h_slices[k].ntx * ws->h_slices[k].nty != tps) tps = 0;
  ws->h_hdr->tiles_per_slice = tps;
  plan->ns = ns; plan->ng = ng; plan->nbins = nbins; plan->total_gauss = total_gauss; plan->npix = off;
  plan->max_group_bins = max_group_bins;
  plan->attr_dtype = ng > 0 ? groups[0].g->attr_dtype : GP_F32;
  plan->posed = poses ? 1 : 0;
  if (poses) std::memcpy(ws->h_poses, poses, sizeof(float) * 12 * (size_t)ns);
  return GP_OK;
}

gp_status upload_batch(Workspace* ws, const BatchPlan& p, hipStream_t s) {
  // one copy: the header, the slices, the groups and (posed batches) the poses
  const size_t bytes = p.ns > 0 && p.posed ? ws->desc_off_poses + sizeof(float) * 12 * (size_t)p.ns
                                           : ws->desc_off_groups + sizeof(GroupDev) * (size_t)p.ng;
  GP_HIP(hipMemcpyAsync(ws->d_desc, ws->h_desc, bytes, hipMemcpyHostToDevice, s));
  GP_HIP(hipEventRecord(ws->upload_done, s));
  ws->last_stream = s;
  return GP_OK;
}

RenderConst make_render_const(const gp_render_opts* o, int attr_dtype, const Workspace* ws) {
  RenderConst rc{};
  rc.q_cut = o->q_cut; rc.bbox = o->bbox_sigmas; rc.scale_mod = o->scale_mod; rc.flags = o->flags;
  rc.rec_cap = (uint32_t)ws->rec_cap; rc.inst_cap = (uint32_t)ws->inst_cap;
  rc.attr_dtype = attr_dtype;
  return rc;
}

// Launch sequence of a forward on the uploaded batch:
//   reset -> count -> wavefront scan -> (automatic sizing: read the counts,
//   grow) -> emit -> radix sort by bin -> bin ranges -> rasterise.
// With fixed capacities nothing synchronises, so the sequence can be captured.
// rec_limit / inst_limit (> 0) lower the capacities the launch may fill (and
// the sort's extent) below the workspace's: a batch that needs more reports
// an overflow.
gp_status enqueue_forward(Workspace* ws, RenderConst rc, const LaunchDims& d, hipStream_t s, int64_t rec_limit,
                          int64_t inst_limit) {
  if (ws->auto_size && (ws->rec_cap == 0 || ws->inst_cap == 0)) {
    // first use: a generous guess, corrected after the first count
    const int64_t guess_rec = std::max<int64_t>(1 << 16, d.gauss / 4);
    gp_status st = reserve_lists(ws, guess_rec, 4 * guess_rec);
    if (st != GP_OK) return st;
  }
  // sort by the bits that tell one group's bins apart (entries are written
  // group after group; a group's bins are one contiguous run of keys)
  const int bits = key_bits(d.sort_bins > 0 ? std::min(d.sort_bins, d.bins) : d.bins);
  gp_status st = reserve_sort(ws, bits);
  if (st != GP_OK) return st;
  const bool clear_ovf = ws->auto_size || ws->overflow_per_forward;
  constexpr int64_t kEmitBasesMaxWaves = 16384;
  const bool scanned = ws->auto_size || d.posed || d.emit_width >= 16 || d.gauss / 64 > kEmitBasesMaxWaves;
  GP_HIP(timed(ws, GP_STAGE_PREPROCESS, s, [&] {
    // (the count also resets the forward's counters).  The wavefront counts
    // are scanned here when the host reads the totals before the emit
    // (automatic sizing), for deep stacks, whose emit runs two rounds of
    // workgroups that would each add up the counts before them (measured:
    // scan kernel 7.8 us, emit +8 us), and for launches of more than
    // kEmitBasesMaxWaves wavefronts (a served batch's capacity); otherwise
    // the emit forms its bases and the totals (8-slice batch: 0.0277 +
    // 0.0183 -> 0.0205 + 0.0226 ms).
    hipError_t e = launch_pre_count(rc, *ws, d, clear_ovf, scanned, s);
    if (e == hipSuccess && scanned)
      e = launch_scan_u32x2(ws->d_wave_cnt, ws->d_wave_cnt, &ws->d_hdr->n_waves, d.gauss / 64, ws->d_scan_part,
                            reinterpret_cast<uint2*>(ws->d_ctr + kCtrRecords), s);
    return e;
  }));
  if (ws->auto_size) {
    GP_HIP(hipMemcpyAsync(ws->h_ctr, ws->d_ctr, sizeof(uint32_t) * kCtrCount, hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    const int64_t R = ws->h_ctr[kCtrRecords], K = ws->h_ctr[kCtrInstances];
    ws->last_records = R;
    ws->last_instances = K;
    if (R > ws->rec_cap || K > ws->inst_cap) {
      st = reserve_lists(ws, std::max<int64_t>(ws->rec_cap, R + R / 4 + 1024),
                         std::max<int64_t>(ws->inst_cap, K + K / 4 + 4096));
      if (st == GP_OK) st = reserve_sort(ws, bits);
      if (st != GP_OK) return st;
    }
  }
  const int64_t rcap = rec_limit > 0 ? std::min<int64_t>(rec_limit, ws->rec_cap) : ws->rec_cap;
  const int64_t icap = inst_limit > 0 ? std::min<int64_t>(inst_limit, ws->inst_cap) : ws->inst_cap;
  rc.rec_cap = (uint32_t)rcap;
  rc.inst_cap = (uint32_t)icap;
  const uint32_t sentinel = (uint32_t)((1ll << bits) - 1);
  const uint32_t* d_count = ws->d_ctr + kCtrInstances;
  GP_HIP(timed(ws, GP_STAGE_EMIT, s, [&] { return launch_pre_emit(rc, *ws, d, sentinel, scanned, s); }));
  GP_HIP(timed(ws, GP_STAGE_SORT, s, [&] {
    const int64_t n_sort = ws->auto_size ? std::min<int64_t>(ws->last_instances, icap) : icap;
    const uint32_t* d_end = ws->d_ctr + kCtrSortEnd;   // before the first overflowed Gaussian's slots
    hipError_t e = launch_radix_sort(ws->d_inst_key, ws->d_inst_val, ws->d_key2, ws->d_val2, d_count, d_end,
                                     std::max<int64_t>(n_sort, 1), bits, ws->d_hist,
                                     reinterpret_cast<uint32_t*>(ws->d_scan_part), s, &ws->d_list_key, &ws->d_list);
    if (e == hipSuccess)
      e = launch_bin_ranges(ws->d_hdr, ws->d_list_key, d_count, d_end, icap, ws->d_bin_lo, ws->d_bin_hi, s);
    return e;
  }));
  GP_HIP(timed(ws, GP_STAGE_RASTER_FWD, s, [&] { return launch_raster_fwd(rc, *ws, d, s); }));
  ws->fwd_rc = rc;
  return GP_OK;
}

gp_status check_gaussians_pub(const gp_gaussians* g) { return check_gaussians(g); }
gp_status check_slice_pub(const gp_slice& sl, int k) { return check_slice(sl, k); }
gp_status check_opts_pub(const gp_render_opts* o) { return check_opts(o); }

gp_status workspace_new(Workspace** out, int64_t max_records, int64_t max_instances) {
  *out = nullptr;
  Workspace* ws = new (std::nothrow) Workspace();
  if (!ws) {
    set_error("workspace: host allocation");
    return GP_ENOMEM;
  }
  hipError_t e = hipGetDevice(&ws->device);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ws->upload_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ws->d_ctr), sizeof(uint32_t) * kCtrCount);
  if (e == hipSuccess) e = hipMemset(ws->d_ctr, 0, sizeof(uint32_t) * kCtrCount);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ws->d_work), sizeof(uint32_t) * kWorkCount);
  if (e == hipSuccess) e = layout_desc(ws, 0, 0);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&ws->h_ctr), sizeof(uint32_t) * kCtrCount, hipHostMallocDefault);
  if (e != hipSuccess) {
    workspace_free(ws);
    return hip_fail(e, "workspace_create");
  }
  ws->auto_size = max_records == 0;
  if (!ws->auto_size) {
    gp_status st = reserve_lists(ws, max_records, max_instances);
    if (st != GP_OK) {
      workspace_free(ws);
      return st;
    }
  }
  *out = ws;
  return GP_OK;
}

void workspace_free(Workspace* ws) {
  if (!ws) return;
  (void)wait_ws(ws);
  void* dev[] = {ws->d_desc, ws->d_work, ws->d_ctr, ws->d_bin_lo, ws->d_bin_hi,
                 ws->d_rec_pay, ws->d_rec_meta, ws->d_g_rbase, ws->d_g_nrec, ws->d_g_ninst, ws->d_g_krange,
                 ws->d_wave_cnt, ws->d_inst_key, ws->d_inst_val, ws->d_key2, ws->d_val2, ws->d_hist,
                 ws->d_scan_part, ws->d_moments, ws->d_ssim, ws->d_vox_rec, ws->d_vox_box, ws->d_vox_mom};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  void* host[] = {ws->h_desc, ws->h_ctr};
  for (void* p : host)
    if (p) (void)hipHostFree(p);
  (void)resolve_timings(ws);
  for (hipEvent_t e : ws->event_pool) (void)hipEventDestroy(e);
  if (ws->upload_done) (void)hipEventDestroy(ws->upload_done);
  delete ws;
}

}  // namespace gp

using namespace gp;

extern "C" {

int32_t gp_version(void) { return 100; }

const char* gp_last_error(void) { return g_err.c_str(); }

gp_status gp_default_opts(gp_render_opts* o) {
  if (!o) return einval("opts: NULL");
  o->q_cut = (float)(2.0 * std::log(255.0));
  o->bbox_sigmas = 3.0f;
  o->scale_mod = 1.0f;
  o->flags = 0u;
  return GP_OK;
}

gp_status gp_workspace_create(gp_workspace** out, int64_t max_records, int64_t max_instances) {
  if (!out) return einval("workspace_create: NULL");
  *out = nullptr;
  if (max_records < 0 || max_instances < 0) return einval("workspace_create: negative capacity");
  if ((max_records == 0) != (max_instances == 0))
    return einval("workspace_create: give both capacities or neither");
  Workspace* ws = nullptr;
  gp_status st = workspace_new(&ws, max_records, max_instances);
  if (st != GP_OK) return st;
  *out = reinterpret_cast<gp_workspace*>(ws);
  return GP_OK;
}

gp_status gp_workspace_destroy(gp_workspace* w) {
  workspace_free(reinterpret_cast<Workspace*>(w));
  return GP_OK;
}

gp_status gp_workspace_check(gp_workspace* w, int64_t* records, int64_t* instances, int64_t* bins) {
  if (!w) return einval("workspace_check: NULL");
  Workspace* ws = reinterpret_cast<Workspace*>(w);
  GP_HIP(wait_ws(ws));
  GP_HIP(hipMemcpy(ws->h_ctr, ws->d_ctr, sizeof(uint32_t) * kCtrCount, hipMemcpyDeviceToHost));
  if (records) *records = ws->h_ctr[kCtrRecords];
  if (instances) *instances = ws->h_ctr[kCtrInstances];
  if (bins) *bins = ws->have_forward ? ws->fwd_nbins : 0;
  if (ws->h_ctr[kCtrOverflow] || ws->overflowed) {
    ws->overflowed = false;
    GP_HIP(hipMemset(ws->d_ctr + kCtrOverflow, 0, sizeof(uint32_t)));
    set_error("a render overflowed the workspace capacity");
    return GP_EOVERFLOW;
  }
  return GP_OK;
}

// Camera poses of posed slices: finite, R_c a rotation (orthonormal to 1e-4,
// determinant > 0).
static gp_status check_poses(const float* poses, int ns) {
  for (int k = 0; k < ns; ++k) {
    const float* p = poses + 12 * (size_t)k;
    char buf[160];
    for (int i = 0; i < 12; ++i)
      if (!std::isfinite(p[i])) {
        snprintf(buf, sizeof buf, "pose %d: non-finite entry", k);
        return einval(buf);
      }
    double worst = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double d = 0.0;
        for (int i = 0; i < 3; ++i) d += (double)p[3 * r + i] * p[3 * c + i];
        worst = std::max(worst, std::fabs(d - (r == c ? 1.0 : 0.0)));
      }
    const double det = (double)p[0] * ((double)p[4] * p[8] - (double)p[5] * p[7]) -
                       (double)p[1] * ((double)p[3] * p[8] - (double)p[5] * p[6]) +
                       (double)p[2] * ((double)p[3] * p[7] - (double)p[4] * p[6]);
    if (worst > 1e-4 || !(det > 0.0)) {
      snprintf(buf, sizeof buf, "pose %d: R_c must be a rotation (|R R^T - I| = %.2e, det = %.3f)", k, worst, det);
      return einval(buf);
    }
  }
  return GP_OK;
}

static uint64_t slices_hash(const gp_slice* hs, const float* poses, int ns, const gp_render_opts* o) {
  uint64_t h = hash_bytes(hs, sizeof(gp_slice) * (size_t)ns, hash_bytes(o, sizeof(*o)));
  return poses ? hash_bytes(poses, sizeof(float) * 12 * (size_t)ns, h ^ 0x9e3779b97f4a7c15ull) : h;
}

gp_status gp_render_slices_posed(gp_workspace* w, const gp_gaussians* g, const gp_slice* hs, const float* poses,
                                 int32_t ns, const gp_render_opts* o, float* out, void* stream) {
  if (!w) return einval("render: NULL workspace");
  Workspace* ws = reinterpret_cast<Workspace*>(w);
  gp_status st = check_gaussians(g);
  if (st != GP_OK) return st;
  if ((st = check_opts(o)) != GP_OK) return st;
  if (ns < 0 || (ns > 0 && (!hs || !out))) return einval("render: bad slices/out");
  for (int k = 0; k < ns; ++k)
    if ((st = check_slice(hs[k], k)) != GP_OK) return st;
  if (poses && (st = check_poses(poses, ns)) != GP_OK) return st;
  GP_HIP(hipSetDevice(ws->device));
  ws->have_forward = false;
  ws->vox_have = false;
  if (ns == 0) return GP_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  GroupIn grp{g, 0, ns};
  BatchPlan plan{};
  if ((st = stage_batch(ws, &grp, 1, hs, ns, out, nullptr, &plan, poses)) != GP_OK) return st;
  if ((st = upload_batch(ws, plan, s)) != GP_OK) return st;
  LaunchDims d{plan.total_gauss, plan.nbins, emit_width_for(ns)};
  d.posed = poses ? 1 : 0;
  d.host_batch = 1;
  if ((st = enqueue_forward(ws, make_render_const(o, g->attr_dtype, ws), d, s)) != GP_OK) return st;
  ws->have_forward = true;
  ws->fwd_forward_only = (o->flags & GP_FLAG_FORWARD_ONLY) != 0;
  ws->fwd_means = g->means;
  ws->fwd_attrs = g->attrs;
  ws->fwd_n = g->n;
  ws->fwd_stride = g->stride;
  ws->fwd_nslices = ns;
  ws->fwd_nbins = (int32_t)plan.nbins;
  ws->fwd_gauss = plan.total_gauss;
  ws->fwd_posed = d.posed;
  ws->fwd_slice_hash = slices_hash(hs, poses, ns, o);
  return GP_OK;
}

gp_status gp_render_slices(gp_workspace* w, const gp_gaussians* g, const gp_slice* hs, int32_t ns,
                           const gp_render_opts* o, float* out, void* stream) {
  return gp_render_slices_posed(w, g, hs, nullptr, ns, o, out, stream);
}

gp_status gp_render_backward_posed(gp_workspace* w, const gp_gaussians* g, const gp_slice* hs, const float* poses,
                                   int32_t ns, const gp_render_opts* o, const float* grad_out, float* grad,
                                   int64_t grad_stride, void* stream) {
  if (!w) return einval("backward: NULL workspace");
  Workspace* ws = reinterpret_cast<Workspace*>(w);
  gp_status st = check_gaussians(g);
  if (st != GP_OK) return st;
  if ((st = check_opts(o)) != GP_OK) return st;
  if (grad_stride < g->n) return einval("backward: grad_stride < n");
  if (g->attr_dtype == GP_QM) return einval("backward: coded (GP_QM) Gaussians are render-only");
  if (ns < 0 || (ns > 0 && (!hs || !grad_out || !grad))) return einval("backward: bad arguments");
  if (!ws->have_forward || ws->fwd_forward_only || ws->fwd_means != g->means || ws->fwd_attrs != g->attrs ||
      ws->fwd_n != g->n ||
      ws->fwd_stride != g->stride || ws->fwd_nslices != ns || ws->fwd_posed != (poses ? 1 : 0) ||
      ws->fwd_slice_hash != slices_hash(hs, poses, ns, o)) {
    set_error("backward: the workspace does not hold the forward of these Gaussians and slices");
    return GP_ESTATE;
  }
  if (ns == 0 || g->n == 0) return GP_OK;
  GP_HIP(hipSetDevice(ws->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  LaunchDims d{ws->fwd_gauss, ws->fwd_nbins};
  d.posed = ws->fwd_posed;
  GP_HIP(timed(ws, GP_STAGE_RASTER_BWD, s, [&] { return launch_raster_bwd(ws->fwd_rc, *ws, grad_out, d, s); }));
  GP_HIP(timed(ws, GP_STAGE_PREPROCESS_BWD, s,
               [&] { return launch_preprocess_bwd(ws->fwd_rc, *ws, grad, grad_stride, d, s); }));
  ws->last_stream = s;
  return GP_OK;
}

gp_status gp_render_backward(gp_workspace* w, const gp_gaussians* g, const gp_slice* hs, int32_t ns,
                             const gp_render_opts* o, const float* grad_out, float* grad, int64_t grad_stride,
                             void* stream) {
  return gp_render_backward_posed(w, g, hs, nullptr, ns, o, grad_out, grad, grad_stride, stream);
}

gp_status gp_l1_loss_grad(const float* img, const float* tgt, int64_t n, float scale, float* grad, float* loss,
                          void* stream) {
  if (n < 0) return einval("l1: n < 0");
  if (n > 0 && (!img || !tgt || !grad)) return einval("l1: NULL array");
  GP_HIP(launch_l1(img, tgt, n, scale, grad, loss, static_cast<hipStream_t>(stream)));
  return GP_OK;
}

gp_status gp_l1_dssim_loss_grad(gp_workspace* w, const float* img, const float* tgt, int32_t n_slices,
                                int32_t width, int32_t height, float lambda, float* grad, float* loss,
                                void* stream) {
  if (!w) return einval("l1_dssim: NULL workspace");
  if (n_slices < 0 || width < 0 || height < 0 || n_slices > 65535) return einval("l1_dssim: bad sizes");
  if (!(lambda >= 0.f) || !std::isfinite(lambda)) return einval("l1_dssim: lambda must be finite and >= 0");
  const int64_t npix = (int64_t)n_slices * width * height;
  if (npix == 0) return GP_OK;
  if (!img || !tgt || !grad) return einval("l1_dssim: NULL array");
  Workspace* ws = reinterpret_cast<Workspace*>(w);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t need = ssim_scratch(n_slices, width, height);
  if (need > ws->ssim_cap) {
    GP_HIP(hipStreamSynchronize(s));
    GP_HIP(wait_ws(ws));
    hipError_t e = dev_alloc(&ws->d_ssim, need);
    if (e != hipSuccess) {
      ws->ssim_cap = 0;
      set_error("l1_dssim: cannot allocate scratch");
      return GP_ENOMEM;
    }
    ws->ssim_cap = need;
  }
  GP_HIP(launch_ssim_loss(img, tgt, n_slices, width, height, (double)lambda, ws->d_ssim, grad, loss, s));
  return GP_OK;
}

gp_status gp_l1_dssim_loss_grad_noalloc(const float* img, const float* tgt, int32_t n_slices, int32_t width,
                                        int32_t height, float lambda, float* grad, float* loss, void* stream) {
  if (n_slices < 0 || width < 0 || height < 0 || n_slices > 65535)
    return einval("l1_dssim_noalloc: bad sizes");
  if (!(lambda >= 0.f) || !std::isfinite(lambda)) return einval("l1_dssim_noalloc: lambda must be finite and >= 0");
  const int64_t npix = (int64_t)n_slices * width * height;
  if (npix == 0) return GP_OK;
  if (!img || !tgt || !grad) return einval("l1_dssim_noalloc: NULL array");
  const int64_t need = ssim_scratch(n_slices, width, height);
  if (need > ssim_noalloc_capacity())
    return einval("l1_dssim_noalloc: slices need " + std::to_string(need) + " float64 scratch elements, more than the " +
                  std::to_string(ssim_noalloc_capacity()) + " of the static scratch");
  double* scratch = nullptr;
  GP_HIP(ssim_noalloc_scratch(&scratch));
  GP_HIP(launch_ssim_loss(img, tgt, n_slices, width, height, (double)lambda, scratch, grad, loss,
                          static_cast<hipStream_t>(stream)));
  return GP_OK;
}

gp_status gp_adam_step(float* p, float* g, float* m, float* v, int64_t n, int64_t stride, const gp_adam_cfg* c,
                       void* stream) {
  if (!c) return einval("adam: NULL cfg");
  if (n < 0 || stride < n) return einval("adam: need 0 <= n <= stride");
  if (c->step < 1) return einval("adam: step must be >= 1");
  if (!(c->beta1 >= 0.f && c->beta1 < 1.f && c->beta2 >= 0.f && c->beta2 < 1.f && c->eps >= 0.f))
    return einval("adam: betas in [0,1), eps >= 0");
  if (c->flags & ~(GP_ADAM_CLAMP_ALPHA | GP_ADAM_ZERO_GRAD)) return einval("adam: unknown flag");
  if (n > 0 && (!p || !g || !m || !v)) return einval("adam: NULL array");
  GP_HIP(launch_adam(p, g, m, v, n, stride, *c, static_cast<hipStream_t>(stream)));
  return GP_OK;
}

gp_status gp_workspace_set_timing(gp_workspace* w, int32_t enable) {
  if (!w) return einval("set_timing: NULL");
  Workspace* ws = reinterpret_cast<Workspace*>(w);
  GP_HIP(resolve_timings(ws));
  for (int i = 0; i < GP_N_STAGES; ++i) {
    ws->stage_ms[i] = 0.0;
    ws->stage_n[i] = 0;
  }
  ws->timing = (uint32_t)enable & ((1u << GP_N_STAGES) - 1u);
  return GP_OK;
}

gp_status gp_workspace_timings(gp_workspace* w, double* ms, int64_t* counts, int32_t n) {
  if (!w || n < 0 || (n > 0 && (!ms || !counts))) return einval("timings: bad arguments");
  Workspace* ws = reinterpret_cast<Workspace*>(w);
  GP_HIP(resolve_timings(ws));
  for (int i = 0; i < n; ++i) {
    ms[i] = i < GP_N_STAGES ? ws->stage_ms[i] : 0.0;
    counts[i] = i < GP_N_STAGES ? ws->stage_n[i] : 0;
  }
  return GP_OK;
}

static gp_status check_grid(const gp_volume_grid* v) {
  if (!v) return einval("voxelize: NULL grid");
  if (v->nx < 0 || v->ny < 0 || v->nz < 0) return einval("voxelize: negative grid size");
  const float h[3] = {v->dx, v->dy, v->dz};
  const float o[3] = {v->x0, v->y0, v->z0};
  for (int a = 0; a < 3; ++a)
    if (!(h[a] > 0.f) || !std::isfinite(h[a]) || !std::isfinite(o[a])) return einval("voxelize: bad pitch or origin");
  if ((int64_t)v->nx > (8ll << 16) || (int64_t)v->ny > (8ll << 16) || (int64_t)v->nz > (8ll << 16))
    return einval("voxelize: more than 2^19 voxels along an axis");
  return GP_OK;
}

static gp_status reserve_vox(Workspace* ws, int64_t n, int64_t inst) {
  if (n > ws->vox_gcap) {
    GP_HIP(wait_ws(ws));
    const int64_t cap = n + n / 8 + 64;
    if (dev_alloc(&ws->d_vox_rec, 3 * cap) != hipSuccess || dev_alloc(&ws->d_vox_box, 3 * cap) != hipSuccess) {
      ws->vox_gcap = 0;
      set_error("voxelize: out of device memory");
      return GP_ENOMEM;
    }
    ws->vox_gcap = cap;
  }
  if (inst > ws->vox_icap) {
    GP_HIP(wait_ws(ws));
    if (dev_alloc(&ws->d_vox_mom, 3 * inst) != hipSuccess) {
      ws->vox_icap = 0;
      set_error("voxelize: out of device memory");
      return GP_ENOMEM;
    }
    ws->vox_icap = inst;
  }
  return GP_OK;
}

gp_status gp_voxelize(gp_workspace* w, const gp_gaussians* g, const gp_volume_grid* grid, const gp_render_opts* o,
                      float* vol, void* stream) {
  if (!w) return einval("voxelize: NULL workspace");
  Workspace* ws = reinterpret_cast<Workspace*>(w);
  gp_status st = check_gaussians(g);
  if (st != GP_OK) return st;
  if ((st = check_opts(o)) != GP_OK) return st;
  if ((st = check_grid(grid)) != GP_OK) return st;
  if (g->attr_dtype == GP_QM) return einval("voxelize: coded (GP_QM) Gaussians are not supported");
  const int64_t nvox = (int64_t)grid->nx * grid->ny * grid->nz;
  if (nvox > 0 && !vol) return einval("voxelize: NULL volume");
  if (g->n > 0x7FFFFFF0ll) return einval("voxelize: too many Gaussians");
  GP_HIP(hipSetDevice(ws->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  ws->have_forward = false;
  ws->vox_have = false;
  if (nvox == 0) return GP_OK;
  const VoxLaunch L = vox_prepare(g, grid, o);
  if (L.n_tiles >= (1ll << 30)) return einval("voxelize: more than 2^30 tiles");
  if (L.n == 0) {
    GP_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(vol), 0u, nvox, s));
  } else {
    if ((st = reserve_small(ws, 0, 0, L.n_tiles, L.n)) != GP_OK) return st;
    if ((st = reserve_vox(ws, L.n, 0)) != GP_OK) return st;
    const int64_t part = scan_parts_needed(L.n);
    if (part > ws->part_cap) {
      GP_HIP(wait_ws(ws));
      GP_HIP(dev_alloc(&ws->d_scan_part, part));
      ws->part_cap = part;
    }
    ws->last_stream = s;
    GP_HIP(launch_vox_count(*ws, g, grid, o, L, s));
    GP_HIP(launch_scan_u32(ws->d_g_ninst, ws->d_g_rbase, nullptr, L.n, reinterpret_cast<uint32_t*>(ws->d_scan_part),
                           ws->d_ctr + kCtrInstances, s));
    GP_HIP(hipMemcpyAsync(ws->h_ctr, ws->d_ctr, sizeof(uint32_t) * kCtrCount, hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    const int64_t K = ws->h_ctr[kCtrInstances];
    if ((st = reserve_lists(ws, 0, std::max<int64_t>(K, 1))) != GP_OK) return st;
    if ((st = reserve_vox(ws, L.n, ws->inst_cap)) != GP_OK) return st;
    const int bits = key_bits(L.n_tiles);
    if ((st = reserve_sort(ws, bits)) != GP_OK) return st;
    ws->last_stream = s;
    GP_HIP(launch_vox_emit(*ws, g, grid, o, L, s));
    GP_HIP(launch_radix_sort(ws->d_inst_key, ws->d_inst_val, ws->d_key2, ws->d_val2, ws->d_ctr + kCtrInstances, nullptr,
                             std::max<int64_t>(K, 1), bits, ws->d_hist, reinterpret_cast<uint32_t*>(ws->d_scan_part),
                             s, &ws->d_list_key, &ws->d_list));
    GP_HIP(launch_vox_ranges(*ws, L, (uint32_t)K, s));
    GP_HIP(launch_vox_fwd(*ws, g, grid, o, L, vol, s));
  }
  ws->vox_have = true;
  ws->vox_ntiles = L.n == 0 ? 0 : L.n_tiles;
  ws->vox_ninst = L.n == 0 ? 0 : (int64_t)ws->h_ctr[kCtrInstances];
  ws->vox_means = g->means;
  ws->vox_attrs = g->attrs;
  ws->vox_n = g->n;
  ws->vox_stride = g->stride;
  ws->vox_hash = hash_bytes(grid, sizeof(*grid), hash_bytes(o, sizeof(*o)));
  return GP_OK;
}

gp_status gp_voxelize_backward(gp_workspace* w, const gp_gaussians* g, const gp_volume_grid* grid,
                               const gp_render_opts* o, const float* gvol, float* grad, int64_t grad_stride,
                               void* stream) {
  if (!w) return einval("voxelize_backward: NULL workspace");
  Workspace* ws = reinterpret_cast<Workspace*>(w);
  gp_status st = check_gaussians(g);
  if (st != GP_OK) return st;
  if ((st = check_opts(o)) != GP_OK) return st;
  if ((st = check_grid(grid)) != GP_OK) return st;
  if (grad_stride < g->n) return einval("voxelize_backward: grad_stride < n");
  const int64_t nvox = (int64_t)grid->nx * grid->ny * grid->nz;
  if (!ws->vox_have || ws->vox_means != g->means || ws->vox_attrs != g->attrs || ws->vox_n != g->n ||
      ws->vox_stride != g->stride || ws->vox_hash != hash_bytes(grid, sizeof(*grid), hash_bytes(o, sizeof(*o)))) {
    set_error("voxelize_backward: the workspace does not hold the voxelisation of these Gaussians and grid");
    return GP_ESTATE;
  }
  if (nvox == 0 || g->n == 0) return GP_OK;
  if (!gvol || !grad) return einval("voxelize_backward: NULL array");
  GP_HIP(hipSetDevice(ws->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const VoxLaunch L = vox_prepare(g, grid, o);
  ws->last_stream = s;
  GP_HIP(launch_vox_bwd(*ws, g, grid, o, L, gvol, grad, grad_stride, s));
  return GP_OK;
}

gp_status gp_encode(const float* p, int64_t n, int64_t stride, uint16_t* codes, int64_t stride_out, uint32_t* perm,
                    float* d_header, void* stream) {
  if (n < 0 || stride < n || stride_out < n || n >= (1ll << 31)) return einval("encode: need 0 <= n <= strides");
  if (!d_header || (n > 0 && (!p || !codes))) return einval("encode: NULL");
  return encode_volume(p, p ? p + 3 * stride : nullptr, n, stride, codes, stride_out, perm, d_header,
                       static_cast<hipStream_t>(stream));
}

gp_status gp_densify_default_cfg(gp_densify_cfg* c) {
  if (!c) return einval("densify_default_cfg: NULL");
  c->grad_threshold = 5e-5f;
  c->min_alpha = 0.02f;
  c->max_radius = 256.0f;
  c->split_scale = 2.0f;
  c->split_factor = 1.6f;
  c->flags = 0u;
  return GP_OK;
}

gp_status gp_workspace_set_densify_stats(gp_workspace* w, float* grad_norm, int32_t* count, float* max_radius,
                                         int64_t n) {
  if (!w) return einval("set_densify_stats: NULL workspace");
  const bool off = !grad_norm && !count && !max_radius;
  if (!off && (!grad_norm || !count || !max_radius || n < 0)) return einval("set_densify_stats: give all or none");
  Workspace* ws = reinterpret_cast<Workspace*>(w);
  ws->st_grad_norm = off ? nullptr : grad_norm;
  ws->st_count = off ? nullptr : count;
  ws->st_max_radius = off ? nullptr : max_radius;
  ws->st_n = off ? 0 : n;
  return GP_OK;
}

gp_status gp_densify_prune(const float* p, const float* m, const float* v, int64_t n, int64_t stride,
                           const float* grad_norm, const int32_t* count, const float* max_radius, const float* noise,
                           const gp_densify_cfg* cfg, float* p_out, float* m_out, float* v_out, int64_t stride_out,
                           int64_t* n_out, void* stream) {
  if (!cfg || !n_out) return einval("densify: NULL");
  if (n < 0 || stride < n || n >= (1ll << 31)) return einval("densify: need 0 <= n <= stride");
  if (n > 0 && (!p || !m || !v || !grad_norm || !count || !max_radius || !noise || !p_out || !m_out || !v_out))
    return einval("densify: NULL array");
  if (!(cfg->split_factor > 0.f) || cfg->flags != 0u) return einval("densify: bad configuration");
  *n_out = 0;
  if (n == 0) return GP_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t *action = nullptr, *outs = nullptr, *part = nullptr, *total = nullptr;
  const int64_t nparts = scan_parts_needed(n);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&action), sizeof(uint32_t) * n);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&outs), sizeof(uint32_t) * n);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&part), sizeof(uint32_t) * nparts);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&total), sizeof(uint32_t));
  uint32_t h_total = 0;
  if (e == hipSuccess)
    e = launch_densify(p, m, v, n, stride, grad_norm, count, max_radius, noise, *cfg, action, outs, part, total,
                       p_out, m_out, v_out, stride_out, false, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&h_total, total, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  gp_status st = GP_OK;
  if (e == hipSuccess) {
    *n_out = h_total;
    if ((int64_t)h_total > stride_out) {
      set_error("densify: output stride too small");
      st = GP_EOVERFLOW;
    } else {
      e = launch_densify(p, m, v, n, stride, grad_norm, count, max_radius, noise, *cfg, action, outs, part, total,
                         p_out, m_out, v_out, stride_out, true, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
  }
  if (e != hipSuccess) st = hip_fail(e, "densify");
  (void)hipFree(action);
  (void)hipFree(outs);
  (void)hipFree(part);
  (void)hipFree(total);
  return st;
}

gp_status gp_debug_export_bins(gp_workspace* w, uint64_t* h_keys, int64_t keys_cap, int64_t* n_keys,
                               int64_t* h_ranges, int64_t ranges_cap) {
  if (!w || !n_keys) return einval("export_bins: NULL");
  Workspace* ws = reinterpret_cast<Workspace*>(w);
  if (!ws->have_forward && !ws->vox_have) {
    set_error("export_bins: no forward in this workspace");
    return GP_ESTATE;
  }
  GP_HIP(wait_ws(ws));
  if (ws->vox_have) {
    // voxelisation: the lists hold Gaussian indices directly
    const int64_t nb = ws->vox_ntiles, K = ws->vox_ninst;
    *n_keys = K;
    if (keys_cap < K || ranges_cap < 2 * nb || (K > 0 && !h_keys) || (nb > 0 && !h_ranges))
      return einval("export_bins: output too small");
    std::vector<uint32_t> lo((size_t)std::max<int64_t>(nb, 1)), hi((size_t)std::max<int64_t>(nb, 1)),
        list((size_t)std::max<int64_t>(K, 1));
    if (nb > 0) {
      GP_HIP(hipMemcpy(lo.data(), ws->d_bin_lo, sizeof(uint32_t) * nb, hipMemcpyDeviceToHost));
      GP_HIP(hipMemcpy(hi.data(), ws->d_bin_hi, sizeof(uint32_t) * nb, hipMemcpyDeviceToHost));
    }
    if (K > 0) GP_HIP(hipMemcpy(list.data(), ws->d_list, sizeof(uint32_t) * K, hipMemcpyDeviceToHost));
    int64_t o = 0;
    for (int64_t b = 0; b < nb; ++b) {
      h_ranges[2 * b] = o;
      for (uint32_t i = lo[b]; i < hi[b]; ++i) h_keys[o++] = ((uint64_t)b << 32) | list[i];
      h_ranges[2 * b + 1] = o;
    }
    return GP_OK;
  }
  const int64_t nb = ws->fwd_nbins;
  std::vector<uint32_t> lo((size_t)nb), hi((size_t)nb);
  if (nb > 0) {
    GP_HIP(hipMemcpy(lo.data(), ws->d_bin_lo, sizeof(uint32_t) * nb, hipMemcpyDeviceToHost));
    GP_HIP(hipMemcpy(hi.data(), ws->d_bin_hi, sizeof(uint32_t) * nb, hipMemcpyDeviceToHost));
  }
  GP_HIP(hipMemcpy(ws->h_ctr, ws->d_ctr, sizeof(uint32_t) * kCtrCount, hipMemcpyDeviceToHost));
  int64_t K = 0;
  for (int64_t b = 0; b < nb; ++b) K += hi[b] - lo[b];
  *n_keys = K;
  if (keys_cap < K || ranges_cap < 2 * nb || (K > 0 && !h_keys) || (nb > 0 && !h_ranges))
    return einval("export_bins: output too small");
  const int64_t n_list = std::min<int64_t>(ws->h_ctr[kCtrInstances], ws->inst_cap);
  const int64_t R = std::min<int64_t>(ws->h_ctr[kCtrRecords], ws->rec_cap);
  std::vector<uint32_t> list((size_t)std::max<int64_t>(n_list, 1));
  if (n_list > 0) GP_HIP(hipMemcpy(list.data(), ws->d_list, sizeof(uint32_t) * n_list, hipMemcpyDeviceToHost));
  // records are contiguous per Gaussian: record -> Gaussian index within its set
  const int64_t T = ws->fwd_gauss;
  std::vector<uint32_t> rbase((size_t)std::max<int64_t>(T, 1)), nrec((size_t)std::max<int64_t>(T, 1));
  if (T > 0) {
    GP_HIP(hipMemcpy(rbase.data(), ws->d_g_rbase, sizeof(uint32_t) * T, hipMemcpyDeviceToHost));
    GP_HIP(hipMemcpy(nrec.data(), ws->d_g_nrec, sizeof(uint32_t) * T, hipMemcpyDeviceToHost));
  }
  std::vector<uint32_t> gid((size_t)std::max<int64_t>(R, 1), 0xFFFFFFFFu);
  const int ng = ws->h_hdr->n_groups;
  for (int64_t t = 0; t < T; ++t) {
    int64_t gb = 0;
    for (int g = 0; g < ng; ++g)
      if (ws->h_groups[g].gbase <= t) gb = ws->h_groups[g].gbase;
    for (uint32_t r = rbase[t]; r < rbase[t] + nrec[t] && r < (uint32_t)R; ++r) gid[r] = (uint32_t)(t - gb);
  }
  // lists are contiguous and in bin order; report them packed, bin by bin
  int64_t o = 0;
  for (int64_t b = 0; b < nb; ++b) {
    h_ranges[2 * b] = o;
    for (uint32_t i = lo[b]; i < hi[b]; ++i) h_keys[o++] = ((uint64_t)b << 32) | gid[list[i]];
    h_ranges[2 * b + 1] = o;
  }
  return GP_OK;
}

}  // extern "C"
