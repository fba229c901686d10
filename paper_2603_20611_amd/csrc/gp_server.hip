// Serving of slices from resident volumes (continuous batching).
//
// A scheduler thread owns the launch slots.  Whenever a slot is free and
// requests are queued it takes a batch from the head of the queue (bounded by
// the slot's capacity for requests, tiles, Gaussians and estimated list
// entries), stages one descriptor table for the whole batch (one group per
// volume, one slice per request, each slice writing into its caller's
// buffer), uploads it on the slot's stream and replays the slot's captured
// hipGraph of the forward launch sequence (reset, preprocess, bin scan,
// scatter, per-tile sort, rasterise).  A host function queued behind the batch
// wakes the scheduler when it finishes, so new requests are admitted while
// other batches are still on the GPU.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gp_internal.h"

namespace gp {
namespace {

using Clock = std::chrono::steady_clock;

double now_ms() {
  return std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
}

// float32 [11][src_stride] -> float32 means [3][dst_stride] + attrs [8][dst_stride] of type DT
template <int DT>
__global__ void k_pack_volume(const float* __restrict__ means, const float* __restrict__ attrs, int64_t src_stride,
                              int64_t n, float* __restrict__ out_means, void* __restrict__ out_attrs,
                              int64_t dst_stride) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int r = 0; r < 3; ++r) out_means[r * dst_stride + i] = means[r * src_stride + i];
  float v[8];
  for (int r = 0; r < 8; ++r) v[r] = attrs[r * src_stride + i];
  if constexpr (DT == GP_Q16) {
#pragma clang fp contract(off)
    // unit quaternion in int16 fixed point (the binary32 rule in the header)
    const float n2 = ((v[3] * v[3] + v[4] * v[4]) + v[5] * v[5]) + v[6] * v[6];
    const float rn = sqrtf(n2);
    for (int r = 3; r < 7; ++r) {
      float qn = v[r] / rn;
      qn = (n2 > 0.0f && isfinite(qn)) ? qn : 0.0f;
      const float q = fminf(fmaxf(rintf(qn * 32767.0f), -32767.0f), 32767.0f);
      static_cast<int16_t*>(out_attrs)[r * dst_stride + i] = (int16_t)q;
    }
    for (int r : {0, 1, 2, 7}) static_cast<__half*>(out_attrs)[r * dst_stride + i] = __float2half(v[r]);
  } else {
    for (int r = 0; r < 8; ++r) {
      if constexpr (DT == GP_BF16) {
        static_cast<__hip_bfloat16*>(out_attrs)[r * dst_stride + i] = __float2bfloat16(v[r]);
      } else if constexpr (DT == GP_F16) {
        static_cast<__half*>(out_attrs)[r * dst_stride + i] = __float2half(v[r]);
      } else {
        static_cast<float*>(out_attrs)[r * dst_stride + i] = v[r];
      }
    }
  }
}

size_t dtype_bytes(int dt) { return dt == GP_F32 ? 4 : 2; }

struct Volume {
  float* means = nullptr;
  void* attrs = nullptr;
  int64_t n = 0, stride = 0;
  size_t bytes = 0;
  // admission estimate: for each sigma_z of kSigmaGrid, cover[k][b] = the
  // Gaussians whose axial window (q_ax <= q_cut) reaches unit depth bin b
  // (from z_lo); and the mean and mean square of each Gaussian's lateral
  // footprint width, 2 bbox sqrt(max(Sigma_xx, Sigma_yy)) in world units
  float z_lo = 0.f;
  int nbins = 0;
  std::vector<int32_t> cover;   // [kSigmaGrid][nbins]
  double foot_m1 = 0.0, foot_m2 = 0.0;
};

// Where a volume's resident planes are.  Copied into each request when it is
// taken into a batch (under the server lock), so that launching the batch never
// reads the volume table, which gp_server_add_volume may grow meanwhile.
struct VolView {
  const void* means = nullptr;
  const void* attrs = nullptr;
  int64_t n = 0, stride = 0;
};

struct Request {
  uint64_t ticket;
  gp_request r;
  float* out;
  double t_submit;
  bool solo;       // render alone (after an overflow)
  VolView vol{};   // set by take_batch
};

struct TicketState {
  bool done = false;
  gp_serve_result res{};
};

struct Server;

// Launch capacities of a batch: flattened Gaussians and bins the launch grids
// cover, records and tile-list entries it may fill.  Each slot has one
// captured graph per bucket and a batch replays the smallest whose capacities
// cover it (empty workgroups of a launch sized for the largest batch cost
// time at light load); a batch that still overflows a smaller bucket reruns
// in the largest.
struct Bucket {
  int64_t gauss, bins, rec, inst;
};
constexpr int kMaxBuckets = 3;
// The captured launches sort list entries by the low 14 bits of their bin:
// enough for a group (one volume's consecutive requests) of up to 16,383
// tiles, four 1024^2 slices.  Larger groups are split; a single request of
// more tiles is launched without the graphs, with the bits it needs.
constexpr int64_t kGroupSortBins = 16383;

struct Slot {
  Server* sv = nullptr;
  Workspace* ws = nullptr;
  hipStream_t stream = nullptr;
  hipGraphExec_t exec[kMaxBuckets] = {};
  std::vector<Request> reqs;
  bool busy = false, finished = false;
  bool rerun = false;         // overflowed a smaller bucket: replay the largest
  int bucket = 0;
  int64_t group_bins = 0;     // the most bins of one group of the batch
  double est_rec = 0.0, est_inst = 0.0;   // admission estimates of the batch
  int64_t batch_id = 0;
  double t_done = 0.0;
};

struct Server {
  gp_server_cfg cfg{};
  std::vector<Volume> vols;
  int64_t resident = 0;
  std::mutex mu;
  std::condition_variable cv;       // scheduler wake-up
  std::condition_variable cv_done;  // pollers
  std::deque<Request> queue;
  std::unordered_map<uint64_t, TicketState> tickets;
  std::vector<Slot*> slots;
  std::thread sched;
  bool stop = false;
  uint64_t next_ticket = 1;
  int64_t next_batch = 1;
  double tiles_factor = 1.0;        // grows after an overflow
  gp_server_stats stats{};
  RenderConst rc{};
  LaunchDims cap_dims{};
  std::vector<Bucket> buckets;      // ascending; the last is the full capacity
};

int64_t tiles_of(const gp_request& r) {
  return (int64_t)((r.width + kTile - 1) / kTile) * ((r.height + kTile - 1) / kTile);
}

// sigma_z values of the admission tables (a request takes the first one at
// least its own; beyond the last, every Gaussian counts)
constexpr float kSigmaGrid[] = {0.f, 0.25f, 0.5f, 0.75f, 1.f, 1.5f, 2.f, 3.f, 4.f, 6.f, 8.f, 12.f, 16.f, 32.f};
constexpr int kNSigma = sizeof(kSigmaGrid) / sizeof(kSigmaGrid[0]);

// Records of a request: the Gaussians of its volume whose axial window at the
// tabulated sigma_z at least the request's reaches the slice's depth bin (an
// upper bound of the records up to the bin's width).
double est_records(const Server* sv, const gp_request& r) {
  const Volume& v = sv->vols[r.volume_id];
  int k = 0;
  while (k < kNSigma && kSigmaGrid[k] < r.sigma_z) ++k;
  if (k == kNSigma || !std::isfinite(r.z)) return (double)v.n;
  const double u = (double)r.z - v.z_lo;
  if (u < 0.0 || u >= (double)v.nbins) {
    // outside the tabulated range: the nearest bin's coverage
    const int b = u < 0.0 ? 0 : v.nbins - 1;
    return (double)v.cover[(size_t)k * v.nbins + b];
  }
  return (double)v.cover[(size_t)k * v.nbins + (int)u];
}

// Tile-list entries of a request: its records times the expected tiles of a
// footprint box over the volume's Gaussians, E[(w / (16 dx) + 1) (w / (16 dy) + 1)]
// (scaled up after each overflow).
double est_instances(const Server* sv, const gp_request& r, double records) {
  const Volume& v = sv->vols[r.volume_id];
  const double ax = 1.0 / (kTile * (double)r.dx), ay = 1.0 / (kTile * (double)r.dy);
  const double per = v.foot_m2 * ax * ay + v.foot_m1 * (ax + ay) + 1.0;
  return records * per * sv->tiles_factor;
}

// The slot's forward launch sequence at the server's capacity, captured once
// when the server is created: the kernels read the batch's sizes from the
// descriptors uploaded before each replay.  Capturing then, in the creating
// thread, keeps any capture away from the time when other threads issue work
// (a capture in progress makes work on the legacy stream fail).
void on_batch_done(void* p);

gp_status capture_slot(Server* sv, Slot* sl) {
  for (size_t b = 0; b < sv->buckets.size(); ++b) {
    const Bucket& k = sv->buckets[b];
    hipGraph_t graph = nullptr;
    GP_HIP(hipStreamBeginCapture(sl->stream, hipStreamCaptureModeThreadLocal));
    LaunchDims d{k.gauss, k.bins};
    d.sort_bins = kGroupSortBins;
    const gp_status st = enqueue_forward(sl->ws, sv->rc, d, sl->stream, k.rec, k.inst);
    hipError_t e = hipStreamEndCapture(sl->stream, &graph);
    if (st != GP_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&sl->exec[b], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  }
  return GP_OK;
}

// The smallest bucket that covers the batch (its exact Gaussians and bins, its
// estimated records and entries with a margin).
int pick_bucket(const Server* sv, const BatchPlan& plan, double est_rec, double est_inst) {
  const int last = (int)sv->buckets.size() - 1;
  for (int b = 0; b < last; ++b) {
    const Bucket& k = sv->buckets[b];
    if (plan.total_gauss <= k.gauss && plan.nbins <= k.bins && 1.5 * est_rec <= (double)k.rec &&
        1.5 * est_inst <= (double)k.inst)
      return b;
  }
  return last;
}

// Launches the slot's batch (descriptors already uploaded) in bucket b.
gp_status launch_bucket(Server* sv, Slot* sl, const BatchPlan* plan, int b) {
  Workspace* ws = sl->ws;
  sl->bucket = b;
  const Bucket& k = sv->buckets[b];
  if (sv->cfg.use_graphs && sl->group_bins <= kGroupSortBins) {
    GP_HIP(hipGraphLaunch(sl->exec[b], sl->stream));
  } else {
    LaunchDims d = plan ? LaunchDims{plan->total_gauss, plan->nbins} : LaunchDims{k.gauss, k.bins};
    d.sort_bins = sl->group_bins;
    const gp_status st = enqueue_forward(ws, sv->rc, d, sl->stream, k.rec, k.inst);
    if (st != GP_OK) return st;
  }
  GP_HIP(hipMemcpyAsync(ws->h_ctr, ws->d_ctr, sizeof(uint32_t) * kCtrCount, hipMemcpyDeviceToHost, sl->stream));
  GP_HIP(hipLaunchHostFunc(sl->stream, on_batch_done, sl));
  return GP_OK;
}

void on_batch_done(void* p) {
  Slot* sl = static_cast<Slot*>(p);
  Server* sv = sl->sv;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sl->finished = true;
    sl->t_done = now_ms();
  }
  sv->cv.notify_all();
}

gp_status launch_batch(Server* sv, Slot* sl) {
  Workspace* ws = sl->ws;
  auto& reqs = sl->reqs;
  std::stable_sort(reqs.begin(), reqs.end(),
                   [](const Request& a, const Request& b) { return a.r.volume_id < b.r.volume_id; });
  std::vector<gp_gaussians> sets;
  std::vector<GroupIn> groups;
  std::vector<gp_slice> hs(reqs.size());
  std::vector<float*> outs(reqs.size());
  sets.reserve(reqs.size());
  int64_t group_tiles = 0;
  for (size_t k = 0; k < reqs.size(); ++k) {
    const gp_request& r = reqs[k].r;
    hs[k] = gp_slice{r.z, r.sigma_z, r.x0, r.y0, r.dx, r.dy, r.width, r.height};
    outs[k] = reqs[k].out;
    // a new group for a new volume, or where the group would outgrow the
    // captured sort's bits
    const int64_t t = tiles_of(r);
    if (groups.empty() || sets.back().means != reqs[k].vol.means || group_tiles + t > kGroupSortBins) {
      group_tiles = 0;
      const VolView& v = reqs[k].vol;
      sets.push_back(gp_gaussians{v.means, v.attrs, v.n, v.stride,
                                  sv->cfg.attr_dtype == GP_QM ? GP_QM : GP_F32, sv->cfg.attr_dtype});
      groups.push_back(GroupIn{nullptr, (int32_t)k, (int32_t)k + 1});
    } else {
      groups.back().k1 = (int32_t)k + 1;
    }
    group_tiles += t;
  }
  for (size_t g = 0; g < groups.size(); ++g) groups[g].g = &sets[g];
  BatchPlan plan{};
  gp_status st = stage_batch(ws, groups.data(), (int)groups.size(), hs.data(), (int)hs.size(), nullptr,
                             outs.data(), &plan);
  if (st != GP_OK) return st;
  sl->group_bins = plan.max_group_bins;
  if ((st = upload_batch(ws, plan, sl->stream)) != GP_OK) return st;
  return launch_bucket(sv, sl, &plan, pick_bucket(sv, plan, sl->est_rec, sl->est_inst));
}

// Called with the lock held: completes a finished slot's requests.  Returns
// true if the batch overflowed a smaller bucket and must be replayed in the
// largest (the slot stays busy).
bool retire(Server* sv, Slot* sl) {
  const bool overflow = sl->ws->h_ctr[kCtrOverflow] != 0;
  if (overflow && sl->bucket + 1 < (int)sv->buckets.size()) {
    sl->finished = false;
    sl->rerun = true;
    return true;
  }
  if (overflow && sl->reqs.size() > 1) {
    // re-run each request alone, at the head of the queue, in the original order
    sv->tiles_factor *= 1.5;
    for (auto it = sl->reqs.rbegin(); it != sl->reqs.rend(); ++it) {
      Request r = *it;
      r.solo = true;
      sv->queue.push_front(r);
    }
    sv->stats.retries += (int64_t)sl->reqs.size();
  } else {
    for (const Request& r : sl->reqs) {
      TicketState& t = sv->tickets[r.ticket];
      t.done = true;
      t.res.status = overflow ? GP_EOVERFLOW : GP_OK;
      t.res.batch_size = (int32_t)sl->reqs.size();
      t.res.batch_id = sl->batch_id;
      t.res.latency_ms = sl->t_done - r.t_submit;
      sv->stats.completed += 1;
    }
  }
  sl->reqs.clear();
  sl->busy = false;
  sl->finished = false;
  return false;
}

// Takes a batch from the head of the queue (lock held).  Returns false if empty.
bool take_batch(Server* sv, Slot* sl) {
  if (sv->queue.empty()) return false;
  int64_t bins = 0, gauss = 0;
  double inst = 0.0, recs = 0.0;
  // volumes in the batch and the tiles of each one's last group (launch_batch
  // groups a volume's requests in this order and starts a new group, which
  // counts the volume's Gaussians again, past kGroupSortBins tiles)
  std::vector<int32_t> vols_in;
  std::vector<int64_t> vol_tiles;
  sl->est_rec = sl->est_inst = 0.0;
  while (!sv->queue.empty() && (int)sl->reqs.size() < sv->cfg.max_batch) {
    const Request& r = sv->queue.front();
    if (r.solo && !sl->reqs.empty()) break;
    const size_t vi = (size_t)(std::find(vols_in.begin(), vols_in.end(), r.r.volume_id) - vols_in.begin());
    const bool new_vol = vi == vols_in.size();
    const int64_t t = tiles_of(r.r);
    const bool new_group = new_vol || vol_tiles[vi] + t > kGroupSortBins;
    const int64_t add_g = new_group ? (sv->vols[r.r.volume_id].n + 63) / 64 * 64 : 0;
    const double add_r = est_records(sv, r.r);
    const double add_i = est_instances(sv, r.r, add_r);
    if (!sl->reqs.empty() && (bins + tiles_of(r.r) > sv->cfg.max_bins || gauss + add_g > sv->cfg.max_gaussians ||
                              inst + add_i > (double)sv->cfg.max_instances ||
                              recs + add_r > (double)sv->cfg.max_records))
      break;
    bins += t;
    gauss += add_g;
    inst += add_i;
    recs += add_r;
    if (new_vol) {
      vols_in.push_back(r.r.volume_id);
      vol_tiles.push_back(t);
    } else {
      vol_tiles[vi] = new_group ? t : vol_tiles[vi] + t;
    }
    sl->reqs.push_back(r);
    const Volume& v = sv->vols[r.r.volume_id];
    sl->reqs.back().vol = VolView{v.means, v.attrs, v.n, v.stride};
    const bool solo = r.solo;
    sv->queue.pop_front();
    if (solo) break;
  }
  sl->est_rec = recs;
  sl->est_inst = inst;
  return true;
}

void scheduler(Server* sv) {
  (void)hipSetDevice(sv->cfg.device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    bool progressed = false;
    std::vector<Slot*> reruns;
    for (Slot* sl : sv->slots) {
      if (sl->busy && sl->finished) {
        if (retire(sv, sl)) reruns.push_back(sl);
        else progressed = true;
      }
    }
    if (progressed) sv->cv_done.notify_all();
    for (Slot* sl : reruns) {
      sl->rerun = false;
      sv->stats.retries += (int64_t)sl->reqs.size();
      lk.unlock();
      const gp_status st = launch_bucket(sv, sl, nullptr, (int)sv->buckets.size() - 1);
      lk.lock();
      if (st != GP_OK) {
        for (const Request& r : sl->reqs) {
          TicketState& t = sv->tickets[r.ticket];
          t.done = true;
          t.res.status = st;
          t.res.batch_id = sl->batch_id;
          sv->stats.completed += 1;
        }
        sl->reqs.clear();
        sl->busy = false;
        sv->cv_done.notify_all();
      }
    }
    if (sv->stop) {
      bool any_busy = false;
      for (Slot* sl : sv->slots) any_busy = any_busy || sl->busy;
      if (!any_busy) break;
      sv->cv.wait(lk);
      continue;
    }
    Slot* free_slot = nullptr;
    for (Slot* sl : sv->slots)
      if (!sl->busy) { free_slot = sl; break; }
    if (free_slot && take_batch(sv, free_slot)) {
      free_slot->busy = true;
      free_slot->batch_id = sv->next_batch++;
      sv->stats.batches += 1;
      lk.unlock();
      const gp_status st = launch_batch(sv, free_slot);
      lk.lock();
      if (st != GP_OK) {
        for (const Request& r : free_slot->reqs) {
          TicketState& t = sv->tickets[r.ticket];
          t.done = true;
          t.res.status = st;
          t.res.batch_id = free_slot->batch_id;
          sv->stats.completed += 1;
        }
        free_slot->reqs.clear();
        free_slot->busy = false;
        sv->cv_done.notify_all();
      }
      continue;
    }
    sv->cv.wait(lk);
  }
  // cancel what is still queued
  for (const Request& r : sv->queue) {
    TicketState& t = sv->tickets[r.ticket];
    t.done = true;
    t.res.status = GP_ECANCELED;
  }
  sv->queue.clear();
  sv->cv_done.notify_all();
}

void free_server(Server* sv) {
  for (Slot* sl : sv->slots) {
    if (sl->stream) (void)hipStreamSynchronize(sl->stream);
    for (hipGraphExec_t x : sl->exec)
      if (x) (void)hipGraphExecDestroy(x);
    if (sl->ws) workspace_free(sl->ws);
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
    delete sl;
  }
  for (Volume& v : sv->vols) {
    if (v.means) (void)hipFree(v.means);
    if (v.attrs) (void)hipFree(v.attrs);
  }
  delete sv;
}

}  // namespace
}  // namespace gp

using namespace gp;

extern "C" {

gp_status gp_server_default_cfg(gp_server_cfg* c) {
  if (!c) {
    set_error("server_default_cfg: NULL");
    return GP_EINVAL;
  }
  *c = gp_server_cfg{};
  c->hbm_budget_bytes = 16ll << 30;
  c->max_gaussians = 64ll << 20;
  c->max_records = 16ll << 20;
  c->max_instances = 64ll << 20;
  c->max_bins = 64 * 4096;
  c->max_batch = 64;
  c->slots = 3;
  c->attr_dtype = GP_Q16;
  c->use_graphs = 1;
  c->device = 0;
  gp_default_opts(&c->opts);
  return GP_OK;
}

gp_status gp_server_create(gp_server** out, const gp_server_cfg* cfg) {
  if (!out || !cfg) {
    set_error("server_create: NULL");
    return GP_EINVAL;
  }
  *out = nullptr;
  gp_status st = check_opts_pub(&cfg->opts);
  if (st != GP_OK) return st;
  if (cfg->slots < 1 || cfg->slots > 4 || cfg->max_batch < 1 || cfg->max_bins < 1 || cfg->max_gaussians < 64 ||
      cfg->max_records < 1 || cfg->max_instances < 1 || cfg->hbm_budget_bytes < 0 ||
      (cfg->attr_dtype != GP_F32 && cfg->attr_dtype != GP_BF16 && cfg->attr_dtype != GP_F16 &&
       cfg->attr_dtype != GP_Q16 && cfg->attr_dtype != GP_QM)) {
    set_error("server_create: bad configuration");
    return GP_EINVAL;
  }
  GP_HIP(hipSetDevice(cfg->device));
  Server* sv = new (std::nothrow) Server();
  if (!sv) {
    set_error("server_create: host allocation");
    return GP_ENOMEM;
  }
  sv->cfg = *cfg;
  sv->cap_dims = LaunchDims{(cfg->max_gaussians + 63) / 64 * 64 + 64ll * cfg->max_batch, cfg->max_bins};
  {
    const Bucket full{sv->cap_dims.gauss, sv->cap_dims.bins, cfg->max_records, cfg->max_instances};
    const Bucket cand[2] = {{1ll << 21, 16384, 1ll << 21, 1ll << 22}, {1ll << 23, 65536, 1ll << 23, 1ll << 24}};
    for (const Bucket& c : cand) {
      const Bucket b{std::min(c.gauss, full.gauss), std::min(c.bins, full.bins), std::min(c.rec, full.rec),
                     std::min(c.inst, full.inst)};
      const bool smaller = b.gauss < full.gauss || b.bins < full.bins || b.rec < full.rec || b.inst < full.inst;
      const bool grows = sv->buckets.empty() || b.gauss > sv->buckets.back().gauss ||
                         b.bins > sv->buckets.back().bins || b.rec > sv->buckets.back().rec ||
                         b.inst > sv->buckets.back().inst;
      if (smaller && grows) sv->buckets.push_back(b);
    }
    sv->buckets.push_back(full);
  }
  for (int i = 0; i < cfg->slots; ++i) {
    Slot* sl = new (std::nothrow) Slot();
    if (!sl) {
      free_server(sv);
      set_error("server_create: host allocation");
      return GP_ENOMEM;
    }
    sl->sv = sv;
    sv->slots.push_back(sl);
    st = workspace_new(&sl->ws, cfg->max_records, cfg->max_instances);
    if (st == GP_OK) sl->ws->overflow_per_forward = true;
    // descriptor buffers sized for the largest batch so captured graphs stay valid
    if (st == GP_OK) st = reserve_small(sl->ws, cfg->max_batch, cfg->max_batch, cfg->max_bins, sv->cap_dims.gauss);
    // sort scratch for every bucket's key width (fewer bits can mean wider digits)
    for (const Bucket& b : sv->buckets)
      if (st == GP_OK) st = reserve_sort(sl->ws, key_bits(b.bins));
    hipError_t e = st == GP_OK ? hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) : hipSuccess;
    if (st != GP_OK || e != hipSuccess) {
      free_server(sv);
      return st != GP_OK ? st : hip_fail(e, "hipStreamCreate");
    }
  }
  sv->rc = make_render_const(&cfg->opts, cfg->attr_dtype, sv->slots[0]->ws);
  sv->rc.flags |= GP_FLAG_FORWARD_ONLY;   // served slices are never differentiated
  if (cfg->use_graphs) {
    for (Slot* sl : sv->slots) {
      if ((st = capture_slot(sv, sl)) != GP_OK) {
        free_server(sv);
        return st;
      }
    }
  }
  sv->sched = std::thread(scheduler, sv);
  *out = reinterpret_cast<gp_server*>(sv);
  return GP_OK;
}

gp_status gp_server_add_volume(gp_server* s, const gp_gaussians* g, int32_t* volume_id) {
  if (!s || !volume_id) {
    set_error("add_volume: NULL");
    return GP_EINVAL;
  }
  Server* sv = reinterpret_cast<Server*>(s);
  gp_status st = check_gaussians_pub(g);
  if (st != GP_OK) return st;
  if (g->attr_dtype != GP_F32 || g->n < 1) {
    set_error("add_volume: give float32 attributes and n >= 1");
    return GP_EINVAL;
  }
  if ((g->n + 63) / 64 * 64 > sv->cfg.max_gaussians) {
    set_error("add_volume: volume larger than max_gaussians");
    return GP_EINVAL;
  }
  Volume v;
  v.n = g->n;
  v.stride = (g->n + 63) / 64 * 64;
  const bool coded = sv->cfg.attr_dtype == GP_QM;
  v.bytes = coded ? (size_t)v.stride * 11 * sizeof(uint16_t) + 12 * sizeof(float)
                  : (size_t)v.stride * (3 * 4 + 8 * dtype_bytes(sv->cfg.attr_dtype));
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->resident + (int64_t)v.bytes > sv->cfg.hbm_budget_bytes) {
      set_error("add_volume: HBM budget exceeded");
      return GP_ENOMEM;
    }
    sv->resident += (int64_t)v.bytes;   // reserved
  }
  auto release = [&](gp_status code) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->resident -= (int64_t)v.bytes;
    if (v.means) (void)hipFree(v.means);
    if (v.attrs) (void)hipFree(v.attrs);
    return code;
  };
  GP_HIP(hipSetDevice(sv->cfg.device));
  const size_t mean_bytes = coded ? sizeof(uint16_t) * 11 * v.stride : sizeof(float) * 3 * v.stride;
  const size_t attr_bytes = coded ? sizeof(float) * 12 : dtype_bytes(sv->cfg.attr_dtype) * 8 * v.stride;
  if (hipMalloc(reinterpret_cast<void**>(&v.means), mean_bytes) != hipSuccess ||
      hipMalloc(&v.attrs, attr_bytes) != hipSuccess) {
    set_error("add_volume: out of device memory");
    return release(GP_ENOMEM);
  }
  const unsigned blocks = (unsigned)((g->n + 255) / 256);
  const float* m = static_cast<const float*>(g->means);
  const float* a = static_cast<const float*>(g->attrs);
  if (coded) {
    // Morton-ordered codes in the volume's planes, the header in its attribute block
    const gp_status cst = encode_volume(m, a, g->n, g->stride, reinterpret_cast<uint16_t*>(v.means), v.stride,
                                        nullptr, static_cast<float*>(v.attrs), nullptr);
    if (cst != GP_OK) return release(cst);
  } else switch (sv->cfg.attr_dtype) {
    case GP_BF16: k_pack_volume<GP_BF16><<<blocks, 256>>>(m, a, g->stride, g->n, v.means, v.attrs, v.stride); break;
    case GP_F16: k_pack_volume<GP_F16><<<blocks, 256>>>(m, a, g->stride, g->n, v.means, v.attrs, v.stride); break;
    case GP_Q16: k_pack_volume<GP_Q16><<<blocks, 256>>>(m, a, g->stride, g->n, v.means, v.attrs, v.stride); break;
    default: k_pack_volume<GP_F32><<<blocks, 256>>>(m, a, g->stride, g->n, v.means, v.attrs, v.stride); break;
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  // admission statistics from the float32 source: each Gaussian's covariance
  // diagonal (float64), its axial window per tabulated sigma_z as a run of
  // depth bins (difference arrays), and the moments of its footprint width
  std::vector<float> z((size_t)g->n), l((size_t)(7 * g->n));
  if (e == hipSuccess) e = hipMemcpy(z.data(), m + 2 * g->stride, sizeof(float) * g->n, hipMemcpyDeviceToHost);
  for (int r = 0; r < 7 && e == hipSuccess; ++r)
    e = hipMemcpy(l.data() + r * g->n, a + r * g->stride, sizeof(float) * g->n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return release(hip_fail(e, "add_volume"));
  const double q_cut = sv->cfg.opts.q_cut, mod = sv->cfg.opts.scale_mod, kb = sv->cfg.opts.bbox_sigmas;
  std::vector<double> szz((size_t)g->n, -1.0);
  float zl = INFINITY, zh = -INFINITY;
  double m1 = 0.0, m2 = 0.0;
  int64_t nf = 0;
  for (int64_t i = 0; i < g->n; ++i) {
    const double qw = l[3 * g->n + i], qx = l[4 * g->n + i], qy = l[5 * g->n + i], qz = l[6 * g->n + i];
    const double qn = std::sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    double sc[3];
    for (int k = 0; k < 3; ++k) sc[k] = std::exp(std::min<double>(l[k * g->n + i], 80.0)) * mod;
    if (!std::isfinite(z[i]) || !(qn > 0.0) || !std::isfinite(qn)) continue;
    const double w = qw / qn, x = qx / qn, y = qy / qn, zz = qz / qn;
    // rows of R(q); Sigma_aa = sum_k R[a][k]^2 s_k^2
    const double R0[3] = {1 - 2 * (y * y + zz * zz), 2 * (x * y - w * zz), 2 * (x * zz + w * y)};
    const double R1[3] = {2 * (x * y + w * zz), 1 - 2 * (x * x + zz * zz), 2 * (y * zz - w * x)};
    const double R2[3] = {2 * (x * zz - w * y), 2 * (y * zz + w * x), 1 - 2 * (x * x + y * y)};
    double sxx = 0.0, syy = 0.0, sz = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double v2 = sc[k] * sc[k];
      sxx += R0[k] * R0[k] * v2;
      syy += R1[k] * R1[k] * v2;
      sz += R2[k] * R2[k] * v2;
    }
    if (!std::isfinite(sxx + syy + sz)) continue;
    szz[(size_t)i] = sz;
    zl = std::min(zl, z[i]);
    zh = std::max(zh, z[i]);
    const double wf = 2.0 * kb * std::sqrt(std::max(sxx, syy));
    m1 += wf;
    m2 += wf * wf;
    ++nf;
  }
  if (!(zl <= zh)) zl = zh = 0.f;
  const int nb = (int)std::min<double>(1 << 16, std::floor(zh - zl) + 2);
  v.z_lo = std::floor(zl);
  v.nbins = nb;
  v.foot_m1 = nf ? m1 / (double)nf : 0.0;
  v.foot_m2 = nf ? m2 / (double)nf : 0.0;
  v.cover.assign((size_t)kNSigma * nb, 0);
  std::vector<int32_t> diff((size_t)nb + 1);
  for (int k = 0; k < kNSigma; ++k) {
    std::fill(diff.begin(), diff.end(), 0);
    const double s2 = (double)kSigmaGrid[k] * kSigmaGrid[k];
    for (int64_t i = 0; i < g->n; ++i) {
      if (szz[(size_t)i] < 0.0) continue;
      const double h = std::sqrt(q_cut * (s2 + szz[(size_t)i])) * 1.001 + 1e-3;
      // bins b whose depth range [z_lo + b, z_lo + b + 1) meets [mu_z - h, mu_z + h]
      const double lo = (double)z[i] - h - v.z_lo, hi = (double)z[i] + h - v.z_lo;
      const int b0 = (int)std::max(0.0, std::floor(lo)), b1 = (int)std::min<double>(nb - 1, std::floor(hi));
      if (b0 > b1) continue;
      diff[(size_t)b0] += 1;
      diff[(size_t)b1 + 1] -= 1;
    }
    int32_t run = 0;
    for (int b = 0; b < nb; ++b) {
      run += diff[(size_t)b];
      v.cover[(size_t)k * nb + b] = run;
    }
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  *volume_id = (int32_t)sv->vols.size();
  sv->vols.push_back(std::move(v));
  sv->stats.volumes = (int32_t)sv->vols.size();
  sv->stats.resident_bytes = sv->resident;
  return GP_OK;
}

gp_status gp_serve_submit_many(gp_server* s, const gp_request* reqs, float* const* outs, const double* t_arrival,
                               int32_t n, uint64_t* tickets) {
  if (!s || n < 0 || (n > 0 && (!reqs || !outs || !tickets))) {
    set_error("submit: NULL or n < 0");
    return GP_EINVAL;
  }
  Server* sv = reinterpret_cast<Server*>(s);
  for (int32_t i = 0; i < n; ++i) {
    const gp_request* req = reqs + i;
    if (!outs[i]) {
      set_error("submit: NULL output");
      return GP_EINVAL;
    }
    const gp_slice sl{req->z, req->sigma_z, req->x0, req->y0, req->dx, req->dy, req->width, req->height};
    gp_status st = check_slice_pub(sl, 0);
    if (st != GP_OK) return st;
    if (tiles_of(*req) > sv->cfg.max_bins) {
      set_error("submit: request has more tiles than a batch may hold");
      return GP_EINVAL;
    }
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (int32_t i = 0; i < n; ++i) {
      if (reqs[i].volume_id < 0 || reqs[i].volume_id >= (int32_t)sv->vols.size()) {
        set_error("submit: unknown volume");
        return GP_EINVAL;
      }
    }
    if (sv->stop) {
      set_error("submit: server is shutting down");
      return GP_ECANCELED;
    }
    const double now = now_ms();
    for (int32_t i = 0; i < n; ++i) {
      const uint64_t t = sv->next_ticket++;
      sv->tickets.emplace(t, TicketState{});
      sv->queue.push_back(Request{t, reqs[i], outs[i], t_arrival ? t_arrival[i] : now, false});
      tickets[i] = t;
    }
    sv->stats.submitted += n;
  }
  if (n > 0) sv->cv.notify_all();
  return GP_OK;
}

gp_status gp_serve_submit(gp_server* s, const gp_request* req, float* out, uint64_t* ticket) {
  if (!s || !req || !out || !ticket) {
    set_error("submit: NULL");
    return GP_EINVAL;
  }
  float* outs[1] = {out};
  return gp_serve_submit_many(s, req, outs, nullptr, 1, ticket);
}

double gp_clock_ms(void) { return now_ms(); }

gp_status gp_serve_poll(gp_server* s, uint64_t ticket, int32_t timeout_us, gp_serve_result* res) {
  if (!s || !res) {
    set_error("poll: NULL");
    return GP_EINVAL;
  }
  Server* sv = reinterpret_cast<Server*>(s);
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) {
    set_error("poll: unknown ticket");
    return GP_EINVAL;
  }
  auto ready = [&] { return sv->tickets[ticket].done; };
  if (!ready()) {
    if (timeout_us < 0) sv->cv_done.wait(lk, ready);
    else if (timeout_us > 0) sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
  }
  TicketState& t = sv->tickets[ticket];
  if (!t.done) return GP_EAGAIN;
  *res = t.res;
  sv->tickets.erase(ticket);
  return GP_OK;
}

gp_status gp_server_stats_get(gp_server* s, gp_server_stats* st) {
  if (!s || !st) {
    set_error("server_stats: NULL");
    return GP_EINVAL;
  }
  Server* sv = reinterpret_cast<Server*>(s);
  std::lock_guard<std::mutex> lk(sv->mu);
  *st = sv->stats;
  return GP_OK;
}

gp_status gp_server_destroy(gp_server* s) {
  if (!s) return GP_OK;
  Server* sv = reinterpret_cast<Server*>(s);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->sched.joinable()) sv->sched.join();
  free_server(sv);
  return GP_OK;
}

}  // extern "C"
