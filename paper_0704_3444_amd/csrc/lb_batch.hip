// Batches of independent runs (lb_batch_* of the C ABI): a first-fit arena
// for admission by device-memory footprint, the slot table read by the
// persistent kernel (k_batch_d2q9), per-slot step counters owned by the
// device, a captured hipGraph of graph_steps steps, snapshots of the
// counters for the host, and the autotuner over kernel configurations.
//
// Stream discipline.  Stepping, table uploads and counter snapshots run on
// the batch stream in issue order.  Admission (initial state) and
// observables of finished slots run on a second stream.  A slot's memory is
// touched by the batch stream only while its counter is below its target,
// so a finished slot can be read, and its arena range reused, while later
// launches are still queued; a slot removed before it finished is first
// waited for.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "lb.h"
#include "lbm_internal.hpp"

namespace lbm {

__global__ void k_batch_set_counter(long long* t_now, int id, long long v) { t_now[id] = v; }

}  // namespace lbm

namespace {

using lbm::BatchHeader;
using lbm::BatchKernel;
using lbm::BatchSlot;

constexpr int kGroupsPerCu[3] = {2, 4, 8};  // persistent grid options
constexpr int kSnapshots = 4;                // counter snapshots in flight
constexpr int kUploads = 2;                  // table uploads in flight
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size): free ranges keyed by offset, merged
// with their neighbours on release.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, next = it->first + bytes;
      free_.erase(it);
      if (rest) free_[next] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct SlotHost {
  bool live = false;
  lb_ctx* ctx = nullptr;
  size_t off = 0, bytes = 0;
  int64_t t_end = 0;
  int64_t first_snapshot = 0;  // snapshots before this one predate the slot
};

int fail(int code, const std::string& msg) { return lbm::fail_with(code, msg.c_str()); }

#define HIP_TRY(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(LB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

struct lb_batch {
  lb_batch_params bp{};
  hipStream_t stream = nullptr;  // stepping
  bool own_stream = false;
  hipStream_t side = nullptr;    // admission and observables
  char* arena = nullptr;
  Arena alloc;
  std::vector<SlotHost> slots;   // by id
  size_t slot_bytes = 0;         // sizeof(BatchSlot<T>)
  // device tables
  char* d_slots = nullptr;       // BatchSlot<T>[max_slots], table order
  BatchHeader* d_hdr = nullptr;
  long long* d_t = nullptr;      // step counters by slot id
  int* d_item = nullptr;         // work item -> table entry
  int item_cap = 0;
  int nslots_table = 0;          // live entries in the device table
  // pinned staging of table uploads
  char* h_up[kUploads] = {nullptr, nullptr};
  hipEvent_t up_ev[kUploads] = {nullptr, nullptr};
  int up_next = 0;
  size_t up_bytes = 0;
  // kernels
  const BatchKernel* kernels = nullptr;
  int nkernels = 0;
  int config = 0;
  int cus = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // counter snapshots
  long long* h_snap[kSnapshots] = {};
  hipEvent_t snap_ev[kSnapshots] = {};
  int64_t seq = 0;               // snapshots queued so far
  int64_t polled = -1;           // index of the last snapshot lb_batch_poll returned
  std::vector<int64_t> done;     // counters of that snapshot (by id)
  // device scratch of admission and observables
  double* staging = nullptr;
  size_t staging_bytes = 0;
  void* obs = nullptr;
  size_t obs_bytes = 0;
};

namespace {

int ncfg(const lb_batch* b) { return b->nkernels * 3; }
const BatchKernel& kern(const lb_batch* b) { return b->kernels[b->config / 3]; }
int grid_of(const lb_batch* b) {
  const int g = kGroupsPerCu[b->config % 3] * b->cus;
  return (g + 7) / 8 * 8;
}

void launch_step(lb_batch* b) {
  kern(b).step(b->d_slots, b->d_t, b->d_hdr, b->d_item, grid_of(b), b->stream);
  kern(b).advance(b->d_slots, b->d_t, b->d_hdr, b->bp.max_slots, b->stream);
}

// Table entry of one slot in the working precision T.
template <typename T>
void fill_slot(const lb_batch* b, int id, int first_item, int tiles_x, char* dst) {
  BatchSlot<T> e;
  std::memset(&e, 0, sizeof(e));
  const lbm::Ctx& c = b->slots[id].ctx->c;
  e.p = c.params<T>();
  e.f[0] = c.f[0];
  e.f[1] = c.f[1];
  e.t_end = b->slots[id].t_end;
  e.id = id;
  e.first_item = first_item;
  e.tiles_x = tiles_x;
  std::memcpy(dst, &e, sizeof(e));
}

// Rebuild the slot table, the header and the item map for the current
// configuration, and queue their upload on the batch stream.
int upload_table(lb_batch* b) {
  const int k = b->up_next;
  b->up_next = (k + 1) % kUploads;
  HIP_TRY(hipEventSynchronize(b->up_ev[k]));  // the buffer's previous upload is done
  char* h = b->h_up[k];
  char* h_slots = h;
  BatchHeader* h_hdr = reinterpret_cast<BatchHeader*>(h + align_up(size_t(b->bp.max_slots) * b->slot_bytes));
  int* h_item = reinterpret_cast<int*>(reinterpret_cast<char*>(h_hdr) + kAlign);
  const int tx = kern(b).tx, ty = kern(b).ty;
  int n = 0, items = 0;
  for (int id = 0; id < b->bp.max_slots; ++id) {
    const SlotHost& s = b->slots[id];
    if (!s.live) continue;
    const lb_params& p = s.ctx->c.prm;
    const int tiles_x = int((p.nx + tx - 1) / tx), tiles_y = int((p.ny + ty - 1) / ty);
    const int tiles = tiles_x * tiles_y;
    if (items + tiles > b->item_cap) return fail(LB_ENOMEM, "batch work-item table full");
    if (b->bp.storage == LB_F64)
      fill_slot<double>(b, id, items, tiles_x, h_slots + size_t(n) * b->slot_bytes);
    else
      fill_slot<float>(b, id, items, tiles_x, h_slots + size_t(n) * b->slot_bytes);
    for (int j = 0; j < tiles; ++j) h_item[items + j] = n;
    items += tiles;
    ++n;
  }
  h_hdr->nslots = n;
  h_hdr->items = items;
  b->nslots_table = n;
  if (n) HIP_TRY(hipMemcpyAsync(b->d_slots, h_slots, size_t(n) * b->slot_bytes, hipMemcpyHostToDevice, b->stream));
  if (items)
    HIP_TRY(hipMemcpyAsync(b->d_item, h_item, size_t(items) * sizeof(int), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_hdr, h_hdr, sizeof(BatchHeader), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipEventRecord(b->up_ev[k], b->stream));
  return LB_OK;
}

int capture_graph(lb_batch* b) {
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < b->bp.graph_steps; ++k) launch_step(b);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (e != hipSuccess) return fail(LB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  b->graph = g;
  HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return LB_OK;
}

int set_config(lb_batch* b, int config) {
  if (config < 0 || config >= ncfg(b)) return fail(LB_EINVAL, "no such batch configuration");
  b->config = config;
  int rc = upload_table(b);
  if (rc != LB_OK) return rc;
  return capture_graph(b);
}

int queue_snapshot(lb_batch* b) {
  const int k = int(b->seq % kSnapshots);
  HIP_TRY(hipMemcpyAsync(b->h_snap[k], b->d_t, size_t(b->bp.max_slots) * sizeof(long long), hipMemcpyDeviceToHost,
                         b->stream));
  HIP_TRY(hipEventRecord(b->snap_ev[k], b->stream));
  b->seq += 1;
  return LB_OK;
}

// Grow a device scratch buffer (rare: only when a larger run is admitted).
int ensure(void** buf, size_t* have, size_t need, hipStream_t side) {
  if (*have >= need) return LB_OK;
  HIP_TRY(hipStreamSynchronize(side));
  if (*buf) HIP_TRY(hipFree(*buf));
  *buf = nullptr;
  *have = 0;
  HIP_TRY(hipMalloc(buf, need));
  *have = need;
  return LB_OK;
}

// Stored bytes of the nine populations of one site and component.
size_t site_bytes(int storage) { return storage == LB_F64 ? 72 : (storage == LB_F32 ? 36 : 4 + 8 * 2); }

int check_run(const lb_batch* b, const lb_params* p, size_t* bytes) {
  if (!p) return fail(LB_EINVAL, "params is NULL");
  if (p->lattice != LB_D2Q9) return fail(LB_ENOTSUP, "batches take D2Q9 runs");
  if (p->walls != 0) return fail(LB_ENOTSUP, "batches take periodic runs (walls need the split path)");
  if (p->storage != b->bp.storage) return fail(LB_EINVAL, "the run's storage differs from the batch's");
  if (p->n_comp > b->bp.max_comp) return fail(LB_ENOTSUP, "the run has more components than the batch's max_comp");
  const size_t need = lb_workspace_bytes(p);
  if (need == 0) return LB_EINVAL;  // message set by lb_workspace_bytes
  const size_t copy = size_t(p->ny) * size_t((p->nx + 63) / 64) * 64 * size_t(p->n_comp) * site_bytes(p->storage);
  if (copy >= (size_t(1) << 32)) return fail(LB_ENOTSUP, "a batched run's population copy must be below 4 GiB");
  *bytes = need;
  return LB_OK;
}

}  // namespace

extern "C" {

int lb_batch_create(const lb_batch_params* bp, lb_batch** out) {
  if (!out) return fail(LB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!bp) return fail(LB_EINVAL, "params is NULL");
  if (bp->storage != LB_F32 && bp->storage != LB_F64 && bp->storage != LB_F16S)
    return fail(LB_ENOTSUP, "batches take LB_F64, LB_F32 or LB_F16S");
  if (bp->max_comp < 1 || bp->max_comp > 4) return fail(LB_ENOTSUP, "max_comp must be in 1..4");
  if (bp->max_slots < 1 || bp->max_slots > 4096) return fail(LB_EINVAL, "max_slots must be in 1..4096");
  if (bp->graph_steps < 0 || bp->graph_steps > 100000) return fail(LB_EINVAL, "graph_steps must be in 0..100000");
  if (bp->arena_bytes < kAlign) return fail(LB_EINVAL, "arena_bytes too small");
  lb_batch* b = new (std::nothrow) lb_batch;
  if (!b) return fail(LB_ENOMEM, "host allocation failed");
  b->bp = *bp;
  if (b->bp.graph_steps == 0) b->bp.graph_steps = 16;
  b->kernels = lbm::batch_kernels(bp->storage, bp->max_comp, &b->nkernels);
  b->slot_bytes = bp->storage == LB_F64 ? sizeof(BatchSlot<double>) : sizeof(BatchSlot<float>);
  b->slots.assign(bp->max_slots, SlotHost());
  b->done.assign(bp->max_slots, -1);
  auto bail = [&](int rc) {
    lb_batch_free(b);
    return rc;
  };
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return bail(fail(LB_EDEVICE, "no HIP device"));
  b->cus = prop.multiProcessorCount;
  if (bp->stream) {
    b->stream = static_cast<hipStream_t>(bp->stream);
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(LB_EDEVICE, "stream creation failed"));
    b->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(LB_EDEVICE, "stream creation failed"));
  if (hipMalloc(&b->arena, bp->arena_bytes) != hipSuccess)
    return bail(fail(LB_ENOMEM, "arena allocation of " + std::to_string(bp->arena_bytes) + " bytes failed"));
  b->alloc.reset(bp->arena_bytes);
  // work items: at most one per 256 sites of the arena's smallest run, plus
  // the ragged tiles of every slot
  const size_t min_site_bytes = size_t(2) * site_bytes(bp->storage);
  const size_t cap = bp->arena_bytes / (min_site_bytes * 256) * 2 + size_t(bp->max_slots) * 64 + 1024;
  b->item_cap = int(std::min<size_t>(cap, size_t(1) << 28));
  const size_t table = align_up(size_t(bp->max_slots) * b->slot_bytes);
  if (hipMalloc(&b->d_slots, table) != hipSuccess || hipMalloc(&b->d_hdr, kAlign) != hipSuccess ||
      hipMalloc(&b->d_t, size_t(bp->max_slots) * sizeof(long long)) != hipSuccess ||
      hipMalloc(&b->d_item, size_t(b->item_cap) * sizeof(int)) != hipSuccess)
    return bail(fail(LB_ENOMEM, "batch table allocation failed"));
  b->up_bytes = table + kAlign + size_t(b->item_cap) * sizeof(int);
  for (int k = 0; k < kUploads; ++k) {
    if (hipHostMalloc(reinterpret_cast<void**>(&b->h_up[k]), b->up_bytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->up_ev[k], hipEventDisableTiming) != hipSuccess)
      return bail(fail(LB_ENOMEM, "pinned host allocation failed"));
  }
  for (int k = 0; k < kSnapshots; ++k) {
    if (hipHostMalloc(reinterpret_cast<void**>(&b->h_snap[k]), size_t(bp->max_slots) * sizeof(long long),
                      hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->snap_ev[k], hipEventDisableTiming) != hipSuccess)
      return bail(fail(LB_ENOMEM, "pinned host allocation failed"));
  }
  int config = bp->config;
  if (config < 0) config = 1;  // first tile shape, 4 workgroups per CU
  const int rc = set_config(b, config);
  if (rc != LB_OK) return bail(rc);
  *out = b;
  return LB_OK;
}

size_t lb_batch_footprint(const lb_batch* b, const lb_params* p) {
  size_t bytes = 0;
  if (!b || check_run(b, p, &bytes) != LB_OK) return 0;
  return align_up(bytes);
}

int lb_batch_add(lb_batch* b, const lb_params* p, const double* rho0, int64_t nsteps, int32_t* slot) {
  if (!b || !slot) return fail(LB_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  size_t bytes = 0;
  int rc = check_run(b, p, &bytes);
  if (rc != LB_OK) return rc;
  int id = -1;
  for (int k = 0; k < b->bp.max_slots; ++k)
    if (!b->slots[k].live) {
      id = k;
      break;
    }
  if (id < 0) return fail(LB_ENOMEM, "no free slot");
  size_t off = 0;
  if (!b->alloc.alloc(bytes, &off)) return fail(LB_ENOMEM, "no arena range of " + std::to_string(bytes) + " bytes");
  const size_t S = size_t(p->nx) * size_t(p->ny);
  const size_t obs_need = (3 * size_t(p->n_comp) + 2 + 3) * S * sizeof(double);
  rc = ensure(reinterpret_cast<void**>(&b->staging), &b->staging_bytes, size_t(p->n_comp) * S * sizeof(double),
              b->side);
  if (rc == LB_OK) rc = ensure(&b->obs, &b->obs_bytes, obs_need, b->side);
  if (rc != LB_OK) {
    b->alloc.release(off, bytes);
    return rc;
  }
  lb_params q = *p;
  q.stream = b->side;
  q.path = LB_PATH_AUTO;
  q.check_every = 0;
  lb_ctx* ctx = nullptr;
  rc = lbm::init_impl(&q, rho0, b->arena + off, bytes, b->staging, false, &ctx);
  if (rc != LB_OK) {
    b->alloc.release(off, bytes);
    return rc;
  }
  SlotHost& s = b->slots[id];
  s.live = true;
  s.ctx = ctx;
  s.off = off;
  s.bytes = bytes;
  s.t_end = nsteps;
  s.first_snapshot = b->seq;
  b->done[id] = 0;
  lbm::k_batch_set_counter<<<1, 1, 0, b->stream>>>(b->d_t, id, 0);
  rc = upload_table(b);
  if (rc != LB_OK) {
    lb_batch_remove(b, id);
    return rc;
  }
  *slot = id;
  return LB_OK;
}

int lb_batch_step(lb_batch* b, int64_t nsteps) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  const int64_t gs = b->bp.graph_steps;
  for (int64_t k = 0; k < nsteps / gs; ++k) HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  for (int64_t k = 0; k < nsteps % gs; ++k) launch_step(b);
  HIP_TRY(hipGetLastError());
  return queue_snapshot(b);
}

int lb_batch_poll(lb_batch* b, int32_t lag, int64_t* steps_done) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  if (lag < 0 || lag >= kSnapshots) return fail(LB_EINVAL, "lag must be in 0..3");
  const int64_t idx = b->seq - 1 - lag;
  if (idx >= 0) {
    const int k = int(idx % kSnapshots);
    HIP_TRY(hipEventSynchronize(b->snap_ev[k]));
    if (idx > b->polled) {
      for (int id = 0; id < b->bp.max_slots; ++id) {
        const SlotHost& s = b->slots[id];
        if (s.live && idx >= s.first_snapshot) b->done[id] = b->h_snap[k][id];
      }
      b->polled = idx;
    }
  }
  if (steps_done)
    for (int id = 0; id < b->bp.max_slots; ++id) steps_done[id] = b->slots[id].live ? b->done[id] : -1;
  return LB_OK;
}

int lb_batch_moments(lb_batch* b, int32_t slot, double* rho, double* U, double* mu, double* P, double* mass,
                     double* mom, int64_t* step) {
  if (!b || slot < 0 || slot >= b->bp.max_slots || !b->slots[slot].live) return fail(LB_EINVAL, "no such slot");
  SlotHost& s = b->slots[slot];
  if (b->done[slot] != s.t_end) return fail(LB_EINVAL, "the slot has not finished (poll first)");
  lbm::Ctx& c = s.ctx->c;
  c.t = s.t_end;
  c.cur = int(s.t_end & 1);
  return lbm::moments_impl(s.ctx, b->obs, rho, U, mu, P, mass, mom, step);
}

int lb_batch_remove(lb_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->bp.max_slots || !b->slots[slot].live) return fail(LB_EINVAL, "no such slot");
  SlotHost& s = b->slots[slot];
  if (b->done[slot] != s.t_end) {
    // still running: stop it and let the queued launches that step it finish
    s.t_end = 0;
    int rc = upload_table(b);
    if (rc != LB_OK) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream));
  }
  lb_free(s.ctx);
  b->alloc.release(s.off, s.bytes);
  s = SlotHost();
  b->done[slot] = -1;
  return upload_table(b);
}

int lb_batch_config_count(int32_t storage, int32_t max_comp) {
  int n = 0;
  lbm::batch_kernels(storage, max_comp, &n);
  return n ? n * 3 : fail(LB_ENOTSUP, "no batched kernel for this storage / max_comp");
}

int lb_batch_config_info(int32_t storage, int32_t max_comp, int32_t config, int32_t* tile_x, int32_t* tile_y,
                         int32_t* threads, int32_t* groups_per_cu) {
  int n = 0;
  const BatchKernel* k = lbm::batch_kernels(storage, max_comp, &n);
  if (!k) return fail(LB_ENOTSUP, "no batched kernel for this storage / max_comp");
  if (config < 0 || config >= 3 * n) return fail(LB_EINVAL, "no such configuration");
  if (tile_x) *tile_x = k[config / 3].tx;
  if (tile_y) *tile_y = k[config / 3].ty;
  if (threads) *threads = k[config / 3].threads;
  if (groups_per_cu) *groups_per_cu = kGroupsPerCu[config % 3];
  return LB_OK;
}

int lb_batch_set_config(lb_batch* b, int32_t config) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  return set_config(b, config);
}

int lb_batch_tune(lb_batch* b, int32_t steps, double* ms_per_step, int32_t* best) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  if (steps < 1) return fail(LB_EINVAL, "steps must be >= 1");
  if (b->nslots_table == 0) return fail(LB_EINVAL, "the batch has no live slot to time");
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int chosen = -1;
  double best_ms = 0.0;
  int rc = LB_OK;
  for (int c = 0; c < ncfg(b) && rc == LB_OK; ++c) {
    rc = set_config(b, c);
    if (rc != LB_OK) break;
    launch_step(b);  // warm-up
    (void)hipEventRecord(e0, b->stream);
    const int64_t gs = b->bp.graph_steps;
    for (int64_t k = 0; k < steps / gs; ++k) (void)hipGraphLaunch(b->exec, b->stream);
    for (int64_t k = 0; k < steps % gs; ++k) launch_step(b);
    (void)hipEventRecord(e1, b->stream);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      rc = fail(LB_EDEVICE, std::string("autotuner timing: ") + hipGetErrorString(e));
      break;
    }
    const double per = double(ms) / steps;
    if (ms_per_step) ms_per_step[c] = per;
    if (chosen < 0 || per < best_ms) {
      chosen = c;
      best_ms = per;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != LB_OK) return rc;
  rc = set_config(b, chosen);
  if (rc == LB_OK && best) *best = chosen;
  if (rc == LB_OK) rc = queue_snapshot(b);
  return rc;
}

void lb_batch_free(lb_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->side) (void)hipStreamSynchronize(b->side);
  for (SlotHost& s : b->slots)
    if (s.live) lb_free(s.ctx);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (int k = 0; k < kSnapshots; ++k) {
    if (b->h_snap[k]) (void)hipHostFree(b->h_snap[k]);
    if (b->snap_ev[k]) (void)hipEventDestroy(b->snap_ev[k]);
  }
  for (int k = 0; k < kUploads; ++k) {
    if (b->h_up[k]) (void)hipHostFree(b->h_up[k]);
    if (b->up_ev[k]) (void)hipEventDestroy(b->up_ev[k]);
  }
  (void)hipFree(b->d_slots);
  (void)hipFree(b->d_hdr);
  (void)hipFree(b->d_t);
  (void)hipFree(b->d_item);
  (void)hipFree(b->staging);
  (void)hipFree(b->obs);
  (void)hipFree(b->arena);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
