// szx_server.hip -- serving runtime declared in include/szx_server.h.
//
// Threads:
//   scheduler   forms launch groups. While a slot is idle and the queue is
//               not empty, it takes requests from the head in arrival order.
//               It reserves each one's arena bytes (the worst-case stream size
//               for a compression, the values for a decompression into the
//               arena) and stops at the first that does not fit or at
//               max_batch. Then it reserves the group's batch workspaces,
//               giving requests back from the tail while those do not fit.
//               Descriptors go up through the slot's pinned staging; the
//               compression batch, the decompression batch and a copy of the
//               per-request sizes and statuses to pinned memory follow on the
//               slot's stream.
//   completion  one per slot: waits for the slot's event, then turns each
//               compressed stream into an item and shrinks its reservation to
//               the real size. It also records the decompression statuses,
//               frees the workspaces and wakes the scheduler.
// One mutex guards all server state. HIP calls that only enqueue are made
// under it; waiting for the device is not.
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/szx_server.h"
#include "szx_arena.hpp"
#include "szx_host.hpp"

using szx::Arena;
using szx::Job;
using namespace szx::host;

namespace {

struct Request {
  uint64_t id = 0;
  uint32_t kind = 0;
  sz_params p{};
  Job j{};
  const void* in = nullptr;
  void* out = nullptr;  // decompress: caller output, or nullptr for an arena item
  uint64_t out_cap = 0;
  uint64_t item = 0;    // decompress: the item read
  uint64_t t_arrival = 0;
  uint64_t need = 0;    // arena bytes of the request itself
  uint64_t res_off = Arena::kFail;
};

struct Item {
  sz_params p{};
  Job j{};
  uint64_t off = 0, bytes = 0;
  uint32_t readers = 0;
  bool released = false;
  bool values = false;  // decompressed values rather than a stream
};

struct Group {
  std::vector<Request> reqs;  // arrival order; the batches list compressions, then decompressions
  uint32_t ncomp = 0, ndec = 0;
  uint64_t ws_off = Arena::kFail;
  uint64_t t_admit = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t begin = nullptr;  // recorded before the group's first copy
  hipEvent_t done = nullptr;   // after its last copy
  std::thread th;
  std::condition_variable cv;
  std::unique_ptr<Group> g;  // in flight
  uint8_t* stage = nullptr;  // pinned: descriptor images
  uint64_t stage_cap = 0;
  uint8_t* results = nullptr;  // pinned: sizes then statuses
};

}  // namespace

struct sz_server_s {
  sz_server_config cfg{};
  int ncu = 0;
  uint8_t* base = nullptr;  // the arena
  Arena arena;
  std::vector<std::unique_ptr<Slot>> slots;
  std::thread scheduler;
  std::mutex mu;
  std::condition_variable sched_cv, done_cv;
  std::deque<Request> queue;
  std::deque<sz_completion> done_q;
  std::unordered_map<uint64_t, Item> items;
  uint64_t next_req = 1, next_item = 1;
  uint64_t in_flight = 0, peak_in_flight = 0, groups = 0, completed = 0;
  bool stop = false, stop_all = false;
  hipEvent_t ref = nullptr;  // device time origin of the groups' begin/end stamps
  std::chrono::steady_clock::time_point t0;

  uint64_t now() const {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0)
        .count();
  }
};

namespace {

constexpr uint64_t kResultBytes = 12;  // per request: u64 size + u32 status

uint64_t stream_bound(const Job& j) { return szx::sections(j.nblk, j.nblk, j.w, j.b, j.n * j.w).total; }

sz_completion completion_of(const Request& r, uint32_t status) {
  sz_completion c;
  memset(&c, 0, sizeof c);
  c.request = r.id;
  c.kind = r.kind;
  c.status = status;
  c.item = r.kind == SZ_REQ_DECOMPRESS ? r.item : 0;
  c.bytes_in = r.j.n * r.j.w;
  c.t_arrival = r.t_arrival;
  return c;
}

void drop_reader(sz_server_s* S, uint64_t id) {
  auto it = S->items.find(id);
  if (it == S->items.end()) return;
  if (it->second.readers) --it->second.readers;
  if (it->second.released && it->second.readers == 0) {
    S->arena.release(it->second.off);
    S->items.erase(it);
  }
}

// Batch fields of a group, pointing into the arena: the compressions in
// arrival order (result i = stream size, u64 at results_off + 8 i), then the
// decompressions (status, u32 after the sizes).
void group_fields(sz_server_s* S, const Group& g, uint64_t results_off, std::vector<sz_cfield>& cf,
                  std::vector<sz_dfield>& df) {
  cf.clear();
  df.clear();
  for (const Request& r : g.reqs) {
    if (r.kind == SZ_REQ_COMPRESS) {
      sz_cfield f;
      memset(&f, 0, sizeof f);
      f.params = r.p;
      f.d_in = r.in;
      f.d_out = S->base + (r.res_off == Arena::kFail ? 0 : r.res_off);
      f.out_cap = r.need;
      f.d_out_size = (uint64_t*)(S->base + results_off + 8 * cf.size());
      cf.push_back(f);
    }
  }
  for (const Request& r : g.reqs) {
    if (r.kind == SZ_REQ_DECOMPRESS) {
      const Item& it = S->items.at(r.item);
      sz_dfield f;
      memset(&f, 0, sizeof f);
      f.expected = it.p;
      f.d_in = S->base + it.off;
      f.in_bytes = it.bytes;
      f.d_out = r.out ? r.out : (void*)(S->base + (r.res_off == Arena::kFail ? 0 : r.res_off));
      f.out_cap = r.out ? r.out_cap : r.need;
      f.d_status = (uint32_t*)(S->base + results_off + 8 * (uint64_t)g.ncomp + 4 * df.size());
      df.push_back(f);
    }
  }
}

struct GroupSizes {
  uint64_t ws_c, ws_d, results, total;
};

sz_status group_sizes(sz_server_s* S, const Group& g, GroupSizes& z) {
  std::vector<sz_cfield> cf;
  std::vector<sz_dfield> df;
  // sizes depend only on the parameters; any non-null addresses will do
  group_fields(S, g, 0, cf, df);
  BatchPlan P;
  z.ws_c = z.ws_d = 0;
  if (!cf.empty()) {
    const sz_status s = plan_compress(cf.data(), (uint32_t)cf.size(), nullptr, nullptr, P, nullptr, nullptr);
    if (s != SZ_OK) return s;
    z.ws_c = Arena::round(P.total);
  }
  if (!df.empty()) {
    const sz_status s = plan_decompress(df.data(), (uint32_t)df.size(), nullptr, nullptr, P, nullptr, nullptr);
    if (s != SZ_OK) return s;
    z.ws_d = Arena::round(P.total);
  }
  z.results = Arena::round(kResultBytes * g.reqs.size());
  z.total = z.ws_c + z.ws_d + z.results;
  return SZ_OK;
}

// Put the request of g that arrived last back at the head of the queue.
void give_back_last(sz_server_s* S, Group& g) {
  Request r = g.reqs.back();
  g.reqs.pop_back();
  if (r.kind == SZ_REQ_COMPRESS)
    --g.ncomp;
  else
    --g.ndec;
  if (r.res_off != Arena::kFail) S->arena.release(r.res_off);
  r.res_off = Arena::kFail;
  S->queue.push_front(r);
}

bool grow_stage(Slot& sl, uint64_t need) {
  if (sl.stage_cap >= need) return true;
  uint64_t cap = sl.stage_cap ? sl.stage_cap : (1 << 20);
  while (cap < need) cap *= 2;
  if (sl.stage) (void)hipHostFree(sl.stage);  // idle slot: no copy reads it
  sl.stage = nullptr;
  sl.stage_cap = 0;
  if (hipHostMalloc((void**)&sl.stage, cap, hipHostMallocDefault) != hipSuccess) return false;
  sl.stage_cap = cap;
  return true;
}

void fail_group(sz_server_s* S, Group& g, uint32_t status) {
  for (Request& r : g.reqs) {
    if (r.res_off != Arena::kFail) S->arena.release(r.res_off);
    if (r.kind == SZ_REQ_DECOMPRESS) drop_reader(S, r.item);
    S->done_q.push_back(completion_of(r, status));
    ++S->completed;
  }
  if (g.ws_off != Arena::kFail) S->arena.release(g.ws_off);
  S->done_cv.notify_all();
}

// Launch g on slot k. Called with the mutex held.
void launch_group(sz_server_s* S, uint32_t k, std::unique_ptr<Group> g, const GroupSizes& z) {
  Slot& sl = *S->slots[k];
  const uint64_t results_off = g->ws_off + z.ws_c + z.ws_d;
  std::vector<sz_cfield> cf;
  std::vector<sz_dfield> df;
  group_fields(S, *g, results_off, cf, df);
  std::vector<uint8_t> img_c, img_d;
  BatchPlan P;
  szx::CBatch cb;
  szx::DBatch db;
  uint32_t block = S->cfg.block_size;
  sz_status s = SZ_OK;
  if (!cf.empty()) s = plan_compress(cf.data(), (uint32_t)cf.size(), S->base + g->ws_off, &img_c, P, &cb, &block);
  if (s == SZ_OK && !df.empty())
    s = plan_decompress(df.data(), (uint32_t)df.size(), S->base + g->ws_off + z.ws_c, &img_d, P, &db, &block);
  const uint64_t off_d = Arena::round(img_c.size());
  if (s == SZ_OK && !grow_stage(sl, off_d + img_d.size() + 1)) s = SZ_ENOMEM;
  if (s != SZ_OK) {
    fail_group(S, *g, s);
    return;
  }
  hipError_t e = hipEventRecord(sl.begin, sl.stream);
  if (e == hipSuccess && !img_c.empty()) {
    memcpy(sl.stage, img_c.data(), img_c.size());
    e = hipMemcpyAsync(S->base + g->ws_off, sl.stage, img_c.size(), hipMemcpyHostToDevice, sl.stream);
  }
  if (e == hipSuccess && !img_d.empty()) {
    memcpy(sl.stage + off_d, img_d.data(), img_d.size());
    e = hipMemcpyAsync(S->base + g->ws_off + z.ws_c, sl.stage + off_d, img_d.size(), hipMemcpyHostToDevice,
                       sl.stream);
  }
  if (e == hipSuccess && !cf.empty())
    e = szx::launch_compress(cb, block, batch_geom(cf.data(), (uint32_t)cf.size(), S->ncu), sl.stream,
                             current_hook());
  if (e == hipSuccess && !df.empty()) e = szx::launch_decompress(db, block, sl.stream, current_hook());
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.results, S->base + results_off, kResultBytes * g->reqs.size(), hipMemcpyDeviceToHost,
                       sl.stream);
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e != hipSuccess) {
    // nothing usable was enqueued past the failure; wait for what was
    (void)hipStreamSynchronize(sl.stream);
    fail_group(S, *g, SZ_EDEVICE);
    return;
  }
  ++S->in_flight;
  S->peak_in_flight = std::max(S->peak_in_flight, S->in_flight);
  ++S->groups;
  sl.g = std::move(g);
  sl.cv.notify_one();
}

// Form and launch groups on idle slots. Called with the mutex held.
void dispatch(sz_server_s* S) {
  for (uint32_t k = 0; k < S->slots.size() && !S->queue.empty(); ++k) {
    if (S->slots[k]->g) continue;
    auto g = std::make_unique<Group>();
    while (!S->queue.empty() && g->reqs.size() < S->cfg.max_batch) {
      Request& r = S->queue.front();
      if (r.need) {
        r.res_off = S->arena.alloc(r.need);
        if (r.res_off == Arena::kFail) break;  // strict arrival order: later requests wait too
      }
      ++(r.kind == SZ_REQ_COMPRESS ? g->ncomp : g->ndec);
      g->reqs.push_back(r);
      S->queue.pop_front();
    }
    GroupSizes z{};
    while (!g->reqs.empty()) {
      if (group_sizes(S, *g, z) != SZ_OK) break;
      g->ws_off = S->arena.alloc(z.total);
      if (g->ws_off != Arena::kFail) break;
      give_back_last(S, *g);
    }
    if (g->reqs.empty()) return;  // the head waits for memory
    if (g->ws_off == Arena::kFail) {  // planning failed: not reached for requests checked at submission
      fail_group(S, *g, SZ_EINVAL);
      continue;
    }
    g->t_admit = S->now();
    launch_group(S, k, std::move(g), z);
  }
}

// Queue r, or complete it at once with SZ_ENOMEM if even alone, in an empty
// arena, its bytes and its batch workspace could not fit. Mutex held.
void enqueue(sz_server_s* S, Request& r) {
  Group alone;
  alone.reqs.push_back(r);
  ++(r.kind == SZ_REQ_COMPRESS ? alone.ncomp : alone.ndec);
  GroupSizes z{};
  if (group_sizes(S, alone, z) != SZ_OK || Arena::round(r.need) + z.total > S->arena.capacity()) {
    if (r.kind == SZ_REQ_DECOMPRESS) drop_reader(S, r.item);
    S->done_q.push_back(completion_of(r, SZ_ENOMEM));
    ++S->completed;
    S->done_cv.notify_all();
    return;
  }
  S->queue.push_back(r);
  S->sched_cv.notify_all();
}

void scheduler_main(sz_server_s* S) {
  (void)hipSetDevice(S->cfg.device);  // checked at creation; later calls report any failure
  std::unique_lock<std::mutex> lk(S->mu);
  while (!S->stop) {
    dispatch(S);
    S->sched_cv.wait(lk);
  }
}

void completion_main(sz_server_s* S, uint32_t k) {
  (void)hipSetDevice(S->cfg.device);  // as in the scheduler
  Slot& sl = *S->slots[k];
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    sl.cv.wait(lk, [&] { return sl.g != nullptr || S->stop_all; });
    if (!sl.g) return;
    lk.unlock();
    const hipError_t e = hipEventSynchronize(sl.done);
    const uint64_t t_done = S->now();
    // the group's span on the device, from the two events on its stream
    float ms_b = 0.f, ms_e = 0.f;
    const bool stamped = e == hipSuccess && hipEventElapsedTime(&ms_b, S->ref, sl.begin) == hipSuccess &&
                         hipEventElapsedTime(&ms_e, S->ref, sl.done) == hipSuccess;
    lk.lock();
    Group& g = *sl.g;
    const uint64_t* sizes = (const uint64_t*)sl.results;
    const uint32_t* stat = (const uint32_t*)(sl.results + 8 * g.ncomp);
    const uint32_t n = (uint32_t)g.reqs.size();
    uint32_t ci = 0, di = 0;
    for (uint32_t i = 0; i < n; ++i) {
      Request& r = g.reqs[i];
      uint32_t st = e == hipSuccess ? SZ_OK : SZ_EDEVICE;
      sz_completion c = completion_of(r, st);
      if (r.kind == SZ_REQ_COMPRESS) {
        const uint64_t sz = e == hipSuccess ? sizes[ci++] : 0;
        if (sz == 0 || sz > r.need) st = SZ_EDEVICE;
        if (st == SZ_OK) {
          S->arena.shrink(r.res_off, sz);
          Item it;
          it.p = r.p;
          it.j = r.j;
          it.off = r.res_off;
          it.bytes = sz;
          c.item = S->next_item++;
          S->items[c.item] = it;
          c.stream_bytes = sz;
        } else {
          S->arena.release(r.res_off);
        }
      } else {
        const uint32_t ds = stat[di++];
        if (st == SZ_OK && ds != 0) st = ds;
        auto it = S->items.find(r.item);
        c.stream_bytes = it != S->items.end() ? it->second.bytes : 0;
        if (!r.out) {
          if (st == SZ_OK) {
            Item v;
            v.p = r.p;
            v.j = r.j;
            v.off = r.res_off;
            v.bytes = r.need;
            v.values = true;
            c.out_item = S->next_item++;
            S->items[c.out_item] = v;
          } else {
            S->arena.release(r.res_off);
          }
        }
        drop_reader(S, r.item);
      }
      c.status = st;
      c.t_admit = g.t_admit;
      c.t_done = t_done;
      c.t_dev_begin = stamped ? (uint64_t)((double)ms_b * 1e6) : 0;
      c.t_dev_end = stamped ? (uint64_t)((double)ms_e * 1e6) : 0;
      c.group_size = n;
      c.slot = k;
      S->done_q.push_back(c);
      ++S->completed;
    }
    S->arena.release(g.ws_off);
    sl.g.reset();
    --S->in_flight;
    S->sched_cv.notify_all();
    S->done_cv.notify_all();
  }
}

}  // namespace

extern "C" {

sz_status sz_server_create(const sz_server_config* cfg, sz_server* out) {
  clear_error();
  if (!cfg || !out) return fail(SZ_EINVAL, "null pointer");
  if (cfg->slots < 1 || cfg->slots > 16) return fail(SZ_EINVAL, "slots must be in [1, 16]");
  if (cfg->max_batch < 1 || cfg->max_batch > 65536) return fail(SZ_EINVAL, "max_batch must be in [1, 65536]");
  const uint32_t b = cfg->block_size;
  if (b < 8 || b > 1024 || (b & (b - 1))) return fail(SZ_EINVAL, "block_size must be a power of two in [8, 1024]");
  if (cfg->hbm_budget < (1 << 20)) return fail(SZ_EINVAL, "hbm_budget below 1 MiB");
  if (hipSetDevice(cfg->device) != hipSuccess) return fail(SZ_EDEVICE, "bad device");
  auto S = std::make_unique<sz_server_s>();
  S->cfg = *cfg;
  S->t0 = std::chrono::steady_clock::now();
  S->ncu = cu_count();
  if (S->ncu <= 0) return fail(SZ_EDEVICE, "no HIP device");
  const uint64_t bytes = cfg->hbm_budget / Arena::kAlign * Arena::kAlign;
  if (hipMalloc((void**)&S->base, bytes) != hipSuccess) return fail(SZ_ENOMEM, "arena allocation failed");
  S->arena.reset(bytes);
  bool ok = true;
  for (uint32_t k = 0; k < cfg->slots && ok; ++k) {
    auto sl = std::make_unique<Slot>();
    ok = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreate(&sl->begin) == hipSuccess && hipEventCreate(&sl->done) == hipSuccess &&
         hipHostMalloc((void**)&sl->results, kResultBytes * cfg->max_batch + 256, hipHostMallocDefault) ==
             hipSuccess &&
         grow_stage(*sl, 1 << 20);
    S->slots.push_back(std::move(sl));
  }
  // the device time origin of the groups' stamps
  ok = ok && hipEventCreate(&S->ref) == hipSuccess && hipEventRecord(S->ref, S->slots[0]->stream) == hipSuccess &&
       hipEventSynchronize(S->ref) == hipSuccess;
  sz_server_s* raw = S.release();
  if (!ok) {
    sz_server_destroy(raw);
    return fail(SZ_EDEVICE, "stream, event or pinned staging creation failed");
  }
  for (uint32_t k = 0; k < cfg->slots; ++k) raw->slots[k]->th = std::thread(completion_main, raw, k);
  raw->scheduler = std::thread(scheduler_main, raw);
  *out = raw;
  return SZ_OK;
}

void sz_server_destroy(sz_server S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->queue.clear();
    S->sched_cv.notify_all();
  }
  if (S->scheduler.joinable()) S->scheduler.join();
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->done_cv.wait(lk, [&] { return S->in_flight == 0; });
    S->stop_all = true;
    for (auto& sl : S->slots) sl->cv.notify_all();
  }
  for (auto& sl : S->slots)
    if (sl->th.joinable()) sl->th.join();
  // teardown: nothing is left to report a failure to
  (void)hipSetDevice(S->cfg.device);
  for (auto& sl : S->slots) {
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
    if (sl->begin) (void)hipEventDestroy(sl->begin);
    if (sl->done) (void)hipEventDestroy(sl->done);
    if (sl->stage) (void)hipHostFree(sl->stage);
    if (sl->results) (void)hipHostFree(sl->results);
  }
  if (S->ref) (void)hipEventDestroy(S->ref);
  if (S->base) (void)hipFree(S->base);
  delete S;
}

uint64_t sz_server_clock(sz_server S) { return S ? S->now() : 0; }

sz_status sz_server_submit_compress(sz_server S, const sz_params* p, const void* d_in, uint64_t t_arrival,
                                    uint64_t* request) {
  clear_error();
  if (!S || !request) return fail(SZ_EINVAL, "null pointer");
  Request r;
  sz_status s = make_job(p, r.j);
  if (s != SZ_OK) return s;
  if (p->block_size != S->cfg.block_size) return fail(SZ_EINVAL, "block size differs from the server's");
  if ((!d_in && r.j.n) || ((uintptr_t)d_in & 15u)) return fail(SZ_EINVAL, "input must be 16-byte aligned");
  r.kind = SZ_REQ_COMPRESS;
  r.p = *p;
  r.in = d_in;
  r.need = stream_bound(r.j);
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return fail(SZ_EINVAL, "server stopping");
  r.id = S->next_req++;
  r.t_arrival = t_arrival ? t_arrival : S->now();
  *request = r.id;
  enqueue(S, r);
  return SZ_OK;
}

sz_status sz_server_submit_decompress(sz_server S, uint64_t item, void* d_out, uint64_t out_cap, uint64_t t_arrival,
                                      uint64_t* request) {
  clear_error();
  if (!S || !request) return fail(SZ_EINVAL, "null pointer");
  if ((uintptr_t)d_out & 15u) return fail(SZ_EINVAL, "output must be 16-byte aligned");
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return fail(SZ_EINVAL, "server stopping");
  auto it = S->items.find(item);
  if (it == S->items.end() || it->second.released || it->second.values)
    return fail(SZ_EINVAL, "no such resident stream");
  Request r;
  r.kind = SZ_REQ_DECOMPRESS;
  r.p = it->second.p;
  r.j = it->second.j;
  r.item = item;
  r.out = d_out;
  r.out_cap = out_cap;
  if (d_out && out_cap < r.j.n * r.j.w) return fail(SZ_ENOSPC, "output capacity below N * sizeof(T)");
  r.need = d_out ? 0 : r.j.n * r.j.w;
  r.id = S->next_req++;
  r.t_arrival = t_arrival ? t_arrival : S->now();
  ++it->second.readers;
  *request = r.id;
  enqueue(S, r);
  return SZ_OK;
}

uint32_t sz_server_poll(sz_server S, sz_completion* out, uint32_t max, uint32_t wait_us) {
  if (!S || !out || max == 0) return 0;
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->done_q.empty() && wait_us)
    S->done_cv.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return !S->done_q.empty(); });
  uint32_t k = 0;
  while (k < max && !S->done_q.empty()) {
    out[k++] = S->done_q.front();
    S->done_q.pop_front();
  }
  return k;
}

sz_status sz_server_item_info(sz_server S, uint64_t item, sz_params* params, uint64_t* bytes, const void** d_data) {
  clear_error();
  if (!S) return fail(SZ_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->items.find(item);
  if (it == S->items.end() || it->second.released) return fail(SZ_EINVAL, "no such item");
  if (params) *params = it->second.p;
  if (bytes) *bytes = it->second.bytes;
  if (d_data) *d_data = S->base + it->second.off;
  return SZ_OK;
}

sz_status sz_server_copy_item(sz_server S, uint64_t item, void* d_dst, uint64_t cap, hipStream_t stream) {
  clear_error();
  if (!S || !d_dst) return fail(SZ_EINVAL, "null pointer");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->items.find(item);
  if (it == S->items.end() || it->second.released) return fail(SZ_EINVAL, "no such item");
  if (cap < it->second.bytes) return fail(SZ_ENOSPC, "destination smaller than the item");
  if (hipMemcpyAsync(d_dst, S->base + it->second.off, it->second.bytes, hipMemcpyDeviceToDevice, stream) !=
      hipSuccess)
    return fail(SZ_EDEVICE, "copy failed");
  return SZ_OK;
}

sz_status sz_server_release(sz_server S, uint64_t item) {
  clear_error();
  if (!S) return fail(SZ_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->items.find(item);
  if (it == S->items.end() || it->second.released) return fail(SZ_EINVAL, "no such item");
  if (it->second.readers) {
    it->second.released = true;
  } else {
    S->arena.release(it->second.off);
    S->items.erase(it);
  }
  S->sched_cv.notify_all();
  return SZ_OK;
}

sz_status sz_server_get_stats(sz_server S, sz_server_stats* out) {
  clear_error();
  if (!S || !out) return fail(SZ_EINVAL, "null pointer");
  std::lock_guard<std::mutex> lk(S->mu);
  out->arena_bytes = S->arena.capacity();
  out->arena_in_use = S->arena.in_use();
  out->arena_peak = S->arena.peak();
  out->queued = S->queue.size();
  out->in_flight_groups = S->in_flight;
  out->peak_in_flight_groups = S->peak_in_flight;
  out->groups_launched = S->groups;
  out->completed = S->completed;
  out->items_resident = S->items.size();
  return SZ_OK;
}

sz_status sz_server_replay(sz_server S, const sz_trace_req* reqs, uint32_t n, const uint64_t* warm,
                           uint32_t nwarm, uint32_t keep, uint32_t timeout_ms, sz_completion* out,
                           uint64_t* pool_out, uint32_t* npool) {
  clear_error();
  if (!S || (!reqs && n) || (!out && n) || (!warm && nwarm) || keep == 0)
    return fail(SZ_EINVAL, "bad replay arguments");
  std::deque<uint64_t> pool(warm, warm + nwarm);
  std::unordered_map<uint64_t, uint32_t> index;  // request id -> trace position
  std::vector<sz_completion> buf(256);
  uint32_t done = 0;
  auto collect = [&](uint32_t wait_us) {
    const uint32_t k = sz_server_poll(S, buf.data(), (uint32_t)buf.size(), wait_us);
    for (uint32_t i = 0; i < k; ++i) {
      const sz_completion& c = buf[i];
      auto it = index.find(c.request);
      if (it == index.end()) continue;
      out[it->second] = c;
      index.erase(it);
      ++done;
      if (c.status != SZ_OK) continue;
      if (c.kind == SZ_REQ_COMPRESS) {
        pool.push_back(c.item);
        if (pool.size() > keep) {
          sz_server_release(S, pool.front());
          pool.pop_front();
        }
      } else if (c.out_item) {
        sz_server_release(S, c.out_item);
      }
    }
  };
  for (uint32_t i = 0; i < n; ++i) {
    const sz_trace_req& r = reqs[i];
    // wait for the arrival time, collecting completions every 2 us meanwhile
    uint64_t last = 0;
    for (uint64_t now = sz_server_clock(S); now < r.t_arrival; now = sz_server_clock(S)) {
      if (now - last >= 2000) {
        collect(0);
        last = now;
      }
    }
    uint64_t id = 0;
    sz_status st;
    if (r.kind == SZ_REQ_COMPRESS) {
      st = sz_server_submit_compress(S, &r.params, r.d_in, r.t_arrival, &id);
    } else if (pool.empty()) {
      st = SZ_EINVAL;
    } else {
      st = sz_server_submit_decompress(S, pool[r.pick % pool.size()], nullptr, 0, r.t_arrival, &id);
    }
    if (st != SZ_OK) {
      memset(&out[i], 0, sizeof out[i]);
      out[i].kind = r.kind;
      out[i].status = st;
      out[i].t_arrival = r.t_arrival;
      ++done;
      continue;
    }
    index[id] = i;
  }
  const uint64_t t_end = sz_server_clock(S) + (uint64_t)timeout_ms * 1000000ull;
  while (done < n && sz_server_clock(S) < t_end) collect(1000);
  if (npool) {
    *npool = (uint32_t)pool.size();
    if (pool_out)
      for (uint32_t i = 0; i < pool.size(); ++i) pool_out[i] = pool[i];
  }
  if (done < n) return fail(SZ_EDEVICE, "replay timed out");
  return SZ_OK;
}

}  // extern "C"
