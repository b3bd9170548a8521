// szx_api.hip -- host side of the C ABI declared in include/szx.h.
//
// Argument checks, workspace carve-up and kernel launches. No device memory is
// allocated and no call synchronises, except sz_timing_read.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/szx.h"
#include "szx_host.hpp"

static_assert(SZ_WS_KEPT_BYTES == szx::kSlotRegionBytes, "the header states the bytes a workspace keeps");

namespace szx {
namespace host {

thread_local std::string g_err;

sz_status fail(sz_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

void clear_error() { g_err.clear(); }

bool is_pow2_block(uint32_t b) { return b >= 8 && b <= 1024 && (b & (b - 1)) == 0; }

// Checks the parameters and fills the job. Limits: N < 2^40 values and fewer
// than 2^32 blocks (the list of non-constant blocks holds 32-bit indices).
sz_status make_job(const sz_params* p, szx::Job& j) {
  if (!p) return fail(SZ_EINVAL, "null parameters");
  if (p->dtype > 1) return fail(SZ_EINVAL, "dtype must be SZ_F32 or SZ_F64");
  if (p->eb_mode > 1) return fail(SZ_EINVAL, "eb_mode must be SZ_ABS or SZ_REL");
  if (p->ndims < 1 || p->ndims > 4) return fail(SZ_EINVAL, "ndims must be in [1, 4]");
  if (!is_pow2_block(p->block_size)) return fail(SZ_EINVAL, "block_size must be a power of two in [8, 1024]");
  if (!(p->eb >= 0.0) || !std::isfinite(p->eb)) return fail(SZ_EINVAL, "eb must be finite and >= 0");
  uint64_t n = 1;
  for (uint32_t d = 0; d < 4; ++d) {
    if (d >= p->ndims) {
      if (p->dims[d] != 0) return fail(SZ_EINVAL, "unused dims must be 0");
      continue;
    }
    if (p->dims[d] != 0 && n > ((uint64_t)1 << 62) / p->dims[d]) return fail(SZ_EUNSUPPORTED, "field too large");
    n *= p->dims[d];
  }
  if (n >= ((uint64_t)1 << 40)) return fail(SZ_EUNSUPPORTED, "more than 2^40 values");
  j.dtype = p->dtype;
  j.eb_mode = p->eb_mode;
  j.ndims = p->ndims;
  j.b = p->block_size;
  for (int d = 0; d < 4; ++d) j.dims[d] = p->dims[d];
  j.n = n;
  j.nblk = (n + j.b - 1) / j.b;
  if (j.nblk >= ((uint64_t)1 << 32)) return fail(SZ_EUNSUPPORTED, "2^32 or more blocks");
  j.eb = p->eb;
  j.w = p->dtype == SZ_F32 ? 4 : 8;
  return SZ_OK;
}

int cu_count() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return -1;
    cache[dev] = v;
  }
  return cache[dev];
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// ---- optional per-kernel timing -------------------------------------------
struct TimedLaunch {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimedLaunch> g_open;  // recorded, not yet read
std::vector<std::pair<hipStream_t, hipEvent_t>> g_pending;  // begin events by stream

void timer_hook(const char* name, hipStream_t s, int begin) {
  std::lock_guard<std::mutex> lock(g_tmu);
  // measurement only: a failed event call leaves that launch untimed
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, s);
  if (begin) {
    g_pending.push_back({s, e});
    return;
  }
  for (size_t i = g_pending.size(); i-- > 0;) {
    if (g_pending[i].first != s) continue;
    g_open.push_back({name, g_pending[i].second, e});
    g_pending.erase(g_pending.begin() + i);
    return;
  }
  (void)hipEventDestroy(e);
}

TimerHook current_hook() {
  std::lock_guard<std::mutex> lock(g_tmu);
  return g_timing ? timer_hook : nullptr;
}

// ---- descriptors --------------------------------------------------------

// Descriptor of one compression field whose workspace pieces come from the
// single-field layout at ws.
szx::FieldC single_field_c(const szx::Job& j, const void* in, void* out, uint64_t* out_size, uint8_t* ws) {
  const szx::WsLayout W = szx::ws_layout(j.n, j.nblk, j.w, j.b);
  const szx::FieldTiles ft = szx::field_tiles(j.n, j.nblk, j.w, j.b);
  szx::FieldC f;
  memset(&f, 0, sizeof f);
  f.in = in;
  f.out = (uint8_t*)out;
  f.out_size = out_size;
  f.n = j.n;
  f.nblk = j.nblk;
  f.mu_off = szx::sections(j.nblk, 0, j.w, j.b, 0).mu;
  for (int d = 0; d < 4; ++d) f.dims[d] = j.dims[d];
  f.eb = j.eb;
  f.dtype = j.dtype;
  f.eb_mode = j.eb_mode;
  f.ndims = j.ndims;
  f.b = j.b;
  f.ctr = (szx::Counters*)(ws + W.counters);
  f.clean = (uint64_t*)(ws + W.clean);
  f.range = (uint64_t*)(ws + W.range);
  f.nslots = szx::range_slots(ft.chunks);
  f.parts = (uint64_t*)(ws + W.parts);
  f.stats = ws + W.stats;
  f.plan = ws + W.plan;
  f.enc_r0 = (uint64_t*)(ws + W.enc_r0);
  f.cls_status = (uint64_t*)(ws + W.cls_status);
  f.enc_mid = (uint64_t*)(ws + W.enc_mid);
  return f;
}

szx::FieldD single_field_d(const szx::Job& j, const void* in, uint64_t in_bytes, void* out, uint32_t* status,
                           uint8_t* ws) {
  const szx::WsLayout W = szx::ws_layout(j.n, j.nblk, j.w, j.b);
  szx::FieldD f;
  memset(&f, 0, sizeof f);
  f.in = (const uint8_t*)in;
  f.in_bytes = in_bytes;
  f.out = (uint8_t*)out;
  f.status = status;
  f.index = (uint64_t*)(ws + W.dec_index);
  f.rank_st = (uint64_t*)(ws + W.dec_rank);
  f.mid_st = (uint64_t*)(ws + W.dec_mid);
  f.n = j.n;
  f.nblk = j.nblk;
  f.dtype = j.dtype;
  f.ndims = j.ndims;
  for (int d = 0; d < 4; ++d) f.dims[d] = j.dims[d];
  return f;
}

// Process-wide encode geometry per element type and size class (0: default).
constexpr uint32_t kSizeClasses = 8;
std::atomic<uint32_t> g_geom[2][kSizeClasses];

uint32_t size_class_of(uint64_t bytes) {
  uint32_t c = 0;
  for (uint64_t lim = 256ull << 10; c + 1 < kSizeClasses && bytes >= lim; lim <<= 2) ++c;
  return c;
}

uint32_t encode_wgs_for(uint32_t dtype, uint64_t bytes, int ncu) {
  const uint32_t v = g_geom[dtype][size_class_of(bytes)].load(std::memory_order_relaxed);
  return v ? v : (uint32_t)ncu * 4;
}

CLaunchGeom batch_geom(const sz_cfield* fs, uint32_t n, int ncu) {
  uint64_t bytes[2] = {0, 0};
  for (uint32_t i = 0; i < n; ++i) {
    Job j;
    if (make_job(&fs[i].params, j) == SZ_OK) bytes[j.dtype] += j.n * j.w;
  }
  CLaunchGeom g;
  for (int dt = 0; dt < 2; ++dt) g.encode_wgs[dt] = encode_wgs_for(dt, bytes[dt], ncu);
  return g;
}

}  // namespace host
}  // namespace szx

// Host handle of a planned batch (descriptors already in the workspace).
struct sz_batch_s {
  int decompress;
  uint32_t block;
  szx::CBatch cb;
  szx::DBatch db;
  szx::CLaunchGeom geom;
};

namespace szx {
namespace host {

namespace {
uint64_t a256(uint64_t x) { return align256(x); }
}  // namespace

sz_status check_batch_common(uint32_t n, uint32_t block, const sz_params* p) {
  if (n == 0) return fail(SZ_EINVAL, "empty batch");
  if (p->block_size != block) return fail(SZ_EINVAL, "all fields of a batch share one block size");
  return SZ_OK;
}

sz_status plan_compress(const sz_cfield* fs, uint32_t n, uint8_t* ws, std::vector<uint8_t>* host, BatchPlan& P,
                        CBatch* bout, uint32_t* block_out) {
  if (!fs || n == 0) return fail(SZ_EINVAL, "empty batch");
  std::vector<szx::Job> jobs(n);
  const uint32_t block = fs[0].params.block_size;
  P.nmaps = 6;
  for (int m = 0; m < 6; ++m) P.tiles[m] = 0;
  for (uint32_t i = 0; i < n; ++i) {
    sz_status s = make_job(&fs[i].params, jobs[i]);
    if (s != SZ_OK) return s;
    s = check_batch_common(n, block, &fs[i].params);
    if (s != SZ_OK) return s;
    const szx::FieldTiles ft = szx::field_tiles(jobs[i].n, jobs[i].nblk, jobs[i].w, block);
    const uint32_t dt = jobs[i].dtype;
    P.tiles[0 + dt] += ft.chunks;
    P.tiles[2 + dt] += ft.cls;
    P.tiles[4 + dt] += ft.enc;
  }
  uint64_t off = 256;
  P.fields_off = off;
  off = a256(off + (uint64_t)n * sizeof(szx::FieldC));
  for (int m = 0; m < 6; ++m) {
    P.maps_off[m] = off;
    off = a256(off + P.tiles[m] * 4);
  }
  // clean words and range slots: part of the image written at planning
  // (marked clean), kept clean by every run
  std::vector<uint64_t> slot_off(n);
  for (uint32_t i = 0; i < n; ++i) {
    slot_off[i] = off;
    off = a256(off + szx::kSlotRegionBytes);
  }
  P.zero_off = off;
  off = a256(off + 2ull * szx::kTicketClasses * 256);  // tickets
  std::vector<uint64_t> ctr_off(n), cls_off(n), mid_off(n);
  for (uint32_t i = 0; i < n; ++i) {
    const szx::FieldTiles ft = szx::field_tiles(jobs[i].n, jobs[i].nblk, jobs[i].w, block);
    ctr_off[i] = off;
    off = a256(off + 256);
    cls_off[i] = off;
    off = a256(off + (ft.cls + 1) * 8);
    mid_off[i] = off;
    off = a256(off + (ft.enc + 1) * 8);
  }
  P.zero_end = off;
  std::vector<uint64_t> parts_off(n), stats_off(n), plan_off(n), r0_off(n);
  for (uint32_t i = 0; i < n; ++i) {
    const szx::FieldTiles ft = szx::field_tiles(jobs[i].n, jobs[i].nblk, jobs[i].w, block);
    parts_off[i] = off;
    off = a256(off + ft.chunks * 16);
    stats_off[i] = off;
    off = a256(off + jobs[i].nblk * 2 * (uint64_t)jobs[i].w);
    plan_off[i] = off;
    off = a256(off + jobs[i].nblk);
    r0_off[i] = off;
    off = a256(off + (ft.enc + 1) * 8);
  }
  P.total = off;
  if (!host) return SZ_OK;
  host->assign(P.zero_off, 0);
  szx::FieldC* F = (szx::FieldC*)(host->data() + P.fields_off);
  uint32_t* maps[6];
  for (int m = 0; m < 6; ++m) maps[m] = (uint32_t*)(host->data() + P.maps_off[m]);
  uint64_t bc[2] = {0, 0}, bl[2] = {0, 0}, be[2] = {0, 0};
  uint32_t any_empty = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const szx::Job& j = jobs[i];
    const sz_cfield& c = fs[i];
    if ((!c.d_in && j.n) || !c.d_out || !c.d_out_size) return fail(SZ_EINVAL, "null buffer in batch");
    if (!aligned16(c.d_in) || !aligned16(c.d_out)) return fail(SZ_EINVAL, "batch buffers must be 16-byte aligned");
    if (c.out_cap < szx::sections(j.nblk, j.nblk, j.w, j.b, j.n * j.w).total)
      return fail(SZ_ENOSPC, "a batch output capacity is below sz_compress_bound");
    const szx::FieldTiles ft = szx::field_tiles(j.n, j.nblk, j.w, block);
    szx::FieldC f;
    memset(&f, 0, sizeof f);
    f.in = c.d_in;
    f.out = (uint8_t*)c.d_out;
    f.out_size = c.d_out_size;
    f.n = j.n;
    f.nblk = j.nblk;
    f.mu_off = szx::sections(j.nblk, 0, j.w, j.b, 0).mu;
    for (int d = 0; d < 4; ++d) f.dims[d] = j.dims[d];
    f.eb = j.eb;
    f.dtype = j.dtype;
    f.eb_mode = j.eb_mode;
    f.ndims = j.ndims;
    f.b = j.b;
    f.ctr = (szx::Counters*)(ws + ctr_off[i]);
    f.clean = (uint64_t*)(ws + slot_off[i]);
    f.range = (uint64_t*)(ws + slot_off[i] + 256);
    f.nslots = szx::range_slots(ft.chunks);
    f.parts = (uint64_t*)(ws + parts_off[i]);
    *(uint64_t*)(host->data() + slot_off[i]) = szx::kCleanWord;
    f.stats = ws + stats_off[i];
    f.plan = ws + plan_off[i];
    f.enc_r0 = (uint64_t*)(ws + r0_off[i]);
    f.cls_status = (uint64_t*)(ws + cls_off[i]);
    f.enc_mid = (uint64_t*)(ws + mid_off[i]);
    const uint32_t dt = j.dtype;
    f.base_stats = bc[dt];
    f.base_cls = bl[dt];
    f.base_enc = be[dt];
    F[i] = f;
    for (uint64_t t = 0; t < ft.chunks; ++t) maps[0 + dt][bc[dt] + t] = i;
    for (uint64_t t = 0; t < ft.cls; ++t) maps[2 + dt][bl[dt] + t] = i;
    for (uint64_t t = 0; t < ft.enc; ++t) maps[4 + dt][be[dt] + t] = i;
    bc[dt] += ft.chunks;
    if (j.nblk == 0) any_empty = 1;
    bl[dt] += ft.cls;
    be[dt] += ft.enc;
  }
  szx::CBatch& b = *bout;
  memset(&b, 0, sizeof b);
  b.fields = (const szx::FieldC*)(ws + P.fields_off);
  for (int dt = 0; dt < 2; ++dt) {
    b.field_stats[dt] = (const uint32_t*)(ws + P.maps_off[0 + dt]);
    b.field_cls[dt] = (const uint32_t*)(ws + P.maps_off[2 + dt]);
    b.field_enc[dt] = (const uint32_t*)(ws + P.maps_off[4 + dt]);
    b.tiles_stats[dt] = P.tiles[0 + dt];
    b.tiles_cls[dt] = P.tiles[2 + dt];
    b.tiles_enc[dt] = P.tiles[4 + dt];
  }
  b.tickets = (uint32_t*)(ws + P.zero_off);
  b.zero_begin = (uint64_t*)(ws + P.zero_off);
  b.zero_words = (P.zero_end - P.zero_off) / 8;
  b.nfields = n;
  b.any_empty = any_empty;
  *block_out = block;
  return SZ_OK;
}

sz_status plan_decompress(const sz_dfield* fs, uint32_t n, uint8_t* ws, std::vector<uint8_t>* host, BatchPlan& P,
                          DBatch* bout, uint32_t* block_out) {
  if (!fs || n == 0) return fail(SZ_EINVAL, "empty batch");
  std::vector<szx::Job> jobs(n);
  const uint32_t block = fs[0].expected.block_size;
  P.nmaps = 4;
  for (int m = 0; m < 6; ++m) P.tiles[m] = 0;
  for (uint32_t i = 0; i < n; ++i) {
    sz_status s = make_job(&fs[i].expected, jobs[i]);
    if (s != SZ_OK) return s;
    s = check_batch_common(n, block, &fs[i].expected);
    if (s != SZ_OK) return s;
    const szx::FieldTiles ft = szx::field_tiles(jobs[i].n, jobs[i].nblk, jobs[i].w, block);
    P.tiles[0 + jobs[i].dtype] += ft.cls;
    P.tiles[2 + jobs[i].dtype] += ft.dec;
  }
  uint64_t off = 256;  // line 0: the gate's epoch and go words
  P.fields_off = off;
  off = a256(off + (uint64_t)n * sizeof(szx::FieldD));
  for (int m = 0; m < 4; ++m) {
    P.maps_off[m] = off;
    off = a256(off + P.tiles[m] * 4);
  }
  P.zero_off = off;
  std::vector<uint64_t> rank_off(n), mid_off(n), index_off(n);
  for (uint32_t i = 0; i < n; ++i) {
    const szx::FieldTiles ft = szx::field_tiles(jobs[i].n, jobs[i].nblk, jobs[i].w, block);
    rank_off[i] = off;
    off = a256(off + (ft.cls + 1) * 8);
    mid_off[i] = off;
    off = a256(off + (ft.cls + 1) * 8);
  }
  P.zero_end = off;
  for (uint32_t i = 0; i < n; ++i) {
    const szx::FieldTiles ft = szx::field_tiles(jobs[i].n, jobs[i].nblk, jobs[i].w, block);
    index_off[i] = off;
    off = a256(off + (ft.dec + 1) * 16);
  }
  P.total = off;
  if (!host) return SZ_OK;
  host->assign(P.zero_off, 0);
  szx::FieldD* F = (szx::FieldD*)(host->data() + P.fields_off);
  uint32_t* maps[4];
  for (int m = 0; m < 4; ++m) maps[m] = (uint32_t*)(host->data() + P.maps_off[m]);
  uint64_t bi[2] = {0, 0}, bd[2] = {0, 0};
  for (uint32_t i = 0; i < n; ++i) {
    const szx::Job& j = jobs[i];
    const sz_dfield& d = fs[i];
    if (!d.d_in || (!d.d_out && j.n) || !d.d_status) return fail(SZ_EINVAL, "null buffer in batch");
    if (!aligned16(d.d_in) || !aligned16(d.d_out)) return fail(SZ_EINVAL, "batch buffers must be 16-byte aligned");
    if (d.out_cap < j.n * j.w) return fail(SZ_ENOSPC, "a batch output capacity is below N * sizeof(T)");
    const szx::FieldTiles ft = szx::field_tiles(j.n, j.nblk, j.w, block);
    szx::FieldD f;
    memset(&f, 0, sizeof f);
    f.in = (const uint8_t*)d.d_in;
    f.in_bytes = d.in_bytes;
    f.out = (uint8_t*)d.d_out;
    f.status = d.d_status;
    f.index = (uint64_t*)(ws + index_off[i]);
    f.rank_st = (uint64_t*)(ws + rank_off[i]);
    f.mid_st = (uint64_t*)(ws + mid_off[i]);
    f.n = j.n;
    f.nblk = j.nblk;
    f.dtype = j.dtype;
    f.ndims = j.ndims;
    for (int k = 0; k < 4; ++k) f.dims[k] = j.dims[k];
    const uint32_t dt = j.dtype;
    f.base_idx = bi[dt];
    f.base_dec = bd[dt];
    F[i] = f;
    for (uint64_t t = 0; t < ft.cls; ++t) maps[0 + dt][bi[dt] + t] = i;
    for (uint64_t t = 0; t < ft.dec; ++t) maps[2 + dt][bd[dt] + t] = i;
    bi[dt] += ft.cls;
    bd[dt] += ft.dec;
  }
  szx::DBatch& b = *bout;
  memset(&b, 0, sizeof b);
  b.fields = (const szx::FieldD*)(ws + P.fields_off);
  for (int dt = 0; dt < 2; ++dt) {
    b.field_idx[dt] = (const uint32_t*)(ws + P.maps_off[0 + dt]);
    b.field_dec[dt] = (const uint32_t*)(ws + P.maps_off[2 + dt]);
    b.tiles_idx[dt] = P.tiles[0 + dt];
    b.tiles_dec[dt] = P.tiles[2 + dt];
  }
  b.zero_begin = (uint64_t*)(ws + P.zero_off);
  b.zero_words = (P.zero_end - P.zero_off) / 8;
  b.gate = (uint64_t*)ws;  // the first line (zero in the image: the first run clears)
  b.nfields = n;
  *block_out = block;
  return SZ_OK;
}

}  // namespace host
}  // namespace szx

using namespace szx::host;

extern "C" {

uint64_t sz_compress_bound(const sz_params* p) {
  szx::Job j;
  if (make_job(p, j) != SZ_OK) return 0;
  return szx::sections(j.nblk, j.nblk, j.w, j.b, j.n * j.w).total;
}

uint64_t sz_workspace_size(const sz_params* p) {
  szx::Job j;
  if (make_job(p, j) != SZ_OK) return 0;
  return szx::ws_layout(j.n, j.nblk, j.w, j.b).total;
}

sz_status sz_compress(const sz_params* p, const void* d_in, void* d_out, uint64_t out_cap,
                      uint64_t* d_out_size, void* d_ws, uint64_t ws_bytes, hipStream_t stream) {
  g_err.clear();
  szx::Job j;
  sz_status s = make_job(p, j);
  if (s != SZ_OK) return s;
  return compress_single(j, d_in, d_out, out_cap, d_out_size, d_ws, ws_bytes, stream, nullptr, 0);
}

}  // extern "C"

namespace szx {
namespace host {

sz_status compress_single(const Job& j, const void* d_in, void* d_out, uint64_t out_cap, uint64_t* d_out_size,
                          void* d_ws, uint64_t ws_bytes, hipStream_t stream, const double* d_ranges,
                          uint32_t nranges) {
  if ((!d_in && j.n) || !d_out || !d_out_size || !d_ws) return fail(SZ_EINVAL, "null buffer");
  if (!aligned16(d_in) || !aligned16(d_out) || !aligned16(d_ws))
    return fail(SZ_EINVAL, "input, output and workspace must be 16-byte aligned");
  if (out_cap < szx::sections(j.nblk, j.nblk, j.w, j.b, j.n * j.w).total)
    return fail(SZ_ENOSPC, "output capacity below sz_compress_bound");
  if (ws_bytes < szx::ws_layout(j.n, j.nblk, j.w, j.b).total)
    return fail(SZ_ENOSPC, "workspace below sz_workspace_size");
  const int ncu = cu_count();
  if (ncu <= 0) return fail(SZ_EDEVICE, "no HIP device");
  uint8_t* ws = (uint8_t*)d_ws;
  const szx::WsLayout W = szx::ws_layout(j.n, j.nblk, j.w, j.b);
  const szx::FieldTiles ft = szx::field_tiles(j.n, j.nblk, j.w, j.b);
  szx::CBatch b;
  memset(&b, 0, sizeof b);
  b.one = single_field_c(j, d_in, d_out, d_out_size, ws);
  b.one.ext_range = d_ranges;
  b.one.next_range = nranges;
  b.tiles_stats[j.dtype] = ft.chunks;
  b.tiles_cls[j.dtype] = ft.cls;
  b.tiles_enc[j.dtype] = ft.enc;
  b.tickets = (uint32_t*)(ws + W.tickets);
  b.zero_begin = (uint64_t*)(ws + W.counters);
  b.zero_words = (W.dec_rank - W.counters) / 8;
  b.nfields = 1;
  b.any_empty = j.nblk == 0;
  szx::CLaunchGeom g;
  g.encode_wgs[0] = g.encode_wgs[1] = encode_wgs_for(j.dtype, j.n * j.w, ncu);
  const hipError_t e = szx::launch_compress(b, j.b, g, stream, current_hook());
  if (e != hipSuccess) return fail(SZ_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SZ_OK;
}

}  // namespace host
}  // namespace szx

// ---- allocation-free compression ------------------------------------------
// The workspace of sz_compress_noalloc: one array per GPU, held from the
// library's load on that device until the process ends. Host code never uses
// this name as an address: its device address comes from hipGetSymbolAddress,
// once per device, and is kept in g_scratch_ptr.
static __device__ __align__(256) uint8_t scratch[SZ_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (null: not yet looked up)

// Device address of the current device's scratch array, looked up on the
// first call on that device. Returns SZ_OK and sets *out, or an error.
sz_status scratch_of_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(SZ_EDEVICE, std::string("hipGetDevice failed: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(SZ_EUNSUPPORTED, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SZ_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SZ_OK;
}
}  // namespace

extern "C" {

sz_status sz_compress_noalloc(const sz_params* p, const void* d_in, void* d_out, uint64_t out_cap,
                              uint64_t* d_out_size, hipStream_t stream) {
  g_err.clear();
  szx::Job j;
  sz_status s = make_job(p, j);
  if (s != SZ_OK) return s;
  // the size limit is decided on the host, before any device call
  const uint64_t need = szx::ws_layout(j.n, j.nblk, j.w, j.b).total;
  if (need > SZ_NOALLOC_SCRATCH_BYTES)
    return fail(SZ_EUNSUPPORTED, "field needs " + std::to_string(need) +
                                     " bytes of scratch, above the " + std::to_string(SZ_NOALLOC_SCRATCH_BYTES) +
                                     " bytes of sz_compress_noalloc (use sz_compress with a workspace)");
  void* ptr = nullptr;
  s = scratch_of_current_device(&ptr);
  if (s != SZ_OK) return s;
  // the same kernels as sz_compress; their first pass clears the workspace
  // words that must start at zero (counters, tickets, scan status words)
  return sz_compress(p, d_in, d_out, out_cap, d_out_size, ptr, SZ_NOALLOC_SCRATCH_BYTES, stream);
}

sz_status sz_decompress(const void* d_in, uint64_t in_bytes, const sz_params* expected, void* d_out,
                        uint64_t out_cap, uint32_t* d_status, void* d_ws, uint64_t ws_bytes,
                        hipStream_t stream) {
  g_err.clear();
  szx::Job j;
  sz_status s = make_job(expected, j);
  if (s != SZ_OK) return s;
  if (!d_in || (!d_out && j.n) || !d_status || !d_ws) return fail(SZ_EINVAL, "null buffer");
  if (!aligned16(d_in) || !aligned16(d_out) || !aligned16(d_ws))
    return fail(SZ_EINVAL, "input, output and workspace must be 16-byte aligned");
  if (out_cap < j.n * j.w) return fail(SZ_ENOSPC, "output capacity below N * sizeof(T)");
  if (ws_bytes < sz_workspace_size(expected)) return fail(SZ_ENOSPC, "workspace below sz_workspace_size");
  const int ncu = cu_count();
  if (ncu <= 0) return fail(SZ_EDEVICE, "no HIP device");
  uint8_t* ws = (uint8_t*)d_ws;
  const szx::WsLayout W = szx::ws_layout(j.n, j.nblk, j.w, j.b);
  const szx::FieldTiles ft = szx::field_tiles(j.n, j.nblk, j.w, j.b);
  szx::DBatch b;
  memset(&b, 0, sizeof b);
  b.one = single_field_d(j, d_in, in_bytes, d_out, d_status, ws);
  b.tiles_idx[j.dtype] = ft.cls;
  b.tiles_dec[j.dtype] = ft.dec;
  b.zero_begin = (uint64_t*)(ws + W.dec_rank);
  b.zero_words = (W.zero_end - W.dec_rank) / 8;
  b.gate = (uint64_t*)(ws + W.clean);
  b.nfields = 1;
  const hipError_t e = szx::launch_decompress(b, j.b, stream, current_hook());
  if (e != hipSuccess) return fail(SZ_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SZ_OK;
}

uint64_t sz_batch_workspace_size(const sz_cfield* cf, const sz_dfield* df, uint32_t n) {
  BatchPlan P;
  if ((cf != nullptr) == (df != nullptr)) return 0;
  const sz_status s = cf ? plan_compress(cf, n, nullptr, nullptr, P, nullptr, nullptr)
                         : plan_decompress(df, n, nullptr, nullptr, P, nullptr, nullptr);
  return s == SZ_OK ? P.total : 0;
}

static sz_status batch_create(const sz_cfield* cf, const sz_dfield* df, uint32_t n, void* d_ws, uint64_t ws_bytes,
                              sz_batch* out) {
  g_err.clear();
  if (!out || !d_ws) return fail(SZ_EINVAL, "null pointer");
  if (!aligned16(d_ws)) return fail(SZ_EINVAL, "workspace must be 16-byte aligned");
  const int ncu = cu_count();
  if (ncu <= 0) return fail(SZ_EDEVICE, "no HIP device");
  sz_batch_s* hb = new sz_batch_s;
  memset(hb, 0, sizeof *hb);
  hb->decompress = df != nullptr;
  BatchPlan P;
  std::vector<uint8_t> host;
  sz_status s = cf ? plan_compress(cf, n, (uint8_t*)d_ws, &host, P, &hb->cb, &hb->block)
                   : plan_decompress(df, n, (uint8_t*)d_ws, &host, P, &hb->db, &hb->block);
  if (s == SZ_OK && ws_bytes < P.total) s = fail(SZ_ENOSPC, "workspace below sz_batch_workspace_size");
  if (s == SZ_OK) {
    // descriptors and tile maps, once; run() launches kernels only
    const hipError_t e = hipMemcpy(d_ws, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) s = fail(SZ_EDEVICE, std::string("descriptor upload failed: ") + hipGetErrorString(e));
  }
  if (s != SZ_OK) {
    delete hb;
    return s;
  }
  if (cf) hb->geom = batch_geom(cf, n, ncu);
  *out = hb;
  return SZ_OK;
}

sz_status sz_batch_create_compress(const sz_cfield* fields, uint32_t n, void* d_ws, uint64_t ws_bytes, sz_batch* out) {
  return batch_create(fields, nullptr, n, d_ws, ws_bytes, out);
}

sz_status sz_batch_create_decompress(const sz_dfield* fields, uint32_t n, void* d_ws, uint64_t ws_bytes,
                                     sz_batch* out) {
  return batch_create(nullptr, fields, n, d_ws, ws_bytes, out);
}

sz_status sz_batch_set_geometry(sz_batch b, sz_dtype dtype, uint32_t encode_wgs) {
  g_err.clear();
  if (!b || b->decompress || encode_wgs == 0 || (dtype != SZ_F32 && dtype != SZ_F64))
    return fail(SZ_EINVAL, "bad batch or geometry");
  b->geom.encode_wgs[dtype] = encode_wgs;
  return SZ_OK;
}

uint32_t sz_size_class(uint64_t bytes) { return size_class_of(bytes); }

sz_status sz_set_geometry(sz_dtype dtype, uint32_t size_class, uint32_t encode_wgs) {
  g_err.clear();
  if ((dtype != SZ_F32 && dtype != SZ_F64) || size_class >= kSizeClasses)
    return fail(SZ_EINVAL, "bad element type or size class");
  g_geom[dtype][size_class].store(encode_wgs, std::memory_order_relaxed);
  return SZ_OK;
}

sz_status sz_batch_run(sz_batch b, hipStream_t stream) {
  g_err.clear();
  if (!b) return fail(SZ_EINVAL, "null batch");
  const hipError_t e = b->decompress ? szx::launch_decompress(b->db, b->block, stream, current_hook())
                                     : szx::launch_compress(b->cb, b->block, b->geom, stream, current_hook());
  if (e != hipSuccess) return fail(SZ_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SZ_OK;
}

void sz_batch_destroy(sz_batch b) { delete b; }

sz_status sz_inspect(const void* h_hdr, uint64_t bytes, sz_params* out, uint64_t* total_bytes) {
  g_err.clear();
  if (!h_hdr || !out) return fail(SZ_EINVAL, "null pointer");
  if (bytes < 96) return fail(SZ_ECORRUPT, "shorter than the 96-byte header");
  const uint8_t* h = (const uint8_t*)h_hdr;
  uint32_t magic, b, res;
  memcpy(&magic, h, 4);
  memcpy(&b, h + 8, 4);
  memcpy(&res, h + 12, 4);
  if (magic != 0x4D585A53u || h[4] != 1) return fail(SZ_ECORRUPT, "bad magic or version");
  sz_params p;
  memset(&p, 0, sizeof p);
  p.dtype = h[5];
  p.eb_mode = h[6];
  p.ndims = h[7];
  p.block_size = b;
  memcpy(p.dims, h + 16, 32);
  memcpy(&p.eb, h + 56, 8);
  szx::Job j;
  if (make_job(&p, j) != SZ_OK) return fail(SZ_ECORRUPT, "header parameters invalid");
  uint64_t n, nblk, n_nc, mid_total;
  memcpy(&n, h + 48, 8);
  memcpy(&nblk, h + 72, 8);
  memcpy(&n_nc, h + 80, 8);
  memcpy(&mid_total, h + 88, 8);
  if (n != j.n || nblk != j.nblk || n_nc > nblk || mid_total > j.n * j.w)
    return fail(SZ_ECORRUPT, "header sizes inconsistent");
  *out = p;
  if (total_bytes) *total_bytes = szx::sections(nblk, n_nc, j.w, j.b, mid_total).total;
  return SZ_OK;
}

const char* sz_last_error(void) { return g_err.c_str(); }

void sz_timing_enable(int on) {
  std::lock_guard<std::mutex> lock(g_tmu);
  g_timing = on != 0;
}

uint32_t sz_timing_read(const char** names, double* total_ms, uint32_t* launches, uint32_t cap) {
  std::vector<TimedLaunch> open;
  {
    std::lock_guard<std::mutex> lock(g_tmu);
    open.swap(g_open);
  }
  std::vector<const char*> nm;
  std::vector<double> ms;
  std::vector<uint32_t> cnt;
  for (auto& t : open) {
    (void)hipEventSynchronize(t.b);
    float f = 0.f;
    (void)hipEventElapsedTime(&f, t.a, t.b);
    size_t i = 0;
    while (i < nm.size() && strcmp(nm[i], t.name) != 0) ++i;
    if (i == nm.size()) {
      nm.push_back(t.name);
      ms.push_back(0.0);
      cnt.push_back(0);
    }
    ms[i] += f;
    cnt[i] += 1;
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  uint32_t m = (uint32_t)std::min<size_t>(cap, nm.size());
  for (uint32_t i = 0; i < m; ++i) {
    if (names) names[i] = nm[i];
    if (total_ms) total_ms[i] = ms[i];
    if (launches) launches[i] = cnt[i];
  }
  return m;
}

}  // extern "C"
