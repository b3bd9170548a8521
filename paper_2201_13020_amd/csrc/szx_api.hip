// szx_api.hip -- host side of the C ABI declared in include/szx.h.
//
// Argument checks, workspace carve-up and kernel launches. No device memory is
// allocated and no call synchronises, except sz_timing_read.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/szx.h"
#include "szx_launch.hpp"

namespace {

thread_local std::string g_err;

sz_status fail(sz_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

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
hipEvent_t g_pending_begin = nullptr;

void timer_hook(const char* name, hipStream_t s, int begin) {
  std::lock_guard<std::mutex> lock(g_tmu);
  if (begin) {
    hipEventCreate(&g_pending_begin);
    hipEventRecord(g_pending_begin, s);
  } else {
    hipEvent_t e;
    hipEventCreate(&e);
    hipEventRecord(e, s);
    g_open.push_back({name, g_pending_begin, e});
    g_pending_begin = nullptr;
  }
}

szx::TimerHook current_hook() {
  std::lock_guard<std::mutex> lock(g_tmu);
  return g_timing ? timer_hook : nullptr;
}

}  // namespace

extern "C" {

uint64_t sz_compress_bound(const sz_params* p) {
  szx::Job j;
  if (make_job(p, j) != SZ_OK) return 0;
  return szx::sections(j.nblk, j.nblk, j.w, j.b, j.n * j.w).total;
}

uint64_t sz_workspace_size(const sz_params* p) {
  szx::Job j;
  if (make_job(p, j) != SZ_OK) return 0;
  return szx::ws_layout(j.nblk, j.w, j.b).total;
}

sz_status sz_compress(const sz_params* p, const void* d_in, void* d_out, uint64_t out_cap,
                      uint64_t* d_out_size, void* d_ws, uint64_t ws_bytes, hipStream_t stream) {
  g_err.clear();
  szx::Job j;
  sz_status s = make_job(p, j);
  if (s != SZ_OK) return s;
  if ((!d_in && j.n) || !d_out || !d_out_size || !d_ws) return fail(SZ_EINVAL, "null buffer");
  if (!aligned16(d_in) || !aligned16(d_out) || !aligned16(d_ws))
    return fail(SZ_EINVAL, "input, output and workspace must be 16-byte aligned");
  if (out_cap < sz_compress_bound(p)) return fail(SZ_ENOSPC, "output capacity below sz_compress_bound");
  if (ws_bytes < sz_workspace_size(p)) return fail(SZ_ENOSPC, "workspace below sz_workspace_size");
  const int ncu = cu_count();
  if (ncu <= 0) return fail(SZ_EDEVICE, "no HIP device");
  szx::CompressLaunch L{d_in, (uint8_t*)d_out, d_out_size, (uint8_t*)d_ws, ncu, stream};
  const hipError_t e = szx::launch_compress(j, L, current_hook());
  if (e != hipSuccess) return fail(SZ_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SZ_OK;
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
  szx::DecompressLaunch L{d_in, in_bytes, d_out, d_status, (uint8_t*)d_ws, ncu, stream};
  const hipError_t e = szx::launch_decompress(j, L, current_hook());
  if (e != hipSuccess) return fail(SZ_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SZ_OK;
}

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
    hipEventSynchronize(t.b);
    float f = 0.f;
    hipEventElapsedTime(&f, t.a, t.b);
    size_t i = 0;
    while (i < nm.size() && strcmp(nm[i], t.name) != 0) ++i;
    if (i == nm.size()) {
      nm.push_back(t.name);
      ms.push_back(0.0);
      cnt.push_back(0);
    }
    ms[i] += f;
    cnt[i] += 1;
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
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
