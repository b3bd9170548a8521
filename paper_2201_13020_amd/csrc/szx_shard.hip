// szx_shard.hip -- a field compressed as contiguous block-range shards, and
// the shard streams stitched into the stream of the whole field.
//
// Blocks are independent (Sec. IV: the field is cut into fixed 1-D blocks),
// so a field splits into shards of whole blocks, one per GPU of a multi-GPU
// run. Only the relative bound couples them: e = eb (max - min) over the
// whole field's finite values (Sec. III, footnote). Each shard reports its
// own finite range (sz_range), the ranges are gathered (on several GPUs, an
// all-gather of 16 bytes per shard), and each shard is compressed with the
// bound of the whole field (sz_compress_shard); every shard stream is a valid
// stream of its own values. sz_stitch then joins the shard streams section by
// section: each section of the whole stream is the concatenation of the
// shards' sections, at offsets from an exclusive scan of their sizes, so the
// result is byte for byte the stream of the whole field. Shards start at a
// multiple of 8 blocks, so that their state bits fill whole bytes.
#include <string.h>

#include <algorithm>
#include <string>

#include "../../include/szx.h"
#include "szx_device.hpp"
#include "szx_host.hpp"

namespace szx {

constexpr uint32_t kRangeChunk = 16384;  // values per workgroup of the range pass
constexpr uint32_t kMaxShards = SZ_MAX_SHARDS;

// Finite range of chunk blockIdx.x (kRangeChunk values) as two totalOrder
// keys (lowest > highest: no finite value).
template <typename T>
__global__ __launch_bounds__(256) void k_range_part(const T* __restrict__ x, uint64_t n, uint64_t* __restrict__ parts) {
  using U = typename Traits<T>::U;
  __shared__ uint64_t s_lo[kWavesPerWG], s_hi[kWavesPerWG];
  const uint64_t i0 = (uint64_t)blockIdx.x * kRangeChunk;
  const uint64_t i1 = std::min<uint64_t>(n, i0 + kRangeChunk);
  U lo = (U)~(U)0, hi = 0;
  for (uint64_t i = i0 + threadIdx.x; i < i1; i += kWG) {
    const U u = bits_of(x[i]);
    const U k = order_key<U>(u);
    const bool fin = is_finite_bits<T>(u);
    lo = (fin && k < lo) ? k : lo;
    hi = (fin && k > hi) ? k : hi;
  }
  uint64_t l64 = lo == (U)~(U)0 ? ~0ull : (uint64_t)lo;
  uint64_t h64 = hi;
  l64 = group_min<kWave, uint64_t>(l64);
  h64 = group_max<kWave, uint64_t>(h64);
  if (lane_id() == 0) {
    s_lo[threadIdx.x / kWave] = l64;
    s_hi[threadIdx.x / kWave] = h64;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWavesPerWG; ++w) {
      l64 = s_lo[w] < l64 ? s_lo[w] : l64;
      h64 = s_hi[w] > h64 ? s_hi[w] : h64;
    }
    *reinterpret_cast<ulonglong2*>(parts + 2 * blockIdx.x) = make_ulonglong2(l64, h64);
  }
}

// The partials folded into (min, max) as doubles; (+inf, -inf) when there is
// no finite value. One workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_range_fold(const uint64_t* __restrict__ parts, uint64_t nparts,
                                                    double* __restrict__ out) {
  using U = typename Traits<T>::U;
  __shared__ uint64_t s_lo[kWavesPerWG], s_hi[kWavesPerWG];
  uint64_t lo = ~0ull, hi = 0;
  for (uint64_t i = threadIdx.x; i < nparts; i += kWG) {
    const ulonglong2 p = reinterpret_cast<const ulonglong2*>(parts)[i];
    lo = p.x < lo ? p.x : lo;
    hi = p.y > hi ? p.y : hi;
  }
  lo = group_min<kWave, uint64_t>(lo);
  hi = group_max<kWave, uint64_t>(hi);
  if (lane_id() == 0) {
    s_lo[threadIdx.x / kWave] = lo;
    s_hi[threadIdx.x / kWave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWavesPerWG; ++w) {
      lo = s_lo[w] < lo ? s_lo[w] : lo;
      hi = s_hi[w] > hi ? s_hi[w] : hi;
    }
    if (lo > hi) {
      out[0] = __builtin_inf();
      out[1] = -__builtin_inf();
    } else {
      out[0] = (double)from_bits<T>(key_to_bits<U>((U)lo));
      out[1] = (double)from_bits<T>(key_to_bits<U>((U)hi));
    }
  }
}

// ------------------------------------------------------------------ stitch --

struct StitchArgs {
  const uint8_t* shard[kMaxShards];
  uint64_t cap[kMaxShards];  // readable bytes of each shard stream's buffer
  uint32_t nshards;
  uint32_t dtype, eb_mode, ndims, b;
  uint64_t dims[4];
  uint64_t n, nblk;
  double eb;
  uint8_t* out;
  uint64_t* out_size;
};

// One piece of the whole stream: len bytes at dst, copied from src (a
// section of a shard stream, 16-byte aligned); src_room bytes are readable
// from src on (to the end of that shard stream).
struct Seg {
  uint64_t dst, len, src_room;
  const uint8_t* src;
};

constexpr int kSections = 5;
constexpr int kMaxSegs = kSections * kMaxShards;

// Byte p of the whole stream outside the header: a byte of the segment that
// holds it, else section padding (zero). `i` is a cursor into the segments
// (sorted by dst, possibly empty ones among them), moved forward as needed.
__device__ __forceinline__ uint8_t stitched_byte(const Seg* segs, int nseg, int& i, uint64_t p) {
  while (i + 1 < nseg && segs[i + 1].dst <= p) ++i;
  const Seg& s = segs[i];
  return (p >= s.dst && p < s.dst + s.len) ? s.src[p - s.dst] : (uint8_t)0;
}

// Joins the shard streams. Every workgroup reads the shard headers, checks
// them against the field and builds the segment table (LDS); then the
// workgroups copy consecutive ranges of 16-byte chunks of the whole stream:
// a chunk inside one segment as one 16-byte store from two aligned 16-byte
// loads of its source, a chunk that touches a segment end byte by byte.
// Workgroup 0 writes the header and the stream size (0 if the shards do not
// make up the field).
__global__ __launch_bounds__(256) void k_stitch(StitchArgs a) {
  __shared__ Seg segs[kMaxSegs];
  __shared__ uint64_t s_hdr[kMaxShards][4];  // nblk, n_nc, mid_total, n
  __shared__ uint64_t s_e[kMaxShards];
  __shared__ uint64_t s_total, s_nnc, s_mid;
  __shared__ int s_ok;
  const uint32_t G = a.nshards;
  const uint32_t w = a.dtype == 0 ? 4 : 8;
  if (threadIdx.x < G) {
    const uint8_t* h = a.shard[threadIdx.x];
    const uint32_t w1 = *reinterpret_cast<const uint32_t*>(h + 4);
    bool good = *reinterpret_cast<const uint32_t*>(h) == kMagic && (w1 & 0xFFu) == kVersion &&
                ((w1 >> 8) & 0xFFu) == a.dtype && *reinterpret_cast<const uint32_t*>(h + 8) == a.b;
    if (good) {  // the whole shard stream lies in its buffer
      const uint64_t nb = *reinterpret_cast<const uint64_t*>(h + 72);
      const uint64_t nnc = *reinterpret_cast<const uint64_t*>(h + 80);
      const uint64_t mid = *reinterpret_cast<const uint64_t*>(h + 88);
      good = nb < (1ull << 40) && nnc <= nb && mid < (1ull << 48) && sections(nb, nnc, w, a.b, mid).total <= a.cap[threadIdx.x];
    }
    s_hdr[threadIdx.x][0] = good ? *reinterpret_cast<const uint64_t*>(h + 72) : ~0ull;  // nblk
    s_hdr[threadIdx.x][1] = *reinterpret_cast<const uint64_t*>(h + 80);               // n_nc
    s_hdr[threadIdx.x][2] = *reinterpret_cast<const uint64_t*>(h + 88);               // mid_total
    s_hdr[threadIdx.x][3] = *reinterpret_cast<const uint64_t*>(h + 48);               // n
    s_e[threadIdx.x] = *reinterpret_cast<const uint64_t*>(h + 64);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bool ok = true;
    uint64_t nblk = 0, n = 0, nnc = 0, mid = 0;
    for (uint32_t i = 0; i < G; ++i) {
      const uint64_t nb_i = s_hdr[i][0];
      ok = ok && nb_i != ~0ull && nb_i <= a.nblk && s_hdr[i][1] <= nb_i && s_e[i] == s_e[0];
      ok = ok && (i + 1 == G || (nb_i % 8) == 0);  // state bits of whole bytes
      if (!ok) break;
      nblk += nb_i;
      n += s_hdr[i][3];
      nnc += s_hdr[i][1];
      mid += s_hdr[i][2];
    }
    ok = ok && nblk == a.nblk && n == a.n;
    const Sections W = sections(a.nblk, nnc, w, a.b, mid);
    if (ok) {
      uint64_t kb = 0, rk = 0, mb = 0;
      for (uint32_t i = 0; i < G; ++i) {
        const uint64_t nb_i = s_hdr[i][0], nnc_i = s_hdr[i][1], mid_i = s_hdr[i][2];
        const Sections S = sections(nb_i, nnc_i, w, a.b, mid_i);
        const uint8_t* base = a.shard[i];
        segs[0 * G + i] = {W.state + kb / 8, cdiv(nb_i, 8), S.total - S.state, base + S.state};
        segs[1 * G + i] = {W.mu + kb * w, nb_i * w, S.total - S.mu, base + S.mu};
        segs[2 * G + i] = {W.kbytes + rk, nnc_i, S.total - S.kbytes, base + S.kbytes};
        segs[3 * G + i] = {W.codes + rk * (a.b / 4), nnc_i * (a.b / 4), S.total - S.codes, base + S.codes};
        segs[4 * G + i] = {W.mid + mb, mid_i, S.total - S.mid, base + S.mid};
        kb += nb_i;
        rk += nnc_i;
        mb += mid_i;
      }
    }
    s_total = W.total;
    s_nnc = nnc;
    s_mid = mid;
    s_ok = ok ? 1 : 0;
  }
  __syncthreads();
  if (!s_ok) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.out_size = 0;
    return;
  }
  const uint64_t total = s_total;
  const int nseg = kSections * (int)G;
  uint8_t* out = a.out;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    uint32_t* o32 = reinterpret_cast<uint32_t*>(out);
    uint64_t* o64 = reinterpret_cast<uint64_t*>(out);
    o32[0] = kMagic;
    o32[1] = (uint32_t)kVersion | (a.dtype << 8) | (a.eb_mode << 16) | (a.ndims << 24);
    o32[2] = a.b;
    o32[3] = 0;
    for (int d = 0; d < 4; ++d) o64[2 + d] = a.dims[d];
    o64[6] = a.n;
    o64[7] = (uint64_t)__double_as_longlong(a.eb);
    o64[8] = s_e[0];
    o64[9] = a.nblk;
    o64[10] = s_nnc;
    o64[11] = s_mid;
    *a.out_size = total;
  }
  // chunks 0-5 are the header
  const uint64_t nchunk = cdiv(total, 16);
  const uint64_t per = cdiv(nchunk > 6 ? nchunk - 6 : 0, (uint64_t)gridDim.x);
  const uint64_t c0 = 6 + (uint64_t)blockIdx.x * per;
  const uint64_t c1 = std::min<uint64_t>(nchunk, c0 + per);
  // the segment of this thread's first chunk
  int cur = 0;
  if (c0 + threadIdx.x < c1) {
    const uint64_t p = (c0 + threadIdx.x) * 16;
    int lo = 0, hi = nseg - 1;  // last segment with dst <= p
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (segs[mid].dst <= p) lo = mid; else hi = mid - 1;
    }
    cur = lo;
  }
  for (uint64_t c = c0 + threadIdx.x; c < c1; c += kWG) {
    const uint64_t p = c * 16;
    while (cur + 1 < nseg && segs[cur + 1].dst <= p) ++cur;
    const Seg s = segs[cur];
    const uint64_t rel = p - s.dst;  // chunk start within the segment (if inside)
    bool done = false;
    if (p >= s.dst && p + 16 <= s.dst + s.len && p + 16 <= total) {
      const uint64_t qa = rel & ~(uint64_t)15;  // the source's 16-byte words (src is 16-byte aligned)
      const uint32_t b = (uint32_t)(rel & 15u);
      if (qa + (b ? 32u : 16u) <= s.src_room) {
        const uint4 q0 = *reinterpret_cast<const uint4*>(s.src + qa);
        uint4 u = q0;
        if (b) {
          const uint4 q1 = *reinterpret_cast<const uint4*>(s.src + qa + 16);
          const uint32_t wv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
          const uint32_t k = b >> 2, sh = b & 3u;
          uint32_t r[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            // words k + j and k + j + 1 of the 32 source bytes (k <= 3)
            uint32_t lo = wv[j], hi = wv[j + 1];
            lo = k == 1 ? wv[j + 1] : k == 2 ? wv[j + 2] : k == 3 ? wv[j + 3] : lo;
            hi = k == 1 ? wv[j + 2] : k == 2 ? wv[j + 3] : k == 3 ? wv[j + 4] : hi;
            r[j] = __builtin_amdgcn_alignbyte(hi, lo, sh);
          }
          u = make_uint4(r[0], r[1], r[2], r[3]);
        }
        *reinterpret_cast<uint4*>(out + p) = u;
        done = true;
      }
    }
    if (!done) {
      int i = cur;
      const uint64_t end = std::min<uint64_t>(p + 16, total);
      for (uint64_t q = p; q < end; ++q) out[q] = stitched_byte(segs, nseg, i, q);
    }
  }
}

}  // namespace szx

using namespace szx;
using namespace szx::host;

namespace {

// The 1-D field of blocks [k0, k1) of the field of job jf.
sz_status shard_job(const sz_params* field, uint64_t k0, uint64_t k1, Job& js, sz_params* ps) {
  Job jf;
  sz_status s = make_job(field, jf);
  if (s != SZ_OK) return s;
  if (!(k0 < k1 && k1 <= jf.nblk)) return fail(SZ_EINVAL, "shard blocks must satisfy k0 < k1 <= the field's blocks");
  if (k0 % 8 != 0 || (k1 != jf.nblk && k1 % 8 != 0))
    return fail(SZ_EINVAL, "shards start and end at multiples of 8 blocks (the last may end at the field's end)");
  const uint64_t n = std::min<uint64_t>(jf.n, k1 * jf.b) - k0 * jf.b;
  sz_params p = *field;
  p.ndims = 1;
  p.dims[0] = n;
  p.dims[1] = p.dims[2] = p.dims[3] = 0;
  s = make_job(&p, js);
  if (s != SZ_OK) return s;
  if (ps) *ps = p;
  return SZ_OK;
}

}  // namespace

extern "C" {

sz_status sz_shard_params(const sz_params* field, uint64_t k0, uint64_t k1, sz_params* out) {
  clear_error();
  if (!out) return fail(SZ_EINVAL, "null pointer");
  Job js;
  return shard_job(field, k0, k1, js, out);
}

sz_status sz_range(const sz_params* p, const void* d_in, double* d_range, void* d_ws, uint64_t ws_bytes,
                   hipStream_t stream) {
  clear_error();
  Job j;
  sz_status s = make_job(p, j);
  if (s != SZ_OK) return s;
  if ((!d_in && j.n) || !d_range || !d_ws) return fail(SZ_EINVAL, "null buffer");
  if (!aligned16(d_ws)) return fail(SZ_EINVAL, "workspace must be 16-byte aligned");
  const WsLayout W = ws_layout(j.n, j.nblk, j.w, j.b);
  if (ws_bytes < W.total) return fail(SZ_ENOSPC, "workspace below sz_workspace_size");
  const uint64_t nparts = cdiv(j.n, kRangeChunk);
  // the room of the compression's per-chunk partials (a chunk holds at most
  // kRangeChunk values)
  uint64_t* parts = reinterpret_cast<uint64_t*>((uint8_t*)d_ws + W.parts);
  if (nparts * 16 > W.stats - W.parts) return fail(SZ_EUNSUPPORTED, "range partials exceed the workspace");
  if (nparts >= (1ull << 31)) return fail(SZ_EUNSUPPORTED, "field too large");
  TimerHook hook = current_hook();
  if (hook) hook("k_range", stream, 1);
  if (nparts) {
    if (j.dtype == SZ_F32)
      k_range_part<float><<<(uint32_t)nparts, 256, 0, stream>>>((const float*)d_in, j.n, parts);
    else
      k_range_part<double><<<(uint32_t)nparts, 256, 0, stream>>>((const double*)d_in, j.n, parts);
  }
  if (j.dtype == SZ_F32)
    k_range_fold<float><<<1, 256, 0, stream>>>(parts, nparts, d_range);
  else
    k_range_fold<double><<<1, 256, 0, stream>>>(parts, nparts, d_range);
  if (hook) hook("k_range", stream, 0);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SZ_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SZ_OK;
}

sz_status sz_compress_shard(const sz_params* field, uint64_t k0, uint64_t k1, const void* d_in,
                            const double* d_ranges, uint32_t nranges, void* d_out, uint64_t out_cap,
                            uint64_t* d_out_size, void* d_ws, uint64_t ws_bytes, hipStream_t stream) {
  clear_error();
  Job js;
  sz_status s = shard_job(field, k0, k1, js, nullptr);
  if (s != SZ_OK) return s;
  if (js.eb_mode == SZ_REL && (nranges == 0 || !d_ranges))
    return fail(SZ_EINVAL, "a relative bound needs the shards' ranges");
  if (nranges > (1u << 20)) return fail(SZ_EUNSUPPORTED, "more than 2^20 ranges");
  return compress_single(js, d_in, d_out, out_cap, d_out_size, d_ws, ws_bytes, stream,
                         js.eb_mode == SZ_REL ? d_ranges : nullptr, js.eb_mode == SZ_REL ? nranges : 0);
}

sz_status sz_stitch(const sz_params* field, uint32_t nshards, const void* const* d_shards,
                    const uint64_t* shard_caps, void* d_out, uint64_t out_cap, uint64_t* d_out_size,
                    hipStream_t stream) {
  clear_error();
  Job j;
  sz_status s = make_job(field, j);
  if (s != SZ_OK) return s;
  if (nshards == 0 || nshards > kMaxShards) return fail(SZ_EINVAL, "shard count outside [1, SZ_MAX_SHARDS]");
  if (!d_shards || !shard_caps || !d_out || !d_out_size) return fail(SZ_EINVAL, "null pointer");
  if (!aligned16(d_out)) return fail(SZ_EINVAL, "output must be 16-byte aligned");
  StitchArgs a;
  memset(&a, 0, sizeof a);
  for (uint32_t i = 0; i < nshards; ++i) {
    if (!d_shards[i]) return fail(SZ_EINVAL, "null shard stream");
    if (!aligned16(d_shards[i])) return fail(SZ_EINVAL, "shard streams must be 16-byte aligned");
    if (shard_caps[i] < 96) return fail(SZ_EINVAL, "a shard buffer shorter than a header");
    a.shard[i] = (const uint8_t*)d_shards[i];
    a.cap[i] = shard_caps[i];
  }
  const uint64_t bound = sections(j.nblk, j.nblk, j.w, j.b, j.n * j.w).total;
  if (out_cap < bound) return fail(SZ_ENOSPC, "output capacity below sz_compress_bound");
  a.nshards = nshards;
  a.dtype = j.dtype;
  a.eb_mode = j.eb_mode;
  a.ndims = j.ndims;
  a.b = j.b;
  for (int d = 0; d < 4; ++d) a.dims[d] = j.dims[d];
  a.n = j.n;
  a.nblk = j.nblk;
  a.eb = j.eb;
  a.out = (uint8_t*)d_out;
  a.out_size = d_out_size;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(4096, cdiv(bound, 16ull * 256 * 8)));
  TimerHook hook = current_hook();
  if (hook) hook("k_stitch", stream, 1);
  k_stitch<<<grid, 256, 0, stream>>>(a);
  if (hook) hook("k_stitch", stream, 0);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SZ_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SZ_OK;
}

}  // extern "C"
