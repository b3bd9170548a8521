// szx_layout.hpp -- stream section offsets, workspace layout and the launch
// job shared by the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace szx {

__host__ __device__ inline uint64_t align16(uint64_t x) { return (x + 15u) & ~(uint64_t)15u; }
__host__ __device__ inline uint64_t align256(uint64_t x) { return (x + 255u) & ~(uint64_t)255u; }
__host__ __device__ inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Byte offsets of the sections of a stream (header at 0).
struct Sections {
  uint64_t state, mu, kbytes, codes, mid, total;
};

__host__ __device__ inline Sections sections(uint64_t nblk, uint64_t n_nc, uint64_t w, uint64_t b,
                                             uint64_t mid_total) {
  Sections s;
  s.state = 96;
  s.mu = align16(s.state + (nblk + 7) / 8);
  s.kbytes = align16(s.mu + nblk * w);
  s.codes = align16(s.kbytes + n_nc);
  s.mid = align16(s.codes + n_nc * (b / 4));
  s.total = s.mid + mid_total;
  return s;
}

// Device-side counters at the start of the workspace (256 bytes reserved).
struct Counters {
  uint32_t err;        // nonzero: a bounded wait of the compression gave up
  uint32_t reserved[3];
  uint64_t klo, khi;   // totalOrder keys of the smallest / largest finite value
  uint64_t n_nc;       // non-constant blocks (raw included)
  uint64_t mid_total;  // mid-byte section size
  uint64_t e_bits;     // bit pattern of the bound e in the element type
};

// Validated parameters of one call.
struct Job {
  uint32_t dtype, eb_mode, ndims, b;
  uint64_t dims[4];
  uint64_t n, nblk;
  double eb;
  uint32_t w;
};

// Blocks per tile of the encode/decode passes for block size b and element
// size w (mirrors Geo in szx_device.hpp).
__host__ __device__ inline uint32_t tile_blocks(uint32_t b, uint32_t w) {
  const uint32_t epl = b >= 512 ? b / 64 : 8;
  const uint32_t lpb = b / epl;
  const uint32_t tb = 256 / lpb;
  uint32_t sub = 32768 / (tb * b * w);
  sub = sub < 1 ? 1 : sub;
  while (tb * sub < 8) sub *= 2;
  return tb * sub;
}

// Blocks per tile of the classification pass: a multiple of every encode
// tile, four blocks per thread at most.
__host__ __device__ inline uint32_t cls_blocks(uint32_t b, uint32_t w) {
  const uint32_t t = tile_blocks(b, w);
  return t > 1024 ? t : 1024;
}

// Most workgroups of the extrema pass; each leaves its finite range here.
constexpr uint32_t kMaxRangeParts = 4096;
// Ticket classes of the persistent encode pass.
constexpr uint32_t kTicketClasses = 8;

// Workspace carve-up; every piece 256-byte aligned.
struct WsLayout {
  uint64_t counters, tickets, range_part, stats, enc_r0, cls_status, enc_mid, dec_index, dec_rank, dec_mid, total;
  uint64_t ntile, ncls;
};

__host__ __device__ inline WsLayout ws_layout(uint64_t nblk, uint32_t w, uint32_t b) {
  WsLayout L;
  L.ntile = cdiv(nblk, tile_blocks(b, w)) + 1;
  L.ncls = cdiv(nblk, cls_blocks(b, w)) + 1;
  L.counters = 0;
  L.tickets = 256;
  L.range_part = align256(L.tickets + (uint64_t)kTicketClasses * 256);
  L.stats = align256(L.range_part + (uint64_t)kMaxRangeParts * 16);
  L.enc_r0 = align256(L.stats + nblk * 2 * (uint64_t)w);
  L.cls_status = align256(L.enc_r0 + L.ntile * 8);
  L.enc_mid = align256(L.cls_status + L.ncls * 8);
  L.dec_index = align256(L.enc_mid + L.ntile * 8);
  L.dec_rank = align256(L.dec_index + L.ntile * 16);
  L.dec_mid = align256(L.dec_rank + L.ncls * 8);
  L.total = align256(L.dec_mid + L.ncls * 8);
  return L;
}

}  // namespace szx
