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

// Device-side counters of a field's compression (256 bytes reserved; the
// extrema pass clears them at the start of every call).
struct Counters {
  uint32_t err;        // nonzero: a bounded wait of the compression gave up
  uint32_t e_ready;    // first-use path: the bound is published in e_bits
  uint32_t reserved[2];
  uint64_t reserved2[2];
  uint64_t n_nc;       // non-constant blocks (raw included)
  uint64_t mid_total;  // mid-byte section size (batches: for the finishing pass)
  uint64_t e_bits;     // bit pattern of the bound e in the element type
};

// The range slots of a field are left all zero by every compression that
// used them (its last classification tile clears them), which then sets the
// field's clean word to kCleanWord. A compression that finds another value
// there (a workspace used for the first time) does not use the slots: its
// extrema workgroups leave one partial range per chunk instead, its first
// classification tile folds them and publishes the bound, and its last one
// clears the slots and sets the word.
constexpr uint64_t kCleanWord = 0x534c4f5453303030ull;  // "000STOLS"

// The decompression's gate: two words of the same first line of a workspace
// (word 0 is the compression's clean word). The epoch word is advanced by
// every decompression's last pass; the go word holds the token of the last
// decompression that cleared its index pass's status words. A call's token is
// its epoch mixed with kGateKey, so it differs from the token the go word
// keeps from the call before, and from the bytes of an unused workspace but
// for a chance of 2^-64.
constexpr uint32_t kGateEpochWord = 8;  // byte 64 of the line
constexpr uint32_t kGateGoWord = 16;    // byte 128
constexpr uint64_t kGateKey = 0x9E3779B97F4A7C15ull;

// Validated parameters of one call.
struct Job {
  uint32_t dtype, eb_mode, ndims, b;
  uint64_t dims[4];
  uint64_t n, nblk;
  double eb;
  uint32_t w;
};

// Input bytes per tile of the encode and of the decode pass (targets; a tile
// is a whole number of rows and at least 8 blocks). A decode tile divides an
// encode tile.
constexpr uint32_t kEncodeTileBytes = 32768;
constexpr uint32_t kDecodeTileBytes = 16384;

// Blocks per tile of the encode (or, with kDecodeTileBytes, the decode) pass
// for block size b and element size w (mirrors Geo in szx_device.hpp).
__host__ __device__ inline uint32_t tile_blocks(uint32_t b, uint32_t w, uint32_t target = kEncodeTileBytes) {
  const uint32_t epl = b >= 512 ? b / 64 : 8;
  const uint32_t lpb = b / epl;
  const uint32_t tb = 256 / lpb;
  uint32_t sub = target / (tb * b * w);
  sub = sub < 1 ? 1 : sub;
  while (tb * sub < 8) sub *= 2;
  return tb * sub;
}

// Blocks per tile of the classification and index passes: at least
// kClsMin (a multiple of 256, the workgroup size) and a multiple of every
// encode tile.
constexpr uint32_t kClsMin = 1024;
__host__ __device__ inline uint32_t cls_blocks(uint32_t b, uint32_t w) {
  const uint32_t t = tile_blocks(b, w);
  return t > kClsMin ? t : kClsMin;
}

// Ticket classes of the persistent encode pass (per element type).
constexpr uint32_t kTicketClasses = 8;
// Tiles of the extrema pass per chunk; a chunk leaves one finite range.
constexpr uint32_t kStatsChunk = 2;

// The extrema pass folds each chunk's finite range into one of a field's
// range slots (chunk c into slot c mod slots), by 64-bit atomic maxima of
// the complemented smallest key and of the largest key, so that a zero slot
// is the identity. Device-scope atomics on one address serialise (tens of
// ns each across XCDs), so the slots sit kRangeStride bytes apart; readers
// fold at most kRangeSlots slots, one per lane of a wave.
constexpr uint32_t kRangeSlots = 64;
constexpr uint32_t kRangeStride = 256;
__host__ __device__ inline uint32_t range_slots(uint64_t chunks) {
  return (uint32_t)(chunks < kRangeSlots ? (chunks ? chunks : 1) : kRangeSlots);
}
// Bytes of a field's clean word (one line) and range slots; the same for
// every field size, so that a workspace reused for another size finds them
// where the last compression left them.
constexpr uint64_t kSlotRegionBytes = 256 + (uint64_t)kRangeSlots * kRangeStride;

// Values per row of a tile for block size b (mirrors Geo::TILE).
__host__ __device__ inline uint64_t row_values(uint32_t b) { return 256ull * (b >= 512 ? b / 64 : 8); }

// Per-field sizes of the passes.
struct FieldTiles {
  uint64_t chunks;  // extrema pass (one workgroup a chunk)
  uint64_t cls;     // classification / decoder index tiles
  uint64_t enc;     // encode tiles
  uint64_t dec;     // decode tiles
};

__host__ __device__ inline FieldTiles field_tiles(uint64_t n, uint64_t nblk, uint32_t w, uint32_t b) {
  FieldTiles t;
  t.chunks = cdiv(cdiv(n, row_values(b)), kStatsChunk);
  t.cls = cdiv(nblk, cls_blocks(b, w));
  t.enc = cdiv(nblk, tile_blocks(b, w));
  t.dec = cdiv(nblk, tile_blocks(b, w, kDecodeTileBytes));
  return t;
}

// Workspace of one field: the clean word with the decompression's gate words
// in its line, and the range slots (at the same offsets for every field
// size), then the region that the compression's extrema pass (and the
// decompression's gate) clears first --
// counters, tickets, scan status words -- then the rest; every piece
// 256-byte aligned.
struct WsLayout {
  uint64_t clean, range, counters, tickets, cls_status, enc_mid, dec_rank, dec_mid, zero_end;
  uint64_t parts, stats, plan, enc_r0, dec_index, total;
};

__host__ __device__ inline WsLayout ws_layout(uint64_t n, uint64_t nblk, uint32_t w, uint32_t b) {
  const FieldTiles ft = field_tiles(n, nblk, w, b);
  WsLayout L;
  L.clean = 0;
  L.range = 256;
  L.counters = kSlotRegionBytes;
  L.tickets = L.counters + 256;
  L.cls_status = align256(L.tickets + 2ull * kTicketClasses * 256);
  L.enc_mid = align256(L.cls_status + (ft.cls + 1) * 8);
  L.dec_rank = align256(L.enc_mid + (ft.enc + 1) * 8);
  L.dec_mid = align256(L.dec_rank + (ft.cls + 1) * 8);
  L.zero_end = align256(L.dec_mid + (ft.cls + 1) * 8);
  L.parts = L.zero_end;
  L.stats = align256(L.parts + ft.chunks * 16);
  L.plan = align256(L.stats + nblk * 2 * (uint64_t)w);
  L.enc_r0 = align256(L.plan + nblk);
  L.dec_index = align256(L.enc_r0 + (ft.enc + 1) * 8);
  L.total = align256(L.dec_index + (ft.dec + 1) * 16);
  return L;
}

}  // namespace szx
