// szx_launch.hpp -- what the host API hands to the kernels: one descriptor per
// field, and a batch of descriptors with maps from each pass's global tile
// numbering to the field. A single call is a batch of one field passed by
// value (fields == nullptr), so single and batched calls run the same code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "szx_layout.hpp"

namespace szx {

// One field of a compression.
struct FieldC {
  const void* in;
  uint8_t* out;
  uint64_t* out_size;
  uint64_t n, nblk, mu_off;
  uint64_t dims[4];
  double eb;
  uint32_t dtype, eb_mode, ndims, b;
  uint32_t nslots;
  uint32_t next_range;  // > 0: the relative bound's range comes from ext_range (shards of a larger field)
  const double* ext_range;  // next_range pairs (min, max) of finite values, as doubles
  Counters* ctr;
  uint64_t* clean;      // the clean word (kCleanWord: the range slots are all zero)
  uint64_t* range;      // range slots: slot i at range + i * kRangeStride / 8 (lo_inv, hi)
  uint64_t* parts;      // first use only: per chunk, lowest and highest totalOrder key of its finite values
  void* stats;          // two totalOrder keys per block
  uint8_t* plan;        // one plan byte per block (classification -> encode)
  uint64_t* enc_r0;     // first rank of every encode tile
  uint64_t* cls_status; // scan status words, classification tiles
  uint64_t* enc_mid;    // scan status words, encode tiles
  uint64_t base_stats, base_cls, base_enc;  // first chunk / tile of the field in its type's numbering
};

struct CBatch {
  const FieldC* fields;          // device array, or nullptr: the single field `one`
  // Per element type (0: float32, 1: float64) each pass numbers the tiles of
  // that type's fields consecutively; the maps take such a number to its
  // field (nullptr: field 0). Each pass runs one kernel per element type
  // present, so no kernel carries the registers of both.
  const uint32_t* field_stats[2];  // extrema chunk -> field
  const uint32_t* field_cls[2];    // classification tile -> field
  const uint32_t* field_enc[2];    // encode tile -> field
  uint64_t tiles_stats[2];
  uint64_t tiles_cls[2];
  uint64_t tiles_enc[2];
  uint32_t* tickets;             // 2 * kTicketClasses counters, 256 bytes apart
  uint64_t* zero_begin;          // words the extrema pass clears (counters, tickets, status words)
  uint64_t zero_words;
  uint32_t nfields;
  uint32_t any_empty;            // some field has no values (its header needs a pass of its own)
  FieldC one;
};

// Launch geometry (no effect on the output bytes).
struct CLaunchGeom {
  uint32_t encode_wgs[2];  // persistent workgroups of the encode pass, per element type
};

// One field of a decompression.
struct FieldD {
  const uint8_t* in;
  uint64_t in_bytes;
  uint8_t* out;
  uint32_t* status;
  uint64_t* index;    // per decode tile: first rank, first mid byte
  uint64_t* rank_st;  // scan status words of the index pass
  uint64_t* mid_st;
  uint64_t n, nblk;
  uint32_t dtype, ndims;
  uint64_t dims[4];
  uint64_t base_idx, base_dec;  // first index / decode tile of the field in its type's numbering
};

struct DBatch {
  const FieldD* fields;
  const uint32_t* field_idx[2];  // index tile -> field, per element type as in CBatch
  const uint32_t* field_dec[2];  // decode tile -> field
  uint64_t tiles_idx[2], tiles_dec[2];
  uint64_t* zero_begin;  // the index pass's status words (its gate clears them)
  uint64_t zero_words;
  uint64_t* gate;        // the workspace line of the gate's epoch and go words
  uint32_t nfields, pad;
  FieldD one;
};

// Called around every kernel launch when timing is enabled (begin = 1 before,
// 0 after).
using TimerHook = void (*)(const char* name, hipStream_t s, int begin);

hipError_t launch_compress(const CBatch& b, uint32_t block, const CLaunchGeom& g, hipStream_t stream,
                           TimerHook hook);
hipError_t launch_decompress(const DBatch& b, uint32_t block, hipStream_t stream, TimerHook hook);

}  // namespace szx
