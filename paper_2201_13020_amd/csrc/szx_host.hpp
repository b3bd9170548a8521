// szx_host.hpp -- host-side pieces of the C ABI shared by the single-call and
// batch entry points (szx_api.hip) and the serving runtime (szx_server.hip).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/szx.h"
#include "szx_launch.hpp"

namespace szx {
namespace host {

// Record the calling thread's error message and return s.
sz_status fail(sz_status s, const std::string& msg);
void clear_error();

// Check parameters and derive the job (sizes, element width, block count).
sz_status make_job(const sz_params* p, Job& j);

// Compute units of the current device (cached), or -1.
int cu_count();

// The timing hook when per-kernel timing is on, else nullptr.
TimerHook current_hook();

// Byte layout of a batch workspace. Map m = 2 * pass + element type;
// compression passes: extrema chunks, classification, encode; decompression
// passes: index, decode.
struct BatchPlan {
  uint64_t fields_off, maps_off[6], zero_off, zero_end, total;
  uint64_t tiles[6];
  int nmaps;
};

// Lay out a batch over the device workspace ws. With `host` non-null, also
// write the image of the workspace's first P.zero_off bytes (descriptors and
// tile maps) into *host and fill *b and *block; the caller copies the image
// to ws before launching. With host == nullptr only P is computed.
sz_status plan_compress(const sz_cfield* fs, uint32_t n, uint8_t* ws, std::vector<uint8_t>* host, BatchPlan& P,
                        CBatch* b, uint32_t* block);
sz_status plan_decompress(const sz_dfield* fs, uint32_t n, uint8_t* ws, std::vector<uint8_t>* host, BatchPlan& P,
                          DBatch* b, uint32_t* block);

// One field's compression (the body of sz_compress): argument checks on the
// buffers, then every pass on `stream`. With nranges > 0 the relative
// bound's range is folded from the nranges pairs (min, max) at d_ranges
// (device doubles) instead of the field's own values.
sz_status compress_single(const Job& j, const void* d_in, void* d_out, uint64_t out_cap, uint64_t* d_out_size,
                          void* d_ws, uint64_t ws_bytes, hipStream_t stream, const double* d_ranges,
                          uint32_t nranges);

// Whether p is 16-byte aligned.
bool aligned16(const void* p);

// Encode geometry of a compression batch from the process-wide table, by the
// size class of each element type's total input bytes.
CLaunchGeom batch_geom(const sz_cfield* fs, uint32_t n, int ncu);

}  // namespace host
}  // namespace szx
