// szx_launch.hpp -- what the host API passes to the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "szx_layout.hpp"

namespace szx {

struct CompressLaunch {
  const void* in;
  uint8_t* out;
  uint64_t* out_size;
  uint8_t* ws;
  int n_cu;
  hipStream_t stream;
};

struct DecompressLaunch {
  const void* in;
  uint64_t in_bytes;
  void* out;
  uint32_t* status;
  uint8_t* ws;
  int n_cu;
  hipStream_t stream;
};

// Called around every kernel launch when timing is enabled (begin = 1 before,
// 0 after).
using TimerHook = void (*)(const char* name, hipStream_t s, int begin);

hipError_t launch_compress(const Job& j, const CompressLaunch& L, TimerHook hook);
hipError_t launch_decompress(const Job& j, const DecompressLaunch& L, TimerHook hook);

}  // namespace szx
