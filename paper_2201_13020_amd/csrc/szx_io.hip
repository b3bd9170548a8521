// szx_io.hip -- streams to files and back through pinned, double-buffered
// staging (include/szx_io.h). Host code only.
#include <errno.h>
#include <fcntl.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/szx_io.h"
#include "szx_host.hpp"

namespace {

using szx::host::fail;

// Bytes per staging buffer: large enough that one file call moves a lot,
// small enough that the first copy and the last write (which do not overlap)
// stay short.
constexpr uint64_t kChunk = 16ull << 20;

// The process-wide staging: two pinned buffers and an event for each, made
// on first use; one call holds them at a time.
struct Staging {
  std::mutex mu;
  void* buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ready = false;
};
Staging g_stage;

sz_status stage_ready() {
  if (g_stage.ready) return SZ_OK;
  for (int i = 0; i < 2; ++i) {
    if (hipHostMalloc(&g_stage.buf[i], kChunk, hipHostMallocDefault) != hipSuccess)
      return fail(SZ_EDEVICE, "hipHostMalloc of the file staging failed");
    if (hipEventCreateWithFlags(&g_stage.ev[i], hipEventDisableTiming) != hipSuccess)
      return fail(SZ_EDEVICE, "hipEventCreate for the file staging failed");
  }
  g_stage.ready = true;
  return SZ_OK;
}

std::string sys_error(const char* what, const char* path) {
  return std::string(what) + " " + path + ": " + strerror(errno);
}

// write(2) until all n bytes are out.
bool write_all(int fd, const uint8_t* p, uint64_t n) {
  while (n > 0) {
    const ssize_t w = ::write(fd, p, n > (1ull << 30) ? (1ull << 30) : n);
    if (w < 0) {
      if (errno == EINTR) continue;
      return false;
    }
    p += w;
    n -= (uint64_t)w;
  }
  return true;
}

// read(2) until n bytes are in; false on an error or a short file.
bool read_all(int fd, uint8_t* p, uint64_t n) {
  while (n > 0) {
    const ssize_t r = ::read(fd, p, n > (1ull << 30) ? (1ull << 30) : n);
    if (r < 0) {
      if (errno == EINTR) continue;
      return false;
    }
    if (r == 0) {
      errno = EIO;  // the file shrank while read
      return false;
    }
    p += r;
    n -= (uint64_t)r;
  }
  return true;
}

}  // namespace

extern "C" sz_status sz_file_write(const char* path, const void* src, uint64_t bytes, int durable,
                                   hipStream_t stream) {
  szx::host::clear_error();
  if (!path || (!src && bytes > 0)) return fail(SZ_EINVAL, "sz_file_write: null path or source");
  const int fd = ::open(path, O_WRONLY | O_CREAT | O_TRUNC | O_CLOEXEC, 0644);
  if (fd < 0) return fail(SZ_EIO, sys_error("cannot create", path));
  sz_status st = SZ_OK;
  {
    std::lock_guard<std::mutex> lock(g_stage.mu);
    st = bytes > 0 ? stage_ready() : SZ_OK;
    const uint8_t* s = static_cast<const uint8_t*>(src);
    const uint64_t nchunk = (bytes + kChunk - 1) / kChunk;
    // chunk i is copied into buffer i % 2 while chunk i - 1 is written; the
    // buffer's previous chunk (i - 2) was written in the step before
    for (uint64_t i = 0; st == SZ_OK && i <= nchunk; ++i) {
      if (i < nchunk) {
        const uint64_t off = i * kChunk, len = bytes - off < kChunk ? bytes - off : kChunk;
        if (hipMemcpyAsync(g_stage.buf[i % 2], s + off, len, hipMemcpyDefault, stream) != hipSuccess ||
            hipEventRecord(g_stage.ev[i % 2], stream) != hipSuccess) {
          st = fail(SZ_EDEVICE, "sz_file_write: device-to-host copy failed");
          break;
        }
      }
      if (i > 0) {
        const uint64_t j = i - 1, off = j * kChunk, len = bytes - off < kChunk ? bytes - off : kChunk;
        if (hipEventSynchronize(g_stage.ev[j % 2]) != hipSuccess) {
          st = fail(SZ_EDEVICE, "sz_file_write: device-to-host copy failed");
          break;
        }
        if (!write_all(fd, static_cast<const uint8_t*>(g_stage.buf[j % 2]), len))
          st = fail(SZ_EIO, sys_error("cannot write", path));
      }
    }
    // no copy may still target the staging once the lock is released
    if (st != SZ_OK && g_stage.ready) (void)hipStreamSynchronize(stream);
  }
  if (st == SZ_OK && durable && ::fsync(fd) != 0) st = fail(SZ_EIO, sys_error("cannot flush", path));
  if (::close(fd) != 0 && st == SZ_OK) st = fail(SZ_EIO, sys_error("cannot close", path));
  return st;
}

extern "C" sz_status sz_file_size(const char* path, uint64_t* bytes) {
  szx::host::clear_error();
  if (!path || !bytes) return fail(SZ_EINVAL, "sz_file_size: null argument");
  struct stat sb;
  if (::stat(path, &sb) != 0) return fail(SZ_EIO, sys_error("cannot stat", path));
  if (!S_ISREG(sb.st_mode)) {
    errno = EINVAL;
    return fail(SZ_EIO, sys_error("not a regular file:", path));
  }
  *bytes = (uint64_t)sb.st_size;
  return SZ_OK;
}

extern "C" sz_status sz_file_read(const char* path, void* dst, uint64_t cap, uint64_t* bytes_read,
                                  hipStream_t stream) {
  szx::host::clear_error();
  if (!path || !dst || !bytes_read) return fail(SZ_EINVAL, "sz_file_read: null argument");
  const int fd = ::open(path, O_RDONLY | O_CLOEXEC);
  if (fd < 0) return fail(SZ_EIO, sys_error("cannot open", path));
  struct stat sb;
  if (::fstat(fd, &sb) != 0) {
    const sz_status s = fail(SZ_EIO, sys_error("cannot stat", path));
    ::close(fd);
    return s;
  }
  const uint64_t bytes = (uint64_t)sb.st_size;
  if (bytes > cap) {
    ::close(fd);
    return fail(SZ_ENOSPC, "sz_file_read: the file is larger than the destination");
  }
  sz_status st = SZ_OK;
  {
    std::lock_guard<std::mutex> lock(g_stage.mu);
    st = bytes > 0 ? stage_ready() : SZ_OK;
    uint8_t* d = static_cast<uint8_t*>(dst);
    const uint64_t nchunk = (bytes + kChunk - 1) / kChunk;
    // chunk i is read into buffer i % 2 once that buffer's previous copy
    // (chunk i - 2) has finished, then copied while chunk i + 1 is read
    for (uint64_t i = 0; st == SZ_OK && i < nchunk; ++i) {
      const uint64_t off = i * kChunk, len = bytes - off < kChunk ? bytes - off : kChunk;
      if (i >= 2 && hipEventSynchronize(g_stage.ev[i % 2]) != hipSuccess) {
        st = fail(SZ_EDEVICE, "sz_file_read: host-to-device copy failed");
        break;
      }
      if (!read_all(fd, static_cast<uint8_t*>(g_stage.buf[i % 2]), len)) {
        st = fail(SZ_EIO, sys_error("cannot read", path));
        break;
      }
      if (hipMemcpyAsync(d + off, g_stage.buf[i % 2], len, hipMemcpyDefault, stream) != hipSuccess ||
          hipEventRecord(g_stage.ev[i % 2], stream) != hipSuccess)
        st = fail(SZ_EDEVICE, "sz_file_read: host-to-device copy failed");
    }
    // the staging is free again only once every copy out of it has finished
    if (g_stage.ready && hipStreamSynchronize(stream) != hipSuccess && st == SZ_OK)
      st = fail(SZ_EDEVICE, "sz_file_read: host-to-device copy failed");
  }
  ::close(fd);
  if (st == SZ_OK) *bytes_read = bytes;
  return st;
}
