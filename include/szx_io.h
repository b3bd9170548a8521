/* szx_io.h -- dumping compressed streams to files and loading them back.
 *
 * The single-node counterpart of the paper's data dumping and loading study
 * (Sec. VI, the dumping/loading breakdown on thetaGPU): a compressed stream
 * (or any buffer) goes from device memory to a file and back. Device-to-host
 * and host-to-device copies run through two pinned staging buffers on the
 * caller's stream, each chunk's copy overlapping the file write or read of
 * the chunk before it. The stream format is unchanged: a loaded stream
 * decompresses as it was written.
 *
 * These calls block the calling thread until the data is in the file (or in
 * the destination buffer). They allocate their pinned staging on first use
 * and keep it (a process-wide cache, one call at a time holds it); they are
 * not for the allocation-free compression path. The staging's events belong
 * to the device current at the first call, so `stream` must be a stream of
 * that device (or the null stream). Errors set sz_last_error().
 */
#ifndef SZX_IO_H
#define SZX_IO_H

#include <stdint.h>

#include "szx.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Write bytes [0, bytes) of src (device or host memory) to the file at path,
   created or truncated, once the work queued on `stream` before the call has
   finished. With durable != 0 the file is flushed to its storage (fsync)
   before returning. bytes == 0 creates an empty file.
   Errors: SZ_EINVAL (null path, or null src with bytes > 0), SZ_EIO (open,
   write, fsync or close failed: the file may be partial), SZ_EDEVICE (a copy
   or the staging allocation failed). */
sz_status sz_file_write(const char* path, const void* src, uint64_t bytes, int durable, hipStream_t stream);

/* Size in bytes of the file at path. Errors: SZ_EINVAL, SZ_EIO. */
sz_status sz_file_size(const char* path, uint64_t* bytes);

/* Read the whole file at path into dst (device or host memory, cap bytes);
   the copies are ordered after the work queued on `stream` and complete when
   the call returns. *bytes_read receives the file size.
   Errors: SZ_EINVAL (null path, dst or bytes_read), SZ_ENOSPC (file larger
   than cap; nothing copied), SZ_EIO (open or read failed, or the file changed
   size while read), SZ_EDEVICE. */
sz_status sz_file_read(const char* path, void* dst, uint64_t cap, uint64_t* bytes_read, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SZX_IO_H */
