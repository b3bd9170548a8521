/*
 * szx.h -- C ABI of the MI355X (gfx950) implementation of the SZx block-wise
 * error-bounded lossy compressor (Yu et al., "SZx: an Ultra-fast Error-bounded
 * Lossy Compressor for Scientific Datasets", arXiv 2201.13020).
 *
 * The method (Sec. IV, Alg. 1): the flattened field is cut into fixed 1-D
 * blocks of b values. A block whose values all lie within e of mu, the mean of
 * the block's min and max, is stored as mu alone ("constant" block). Every
 * other block stores mu, the count K of leading IEEE-754 bits kept of each
 * normalised value v = x - mu (eq. (4)), right-shifted so the kept bits fill
 * whole bytes (eq. (5), Sec. V-A), and, per value, a 2-bit code of the leading
 * bytes it shares with its predecessor plus the remaining ("mid") bytes.
 * Decompression inverts this (Sec. V-B). Every reconstructed value x' obeys
 * |x - x'| <= e (eq. (1)).
 *
 * All device pointers are plain HIP device addresses; every buffer is owned
 * by the caller. Calls that take a stream are asynchronous on that stream:
 * they validate arguments on the host, enqueue kernels, and return. They never
 * allocate device memory and never synchronise, so they may be captured in a
 * HIP graph. Results that only the device knows (the compressed size, decode
 * errors) are written to device memory.
 *
 * Stream layout (format version 1; little-endian):
 *   96-byte header: magic "SZXM", version, dtype, eb_mode, ndims, b, dims[4],
 *   N, eb as given, bit pattern of e, nblk, n_nc (non-constant blocks),
 *   mid_total; then five sections, each starting at a multiple of 16 bytes:
 *   state bits (1 = non-constant, LSB-first), mu[nblk] (T), K[n_nc] (u8,
 *   0xFF = raw block), codes[n_nc * b/4] (4 per byte, first value in the top
 *   two bits), mid bytes[mid_total] (values in order, kept bytes most
 *   significant first; raw blocks hold the values' little-endian bytes).
 */
#ifndef SZX_H
#define SZX_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element type of the field. */
typedef enum { SZ_F32 = 0, SZ_F64 = 1 } sz_dtype;

/* SZ_ABS: e = eb. SZ_REL: e = eb * (max - min) over the field's finite values,
   the value-range based relative bound of Sec. III (footnote) and Sec. VI.
   In both modes e is then rounded down to the element type. */
typedef enum { SZ_ABS = 0, SZ_REL = 1 } sz_eb_mode;

typedef enum {
  SZ_OK = 0,
  SZ_EINVAL = 1,       /* bad argument (null pointer, bad parameter, misaligned buffer) */
  SZ_ENOSPC = 2,       /* output or workspace capacity too small */
  SZ_ECORRUPT = 3,     /* stream failed validation (sz_inspect, or *d_status) */
  SZ_EDEVICE = 4,      /* a HIP call failed; see sz_last_error() */
  SZ_ENOMEM = 5,       /* reserved */
  SZ_EUNSUPPORTED = 6, /* parameters beyond this build's limits */
  SZ_EIO = 7           /* a file operation failed (szx_io.h); see sz_last_error() */
} sz_status;

/* Parameters of one field. Dims are metadata: blocks run over the row-major
   flattening (Sec. IV splits the data into short one-dimensional blocks),
   N = dims[0]*...*dims[ndims-1]. */
typedef struct {
  uint32_t dtype;      /* sz_dtype */
  uint32_t ndims;      /* 1..4 */
  uint64_t dims[4];    /* unused entries must be 0 */
  uint32_t eb_mode;    /* sz_eb_mode */
  uint32_t block_size; /* b: a power of two in [8, 1024]; the paper's choice is 128 (Sec. V-A) */
  double eb;           /* >= 0 and finite */
} sz_params;

/* Upper bound of the compressed size in bytes for these parameters (every
   block stored raw, plus header and section padding). 0 if the parameters are
   invalid. Host only, pure. */
uint64_t sz_compress_bound(const sz_params* p);

/* Device workspace in bytes that sz_compress and sz_decompress need for these
   parameters (per-block extrema, the list of non-constant blocks, tile status
   words of the single-pass scans, counters). 0 if the parameters are invalid.
   Host only, pure. A workspace may hold any bytes before its first use.
   Between compressions its first SZ_WS_KEPT_BYTES bytes carry state from one
   call to the next (the global range pass's slots, left zero, and a word
   that marks them so, at the same offsets for every field size); a
   compression that does not find that mark takes a slower path that does
   not trust the slots, and leaves the mark for the next call. Do not write
   into those bytes between calls (overwriting the whole workspace, its first
   bytes included, is fine). sz_decompress keeps two words of its own there
   (bytes 64-71 and 128-135: a call counter and the token of the last call
   that cleared its scan status words; every call clears them, in its first
   kernel) and touches nothing else of them. */
#define SZ_WS_KEPT_BYTES 16640
uint64_t sz_workspace_size(const sz_params* p);

/* Compress N values of p->dtype at d_in (device, 16-byte aligned) into d_out
   (device, 16-byte aligned, out_cap bytes, out_cap >= sz_compress_bound(p)).
   Writes the stream size (bytes) to *d_out_size (device u64); 0 there means a
   device-side failure. d_ws: device workspace of ws_bytes >= sz_workspace_size(p),
   16-byte aligned. Asynchronous on `stream`.
   Errors (returned, nothing enqueued): SZ_EINVAL, SZ_ENOSPC, SZ_EUNSUPPORTED,
   SZ_EDEVICE (launch failure). Implements Alg. 1 of Sec. IV with the GPU
   organisation of Sec. V-B (per-block classification, then encoding of the
   non-constant blocks with a prefix scan for their output offsets). */
sz_status sz_compress(const sz_params* p, const void* d_in, void* d_out,
                      uint64_t out_cap, uint64_t* d_out_size, void* d_ws,
                      uint64_t ws_bytes, hipStream_t stream);

/* Decompress the stream at d_in (device, 16-byte aligned, in_bytes bytes) into
   d_out (device, 16-byte aligned, out_cap >= N * sizeof(T) bytes). `expected`
   gives the field's dtype, dims and block size (from sz_inspect on a host copy
   of the header, or from the caller's own metadata); the kernels check the
   device header against it. *d_status (device u32) receives SZ_OK,
   SZ_ECORRUPT (the stream failed validation) or SZ_EDEVICE (a bounded wait
   between workgroups gave up); otherwise the output is unspecified but no
   access leaves the given buffers. d_ws as for sz_compress, sized with `expected`.
   Asynchronous on `stream`. Sec. V-B: leading bytes are resolved by a parallel
   scan over the 2-bit codes, mid bytes are located by a prefix scan. */
sz_status sz_decompress(const void* d_in, uint64_t in_bytes,
                        const sz_params* expected, void* d_out, uint64_t out_cap,
                        uint32_t* d_status, void* d_ws, uint64_t ws_bytes,
                        hipStream_t stream);

/* ---- allocation-free compression ------------------------------------------
   For callers that cannot allocate device memory at all (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc) and cannot
   provide a workspace either. Same arguments, kernels and output bytes as
   sz_compress, without d_ws: the workspace is a static device array of
   SZ_NOALLOC_SCRATCH_BYTES bytes inside the library, one per GPU, held from
   the library's load on that device until the process ends. Its device
   address is looked up on the first call on each device (with that device
   current); no call allocates or frees device memory.
   Limit: fields whose sz_workspace_size exceeds SZ_NOALLOC_SCRATCH_BYTES are
   rejected with SZ_EUNSUPPORTED before any device call (at b = 128 that is
   above about 1.75 GB of float32 or 1.85 GB of float64 values).
   Every call on one GPU shares that GPU's array: calls that overlap on the
   same GPU (on different streams, or from different threads) race and
   corrupt each other's output; serialise them, e.g. on one stream. The
   kernels clear what must start at zero at the start of every call. */
#define SZ_NOALLOC_SCRATCH_BYTES (32ull << 20)
sz_status sz_compress_noalloc(const sz_params* p, const void* d_in, void* d_out,
                              uint64_t out_cap, uint64_t* d_out_size,
                              hipStream_t stream);

/* ---- shards of a field ----------------------------------------------------
   Blocks are independent (Sec. IV), so a field splits into contiguous shards
   of whole blocks, one per GPU of a multi-GPU run; only the relative bound
   couples them (e = eb (max - min) over the whole field, Sec. III footnote).
   The steps, each on one shard's GPU and stream:
     1. sz_range: the shard's finite (min, max);
     2. gather every shard's pair (an all-gather of 16 bytes per shard);
     3. sz_compress_shard: the shard's stream with the whole field's bound;
     4. sz_stitch: the shard streams joined section by section into the
        stream of the whole field, byte for byte what sz_compress writes
        (or keep the shard streams and decode each with sz_decompress).
   Shard k covers blocks [k0, k1) of the field; k0 and k1 are multiples of 8
   (k1 may be the field's last block count), so that state bits fill whole
   bytes. A shard stream is a valid stream of its own values as a 1-D field
   (sz_shard_params gives its parameters for sz_compress_bound,
   sz_workspace_size and sz_decompress); its bound is the whole field's. */
#define SZ_MAX_SHARDS 64

/* Parameters of the shard of blocks [k0, k1) of `field` as a 1-D field.
   Host only. Errors: SZ_EINVAL (bad field or block range). */
sz_status sz_shard_params(const sz_params* field, uint64_t k0, uint64_t k1, sz_params* out);

/* Finite range of the N values at d_in (device): d_range[0] = min,
   d_range[1] = max as doubles (exact for both element types), or
   (+inf, -inf) if no value is finite. d_ws as for sz_compress with p.
   Asynchronous on `stream`. */
sz_status sz_range(const sz_params* p, const void* d_in, double* d_range, void* d_ws, uint64_t ws_bytes,
                   hipStream_t stream);

/* Compress the shard of blocks [k0, k1) of `field` (its values at d_in,
   device) into d_out like sz_compress with the shard's parameters, except
   that a relative bound takes its range from the nranges (min, max) pairs at
   d_ranges (device doubles, e.g. every shard's sz_range) instead of the
   shard's own values. Errors as sz_compress; SZ_EINVAL for a bad block range
   or a relative bound without ranges. */
sz_status sz_compress_shard(const sz_params* field, uint64_t k0, uint64_t k1, const void* d_in,
                            const double* d_ranges, uint32_t nranges, void* d_out, uint64_t out_cap,
                            uint64_t* d_out_size, void* d_ws, uint64_t ws_bytes, hipStream_t stream);

/* Join the streams of the nshards shards of `field`, in block order
   (d_shards: host array of device pointers, 16-byte aligned; shard_caps:
   host array of the readable bytes of each shard buffer), into the stream of
   the whole field at d_out (out_cap >= sz_compress_bound(field)). Writes the
   stream size to *d_out_size (device u64), or 0 if the shards do not make up
   the field (block counts, element type, block size or bound disagree).
   Section i of the result is the concatenation of the shards' sections i at
   offsets from an exclusive scan of their sizes. Asynchronous on `stream`,
   allocation-free; the shard headers are read on the device. */
sz_status sz_stitch(const sz_params* field, uint32_t nshards, const void* const* d_shards,
                    const uint64_t* shard_caps, void* d_out, uint64_t out_cap, uint64_t* d_out_size,
                    hipStream_t stream);

/* ---- batches (many fields, one launch per pass) ---------------------------
   A batch compresses (or decompresses) many fields of mixed element types,
   sizes and bounds with one launch per pass over all of them: one extrema
   launch, one range launch, one classification launch, one persistent encode
   launch (float32 tiles of every field, then float64 tiles), one finalize
   launch. Each field's stream is byte-identical to what sz_compress writes
   for it alone (the single call runs the same kernels as a batch of one).
   All fields of a batch share one block size. The batch's descriptor table
   and tile maps live in its workspace: sz_batch_create_* writes them there
   once (a synchronous copy; call it outside graph capture), then every
   sz_batch_run enqueues kernels only (asynchronous, allocation-free,
   graph-capturable). The buffers named in the fields must stay valid and the
   workspace untouched for the life of the batch. */
typedef struct {
  sz_params params;      /* as for sz_compress */
  const void* d_in;      /* device, 16-byte aligned */
  void* d_out;           /* device, 16-byte aligned, out_cap bytes */
  uint64_t out_cap;      /* >= sz_compress_bound(&params) */
  uint64_t* d_out_size;  /* device u64: stream size, 0 on device failure */
} sz_cfield;

typedef struct {
  sz_params expected;  /* as for sz_decompress */
  const void* d_in;    /* device stream, 16-byte aligned */
  uint64_t in_bytes;
  void* d_out;         /* device, 16-byte aligned, out_cap bytes */
  uint64_t out_cap;    /* >= N * sizeof(T) */
  uint32_t* d_status;  /* device u32, as for sz_decompress */
} sz_dfield;

typedef struct sz_batch_s* sz_batch;

/* Workspace bytes of a compression batch (cf) or a decompression batch (df);
   exactly one of cf, df is non-null. 0 for invalid fields. Host only. */
uint64_t sz_batch_workspace_size(const sz_cfield* cf, const sz_dfield* df, uint32_t n);

/* Plan a batch into the device workspace d_ws (16-byte aligned, ws_bytes >=
   sz_batch_workspace_size). Errors: SZ_EINVAL (bad field, mixed block sizes),
   SZ_ENOSPC, SZ_EUNSUPPORTED, SZ_EDEVICE. */
sz_status sz_batch_create_compress(const sz_cfield* fields, uint32_t n, void* d_ws, uint64_t ws_bytes,
                                   sz_batch* out);
sz_status sz_batch_create_decompress(const sz_dfield* fields, uint32_t n, void* d_ws, uint64_t ws_bytes,
                                     sz_batch* out);

/* Launch geometry of the encode pass of a compression batch for the fields of
   one element type: the number of persistent workgroups (the autotuner's
   knob; no effect on the output bytes; values below 8 act as 8, one per
   ticket class of the encoder). A new batch starts from the
   process-wide table of sz_set_geometry for the size class of that type's
   total input bytes. */
sz_status sz_batch_set_geometry(sz_batch b, sz_dtype dtype, uint32_t encode_wgs);

/* Size class of an input of `bytes` bytes for launch-geometry tables:
   0 below 256 KiB, then one class per factor 4, 7 from 1 GiB up. */
uint32_t sz_size_class(uint64_t bytes);

/* Process-wide encode geometry for inputs of one element type and size class,
   used by sz_compress and as the starting geometry of new batches;
   encode_wgs = 0 restores the default (4 per compute unit). Thread-safe;
   no effect on the output bytes. */
sz_status sz_set_geometry(sz_dtype dtype, uint32_t size_class, uint32_t encode_wgs);

/* Enqueue every pass of the batch on `stream`. */
sz_status sz_batch_run(sz_batch b, hipStream_t stream);

/* Release the host handle (the workspace stays the caller's). */
void sz_batch_destroy(sz_batch b);

/* Parse a host copy of a stream header (at least 96 bytes). Fills *out and
   *total_bytes (the full stream size). Returns SZ_ECORRUPT for a bad header,
   SZ_EINVAL for null pointers. Host only. */
sz_status sz_inspect(const void* h_hdr, uint64_t bytes, sz_params* out,
                     uint64_t* total_bytes);

/* Message of the last error returned on the calling thread ("" if none). */
const char* sz_last_error(void);

/* Optional per-kernel timing for measurement. When enabled, every kernel the
   library enqueues is bracketed by HIP events on its stream; sz_timing_read
   waits for them and returns, per kernel name, the number of launches and
   their summed duration in milliseconds since the last read (then resets).
   `names` receives pointers to static strings. Returns the number of entries
   written (at most cap). Not for use under graph capture. */
void sz_timing_enable(int on);
uint32_t sz_timing_read(const char** names, double* total_ms, uint32_t* launches,
                        uint32_t cap);

#ifdef __cplusplus
}
#endif
#endif
