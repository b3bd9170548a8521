/* szx_server.h -- serving runtime over the SZx kernels of libszx.so.
 *
 * A request loop with continuous batching. Compression and decompression
 * requests arrive at any time from any thread. They are admitted in arrival
 * order while a slot and enough of the device arena are free. Every
 * admission gathers all queued requests that fit (up to max_batch) into one
 * launch group. The group runs as a batch (the batched entry points of
 * szx.h) on that slot's stream, so the work of several groups overlaps on
 * the device. Compressed streams stay resident in the arena as items, which
 * later decompression requests read.
 *
 * Results do not depend on the mix. Each compressed stream is byte-identical
 * to what sz_compress writes for that field alone, and each decompressed
 * field is bit-identical to sz_decompress. The batched path runs the
 * single-call kernels, and no step of the method reads another field.
 *
 * Ownership. The server allocates its arena (hbm_budget bytes of device
 * memory), its streams, events and pinned host staging at creation, and
 * nothing on the device afterwards. The caller owns compression inputs and
 * caller-given decompression outputs, and keeps them valid until the
 * request completes. Items belong to the server until released.
 *
 * Clock. Timestamps are nanoseconds on a steady clock from the server's
 * creation (sz_server_clock).
 *
 * The method is the paper's, unchanged (Sec. III-V): this layer only
 * schedules it.
 */
#ifndef SZX_SERVER_H
#define SZX_SERVER_H

#include <stdint.h>

#include "szx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sz_server_s* sz_server;

typedef struct {
  int device;           /* HIP device ordinal */
  uint64_t hbm_budget;  /* bytes of the device arena (items, reservations, workspaces) */
  uint32_t slots;       /* streams, each with one launch group in flight: 1..16 */
  uint32_t max_batch;   /* requests per launch group: 1..65536 */
  uint32_t block_size;  /* block size of every compression (power of two, 8..1024) */
  uint32_t reserved;
} sz_server_config;

typedef enum { SZ_REQ_COMPRESS = 0, SZ_REQ_DECOMPRESS = 1 } sz_req_kind;

typedef struct {
  uint64_t request;       /* id returned at submission */
  uint32_t kind;          /* sz_req_kind */
  uint32_t status;        /* SZ_OK; SZ_ENOMEM if the request can never fit
                             the arena; SZ_ECORRUPT / SZ_EDEVICE from the device */
  uint64_t item;          /* compress: the new resident stream; decompress: the item read */
  uint64_t out_item;      /* decompress into the arena: the item holding the values, else 0 */
  uint64_t bytes_in;      /* uncompressed bytes of the field */
  uint64_t stream_bytes;  /* compressed bytes */
  uint64_t t_arrival;     /* as given at submission (or the submission time) */
  uint64_t t_admit;       /* launch group formed */
  uint64_t t_done;        /* group's work finished on the device (observed on the host) */
  uint32_t group_size;    /* requests in its launch group */
  uint32_t slot;
  uint64_t t_dev_begin;   /* its group's span on the device: HIP events on the slot's
                             stream before the group's first copy and after its last, */
  uint64_t t_dev_end;     /* in ns from an event recorded at creation (0: unavailable) */
} sz_completion;

typedef struct {
  uint64_t arena_bytes, arena_in_use, arena_peak;
  uint64_t queued, in_flight_groups, groups_launched, completed, items_resident;
  uint64_t peak_in_flight_groups; /* most launch groups launched and not yet completed at once */
} sz_server_stats;

/* Create a server on cfg->device (allocates the arena, streams with default
   priority, and pinned staging). Errors: SZ_EINVAL, SZ_ENOMEM, SZ_EDEVICE. */
sz_status sz_server_create(const sz_server_config* cfg, sz_server* out);

/* Stop admitting, discard queued requests (no completion is reported for
   them), wait for work in flight, free everything. */
void sz_server_destroy(sz_server s);

/* Nanoseconds since the server's creation. */
uint64_t sz_server_clock(sz_server s);

/* Queue a compression of the device field d_in (16-byte aligned, p->block_size
   must equal the server's). t_arrival: the request's arrival time on the
   server clock (0: now), from which its latency counts. */
sz_status sz_server_submit_compress(sz_server s, const sz_params* p, const void* d_in, uint64_t t_arrival,
                                    uint64_t* request);

/* Queue a decompression of a resident item into d_out (device, 16-byte
   aligned, out_cap >= N * sizeof(T)), or, with d_out == NULL, into a new
   arena item reported as out_item. The item must have completed; it is kept
   until every decompression queued on it has completed, even if released. */
sz_status sz_server_submit_decompress(sz_server s, uint64_t item, void* d_out, uint64_t out_cap, uint64_t t_arrival,
                                      uint64_t* request);

/* Move up to max completions into out, waiting up to wait_us microseconds for
   the first. Returns the number moved. */
uint32_t sz_server_poll(sz_server s, sz_completion* out, uint32_t max, uint32_t wait_us);

/* Parameters, size and device address of a resident item (a compressed
   stream, or decompressed values for an out_item). */
sz_status sz_server_item_info(sz_server s, uint64_t item, sz_params* params, uint64_t* bytes, const void** d_data);

/* Enqueue a device-to-device copy of an item's bytes into d_dst on `stream`. */
sz_status sz_server_copy_item(sz_server s, uint64_t item, void* d_dst, uint64_t cap, hipStream_t stream);

/* Give an item's arena bytes back (deferred while decompressions read it). */
sz_status sz_server_release(sz_server s, uint64_t item);

sz_status sz_server_get_stats(sz_server s, sz_server_stats* out);

/* One request of a load trace for sz_server_replay. */
typedef struct {
  uint64_t t_arrival;  /* ns on the server clock */
  uint32_t kind;       /* sz_req_kind */
  uint32_t pick;       /* decompress: the resident item pool[pick % pool size] */
  sz_params params;    /* compress */
  const void* d_in;    /* compress: device input (16-byte aligned) */
} sz_trace_req;

/* Load driver for measurements: submits the requests in order at their
   arrival times from the calling thread (spinning on the server clock) and
   collects completions in between, so that the submitter is not the
   bottleneck. Completed compressions join a pool of resident items (warm[0..
   nwarm) first; at most keep items, the oldest released beyond that) from
   which decompressions pick; decompressions write into the arena and their
   values are released on completion. A decompression finding the pool empty
   is skipped (status SZ_EINVAL in its completion). Returns when every
   request has completed or timeout_ms has passed (SZ_EDEVICE). out[i] is
   request i's completion; *npool receives the pool's final size and pool its
   items (capacity max(nwarm, keep)). */
sz_status sz_server_replay(sz_server s, const sz_trace_req* reqs, uint32_t n, const uint64_t* warm,
                           uint32_t nwarm, uint32_t keep, uint32_t timeout_ms, sz_completion* out,
                           uint64_t* pool, uint32_t* npool);

#ifdef __cplusplus
}
#endif

#endif /* SZX_SERVER_H */
