/*
 * szref.h -- CPU oracle of the SZx block-wise error-bounded lossy compressor
 * (Yu, Di, Zhao, Tian, Tao, Liang, Cappello: "SZx: an Ultra-fast Error-bounded
 * Lossy Compressor for Scientific Datasets", arXiv 2201.13020).
 *
 * TEST INFRASTRUCTURE. This library exists only to check the GPU path. Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load or
 * call it. It shares no source, header, table or helper with the HIP library;
 * the two only agree because both follow the same written definition of the
 * method and of the stream layout.
 *
 * Plain single-threaded C11, host pointers only, every floating-point step in
 * the element type T (float or double), round-to-nearest-even, no FMA
 * contraction (-ffp-contract=off), no flush-to-zero.
 *
 * What it computes, step by step (each step cites the paper):
 *   e       : the absolute bound; ABS = eb, REL = eb * (global max - global min)
 *             over the finite values (Sec. III, footnote on the value-range
 *             relative bound), rounded down into T.
 *   blocks  : fixed-size 1-D blocks of b values over the row-major flattening
 *             (Sec. IV, Alg. 1 "for each block"); the last block may be short.
 *   mu      : mean of the block's min and max (Sec. IV, Table I, Alg. 1).
 *   constant: every value within e of mu (Alg. 1 constant test) -> store mu.
 *   otherwise (Sec. IV, eq. (4); Sec. V-A, eq. (5)):
 *             keep K = min(W, 1 + E + m) leading IEEE bits of v = x - mu, with
 *             m = max(0, p(r) - p(e)); shift right by s so the kept bits fill
 *             whole bytes; 2-bit code of identical leading bytes against the
 *             predecessor; the remaining bytes go to the mid-byte array.
 * Readings of points the paper leaves open are listed in the repository's
 * design notes and restated at the place in szref.c where each applies.
 */
#ifndef SZREF_H
#define SZREF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SZREF_F32 = 0, SZREF_F64 = 1 };
enum { SZREF_ABS = 0, SZREF_REL = 1 };
enum {
  SZREF_OK = 0,
  SZREF_EINVAL = 1,
  SZREF_ENOSPC = 2,
  SZREF_ECORRUPT = 3,
  SZREF_ENOMEM = 5
};

typedef struct {
  uint32_t dtype;      /* SZREF_F32 or SZREF_F64 */
  uint32_t ndims;      /* 1..4 */
  uint64_t dims[4];    /* row-major; only their product matters to the method */
  uint32_t eb_mode;    /* SZREF_ABS or SZREF_REL */
  uint32_t block_size; /* power of two in [8, 1024] */
  double eb;           /* >= 0 and finite */
} szref_params;

/* Worst-case stream size for these parameters (every block stored raw). */
uint64_t szref_compress_bound(const szref_params* p);

/* The absolute bound e the compressor uses for this input, widened to double. */
int szref_error_bound(const szref_params* p, const void* in, double* e_out);

/* Compress n = prod(dims) values at `in` into `out` (capacity out_cap).
 * Writes the exact stream size to *out_size. */
int szref_compress(const szref_params* p, const void* in, void* out,
                   uint64_t out_cap, uint64_t* out_size);

/* Parse the 96-byte header: parameters and total stream size. */
int szref_inspect(const void* in, uint64_t in_bytes, szref_params* p,
                  uint64_t* total_bytes);

/* Decompress a stream of in_bytes bytes into `out` (capacity out_cap bytes). */
int szref_decompress(const void* in, uint64_t in_bytes, void* out,
                     uint64_t out_cap);

#ifdef __cplusplus
}
#endif
#endif
