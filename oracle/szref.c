/*
 * szref.c -- CPU oracle of the SZx compressor: stream layout, parameter checks
 * and dispatch to the per-type code in szref_typed.inc.
 *
 * TEST INFRASTRUCTURE (see szref.h). Plain, single-threaded, slow on purpose.
 *
 * Stream layout ("format v1"; the paper prints no byte layout -- its figure of
 * the mid-byte array is not reproduced -- so this layout is this project's own
 * reading of the outputs listed at the end of Alg. 1 in Sec. IV: the mu array,
 * the 2-bit leading-byte code array and the mid-byte array):
 *
 *   96-byte header, all integers little-endian:
 *     0  u32 magic "SZXM"        4  u8 version (1)     5  u8 dtype
 *     6  u8  eb_mode             7  u8 ndims           8  u32 block size b
 *     12 u32 reserved (0)        16 u64 dims[4]        48 u64 N
 *     56 f64 eb as given         64 u64 bit pattern of e (zero-extended)
 *     72 u64 nblk                80 u64 n_nc           88 u64 mid_total
 *   then five sections, each starting at a multiple of 16 (zero padding):
 *     state bits  ceil(nblk/8) bytes; bit k%8 of byte k/8 is 1 when block k
 *                 is non-constant (raw blocks included)
 *     mu          nblk values of type T
 *     K           one byte per non-constant block (0xFF = raw block)
 *     codes       b/4 bytes per non-constant block, 4 codes per byte, first
 *                 element in the two most significant bits
 *     mid bytes   mid_total bytes; elements in order, each element's kept
 *                 bytes most significant first
 */
#include "szref.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define HDR_BYTES 96u
#define MAGIC 0x4D585A53u /* the bytes 'S' 'Z' 'X' 'M' read little-endian */
#define VERSION 1u

static uint64_t align16(uint64_t x) { return (x + 15u) & ~(uint64_t)15u; }

static void put_u32(uint8_t* p, uint32_t v) {
  for (int i = 0; i < 4; ++i) p[i] = (uint8_t)(v >> (8 * i));
}
static void put_u64(uint8_t* p, uint64_t v) {
  for (int i = 0; i < 8; ++i) p[i] = (uint8_t)(v >> (8 * i));
}
static uint32_t get_u32(const uint8_t* p) {
  uint32_t v = 0;
  for (int i = 0; i < 4; ++i) v |= (uint32_t)p[i] << (8 * i);
  return v;
}
static uint64_t get_u64(const uint8_t* p) {
  uint64_t v = 0;
  for (int i = 0; i < 8; ++i) v |= (uint64_t)p[i] << (8 * i);
  return v;
}

/* Byte offsets of the five sections and the total size. */
typedef struct {
  uint64_t state, mu, kbytes, codes, mid, total;
} szref_layout;

static szref_layout make_layout(uint64_t nblk, uint64_t n_nc, uint64_t w,
                                uint64_t b, uint64_t mid_total) {
  szref_layout L;
  L.state = HDR_BYTES;
  L.mu = align16(L.state + (nblk + 7) / 8);
  L.kbytes = align16(L.mu + nblk * w);
  L.codes = align16(L.kbytes + n_nc);
  L.mid = align16(L.codes + n_nc * (b / 4));
  L.total = L.mid + mid_total;
  return L;
}

/* Everything the typed code needs about a call, after validation. */
typedef struct {
  uint32_t dtype, eb_mode, ndims, b;
  uint64_t dims[4];
  uint64_t n, nblk;
  double eb;
} szref_job;

static int is_pow2_block(uint32_t b) {
  return b >= 8 && b <= 1024 && (b & (b - 1)) == 0;
}

static int check_params(const szref_params* p, szref_job* j) {
  if (!p) return SZREF_EINVAL;
  if (p->dtype > 1 || p->eb_mode > 1) return SZREF_EINVAL;
  if (p->ndims < 1 || p->ndims > 4) return SZREF_EINVAL;
  if (!is_pow2_block(p->block_size)) return SZREF_EINVAL;
  if (!(p->eb >= 0.0) || !isfinite(p->eb)) return SZREF_EINVAL;
  uint64_t n = 1;
  for (uint32_t d = 0; d < p->ndims; ++d) {
    if (p->dims[d] != 0 && n > (UINT64_MAX >> 4) / p->dims[d]) return SZREF_EINVAL;
    n *= p->dims[d];
  }
  if (n > ((uint64_t)1 << 40)) return SZREF_EINVAL;
  j->dtype = p->dtype;
  j->eb_mode = p->eb_mode;
  j->ndims = p->ndims;
  j->b = p->block_size;
  for (int d = 0; d < 4; ++d) j->dims[d] = (uint32_t)d < p->ndims ? p->dims[d] : 0;
  j->n = n;
  j->nblk = (n + p->block_size - 1) / p->block_size;
  j->eb = p->eb;
  return SZREF_OK;
}

static void write_header(uint8_t* out, const szref_job* j, uint64_t e_bits,
                         uint64_t n_nc, uint64_t mid_total) {
  memset(out, 0, HDR_BYTES);
  put_u32(out + 0, MAGIC);
  out[4] = VERSION;
  out[5] = (uint8_t)j->dtype;
  out[6] = (uint8_t)j->eb_mode;
  out[7] = (uint8_t)j->ndims;
  put_u32(out + 8, j->b);
  put_u32(out + 12, 0);
  for (int d = 0; d < 4; ++d) put_u64(out + 16 + 8 * d, j->dims[d]);
  put_u64(out + 48, j->n);
  uint64_t ebits;
  memcpy(&ebits, &j->eb, 8);
  put_u64(out + 56, ebits);
  put_u64(out + 64, e_bits);
  put_u64(out + 72, j->nblk);
  put_u64(out + 80, n_nc);
  put_u64(out + 88, mid_total);
}

/* Header fields as read back from a stream. */
typedef struct {
  szref_job job;
  uint64_t e_bits, n_nc, mid_total;
  szref_layout L;
} szref_header;

static int read_header(const uint8_t* in, uint64_t in_bytes, szref_header* h) {
  if (!in || in_bytes < HDR_BYTES) return SZREF_ECORRUPT;
  if (get_u32(in) != MAGIC || in[4] != VERSION) return SZREF_ECORRUPT;
  szref_params p;
  memset(&p, 0, sizeof p);
  p.dtype = in[5];
  p.eb_mode = in[6];
  p.ndims = in[7];
  p.block_size = get_u32(in + 8);
  for (int d = 0; d < 4; ++d) p.dims[d] = get_u64(in + 16 + 8 * d);
  uint64_t ebits = get_u64(in + 56);
  memcpy(&p.eb, &ebits, 8);
  if (check_params(&p, &h->job) != SZREF_OK) return SZREF_ECORRUPT;
  for (uint32_t d = p.ndims; d < 4; ++d)
    if (p.dims[d] != 0) return SZREF_ECORRUPT;
  if (get_u64(in + 48) != h->job.n) return SZREF_ECORRUPT;
  if (get_u64(in + 72) != h->job.nblk) return SZREF_ECORRUPT;
  h->e_bits = get_u64(in + 64);
  h->n_nc = get_u64(in + 80);
  h->mid_total = get_u64(in + 88);
  if (h->n_nc > h->job.nblk) return SZREF_ECORRUPT;
  uint64_t w = h->job.dtype == SZREF_F32 ? 4 : 8;
  if (h->mid_total > h->job.n * w) return SZREF_ECORRUPT;
  h->L = make_layout(h->job.nblk, h->n_nc, w, h->job.b, h->mid_total);
  if (h->L.total > in_bytes) return SZREF_ECORRUPT;
  return SZREF_OK;
}

/* ---- the method, once per element type ---------------------------------- */

#define SZREF_CAT2(a, b) a##_##b
#define SZREF_CAT(a, b) SZREF_CAT2(a, b)

#define T float
#define UT uint32_t
#define WBITS 32
#define EBITS 8
#define BIAS 127
#define TMAX FLT_MAX
#define SFX f32
#include "szref_typed.inc"
#undef T
#undef UT
#undef WBITS
#undef EBITS
#undef BIAS
#undef TMAX
#undef SFX

#define T double
#define UT uint64_t
#define WBITS 64
#define EBITS 11
#define BIAS 1023
#define TMAX DBL_MAX
#define SFX f64
#include "szref_typed.inc"
#undef T
#undef UT
#undef WBITS
#undef EBITS
#undef BIAS
#undef TMAX
#undef SFX

/* ---- public entry points ------------------------------------------------- */

uint64_t szref_compress_bound(const szref_params* p) {
  szref_job j;
  if (check_params(p, &j) != SZREF_OK) return 0;
  uint64_t w = j.dtype == SZREF_F32 ? 4 : 8;
  return make_layout(j.nblk, j.nblk, w, j.b, j.n * w).total;
}

int szref_error_bound(const szref_params* p, const void* in, double* e_out) {
  szref_job j;
  int rc = check_params(p, &j);
  if (rc != SZREF_OK) return rc;
  if (!in && j.n) return SZREF_EINVAL;
  if (j.dtype == SZREF_F32) {
    float e;
    rc = error_bound_f32(&j, (const float*)in, &e);
    *e_out = e;
  } else {
    double e;
    rc = error_bound_f64(&j, (const double*)in, &e);
    *e_out = e;
  }
  return rc;
}

int szref_compress(const szref_params* p, const void* in, void* out,
                   uint64_t out_cap, uint64_t* out_size) {
  szref_job j;
  int rc = check_params(p, &j);
  if (rc != SZREF_OK) return rc;
  if ((!in && j.n) || !out || !out_size) return SZREF_EINVAL;
  if (out_cap < szref_compress_bound(p)) return SZREF_ENOSPC;
  if (j.dtype == SZREF_F32)
    return compress_f32(&j, (const float*)in, (uint8_t*)out, out_size);
  return compress_f64(&j, (const double*)in, (uint8_t*)out, out_size);
}

int szref_inspect(const void* in, uint64_t in_bytes, szref_params* p,
                  uint64_t* total_bytes) {
  szref_header h;
  int rc = read_header((const uint8_t*)in, in_bytes, &h);
  if (rc != SZREF_OK) return rc;
  if (p) {
    memset(p, 0, sizeof *p);
    p->dtype = h.job.dtype;
    p->eb_mode = h.job.eb_mode;
    p->ndims = h.job.ndims;
    p->block_size = h.job.b;
    for (int d = 0; d < 4; ++d) p->dims[d] = h.job.dims[d];
    p->eb = h.job.eb;
  }
  if (total_bytes) *total_bytes = h.L.total;
  return SZREF_OK;
}

int szref_decompress(const void* in, uint64_t in_bytes, void* out,
                     uint64_t out_cap) {
  szref_header h;
  int rc = read_header((const uint8_t*)in, in_bytes, &h);
  if (rc != SZREF_OK) return rc;
  uint64_t w = h.job.dtype == SZREF_F32 ? 4 : 8;
  if (out_cap < h.job.n * w) return SZREF_ENOSPC;
  if (!out && h.job.n) return SZREF_EINVAL;
  if (h.job.dtype == SZREF_F32)
    return decompress_f32((const uint8_t*)in, &h, (float*)out);
  return decompress_f64((const uint8_t*)in, &h, (double*)out);
}
