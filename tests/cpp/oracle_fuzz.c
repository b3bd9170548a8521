/* Corrupted streams against the oracle's decoder, built with address and
 * undefined-behaviour sanitizers: every decode of a damaged stream must end
 * in SZREF_OK or SZREF_ECORRUPT without reading or writing outside the exact
 * buffers it is given (any such access aborts the run).
 *
 * Damage: single bit flips anywhere, random bytes stamped into each section,
 * every truncation, and random bytes after a valid header. Fields: smooth
 * float32 and float64 series whose lengths leave a short last block, at two
 * block sizes. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "szref.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static uint64_t next_u64(void) { /* xorshift64* */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return rng_state * 0x2545F4914F6CDD1Dull;
}

static uint64_t below(uint64_t n) { return n ? next_u64() % n : 0; }

static int decode_copy(const uint8_t* s, uint64_t len, uint64_t out_bytes) {
  /* exact-size heap copies, so that any overrun is caught */
  uint8_t* in = (uint8_t*)malloc(len ? len : 1);
  uint8_t* out = (uint8_t*)malloc(out_bytes ? out_bytes : 1);
  if (!in || !out) abort();
  memcpy(in, s, len);
  const int rc = szref_decompress(in, len, out, out_bytes);
  free(in);
  free(out);
  return rc;
}

static int check(int rc, const char* what, uint64_t at) {
  if (rc != SZREF_OK && rc != SZREF_ECORRUPT) {
    fprintf(stderr, "%s at %llu: status %d\n", what, (unsigned long long)at, rc);
    return 1;
  }
  return 0;
}

static int fuzz_one(uint32_t dtype, uint64_t n, uint32_t block) {
  const uint64_t w = dtype == SZREF_F32 ? 4 : 8;
  uint8_t* x = (uint8_t*)malloc(n * w);
  if (!x) abort();
  for (uint64_t i = 0; i < n; ++i) {
    const double t = (double)i / (double)n;
    double v = sin(2 * M_PI * 7.0 * t) + 0.5 * sin(2 * M_PI * 53.0 * t + 1.0);
    v += 1e-4 * ((double)(next_u64() >> 11) / 9007199254740992.0 - 0.5);
    if (t > 0.3 && t < 0.35) v = 0.0; /* constant blocks */
    if (dtype == SZREF_F32) {
      const float f = (float)v;
      memcpy(x + i * 4, &f, 4);
    } else {
      memcpy(x + i * 8, &v, 8);
    }
  }
  szref_params p;
  memset(&p, 0, sizeof p);
  p.dtype = dtype;
  p.ndims = 1;
  p.dims[0] = n;
  p.eb_mode = SZREF_REL;
  p.block_size = block;
  p.eb = 1e-3;
  const uint64_t cap = szref_compress_bound(&p);
  uint8_t* s = (uint8_t*)malloc(cap);
  uint64_t len = 0;
  if (!s || szref_compress(&p, x, s, cap, &len) != SZREF_OK) {
    fprintf(stderr, "compress failed\n");
    return 1;
  }
  int bad = 0;
  bad |= decode_copy(s, len, n * w) != SZREF_OK;
  uint8_t* c = (uint8_t*)malloc(len);
  if (!c) abort();
  for (int trial = 0; trial < 3000 && !bad; ++trial) { /* single bit flips */
    memcpy(c, s, len);
    const uint64_t at = below(len);
    c[at] ^= (uint8_t)(1u << below(8));
    bad |= check(decode_copy(c, len, n * w), "bit flip", at);
  }
  for (int trial = 0; trial < 2000 && !bad; ++trial) { /* byte stomps past the header */
    memcpy(c, s, len);
    const uint64_t at = 96 + below(len - 96);
    const int k = 1 + (int)below(8);
    for (int j = 0; j < k && at + j < len; ++j) c[at + j] = (uint8_t)next_u64();
    bad |= check(decode_copy(c, len, n * w), "stomp", at);
  }
  for (uint64_t cut = 0; cut < len && !bad; ++cut) /* every truncation */
    bad |= check(decode_copy(s, cut, n * w), "truncation", cut);
  for (int trial = 0; trial < 500 && !bad; ++trial) { /* garbage after a valid header */
    memcpy(c, s, 96);
    for (uint64_t j = 96; j < len; ++j) c[j] = (uint8_t)next_u64();
    bad |= check(decode_copy(c, len, n * w), "garbage body", (uint64_t)trial);
  }
  /* a too-small output buffer is rejected, not overrun */
  if (!bad && decode_copy(s, len, n * w - 1) == SZREF_OK) {
    fprintf(stderr, "short output accepted\n");
    bad = 1;
  }
  free(c);
  free(s);
  free(x);
  return bad;
}

int main(void) {
  int bad = 0;
  bad |= fuzz_one(SZREF_F32, 5003, 64);
  bad |= fuzz_one(SZREF_F32, 3001, 128);
  bad |= fuzz_one(SZREF_F64, 2999, 64);
  bad |= fuzz_one(SZREF_F64, 1537, 128);
  if (bad) return 1;
  printf("oracle fuzz ok\n");
  return 0;
}
