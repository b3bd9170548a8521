// szx_compress.hip -- compression kernels of the SZx method for gfx950.
//
// Pipeline of one sz_compress call, or of one batch of fields (all on the
// caller's stream; every pass is one launch over all fields of the batch, a
// single call being a batch of one, so both run the same code):
//   k_stats     clears the counters, tickets and tile status words the later
//               passes use; per-block totalOrder min/max (Alg. 1 needs both
//               for mu_k); each workgroup folds its finite value range into
//               one of the field's range slots (two 64-bit atomic maxima)
//   k_classify  the absolute bound e (for the relative bound: eb times the
//               field's finite range, Sec. III footnote -- every wave folds
//               the range slots itself), then mid-range mu and constant test
//               of every block (Alg. 1), the state bits and the mu section; a
//               light single-pass prefix count of non-constant blocks gives
//               each encode tile its first rank. The field's last tile writes
//               the header (all but the mid-byte total) and the section
//               padding, and leaves the range slots zero for the next call.
//   k_encode    per non-constant block: normalise, keep K bits (eq. (4)), shift
//               (eq. (5)), verify the bound where it is not proved a priori,
//               2-bit leading-byte codes and mid bytes. Persistent workgroups
//               take tiles from interleaved ticket counters (float32 tiles of
//               all fields, then float64 tiles); each tile's output offset comes
//               from a single-pass prefix sum over its field's tiles (Sec. V-B),
//               and while a tile waits for it the next tile's data is loaded.
//               Bytes are packed in LDS and leave in aligned 16-byte stores.
//               A single call's last tile, once its offset is known, writes
//               the mid-byte total and the stream size.
//   k_finalize  batches: every field's mid-byte total and stream size, and
//               the header of fields without values (a single call only
//               runs it when its field has no values)
#include <algorithm>

#include "szx_device.hpp"
#include "szx_launch.hpp"

namespace szx {

// The stream size while a compression runs (the classification pass sets
// it, the field's last encode tile replaces it).
constexpr uint64_t kSizePending = ~0ull;

// Field of a call, or of a batch entry, as the kernels see it (a copy with
// its pointers typed as global memory).
// BATCH: false for a single call (the descriptor is the kernel argument
// itself), true for a table in memory, else decided at run time.
enum : int { kAnyCall = -1, kSingle = 0, kBatch = 1 };
template <int BATCH = kAnyCall>
__device__ __forceinline__ FieldC field_at(const CBatch& b, uint32_t fi) {
  FieldC f = BATCH == kSingle ? b.one : BATCH == kBatch ? b.fields[fi] : (b.fields ? b.fields[fi] : b.one);
  f.in = as_global(f.in);
  f.out = as_global(f.out);
  f.out_size = as_global(f.out_size);
  f.ctr = as_global(f.ctr);
  f.clean = as_global(f.clean);
  f.range = as_global(f.range);
  f.ext_range = as_global(f.ext_range);
  f.parts = as_global(f.parts);
  f.stats = as_global(f.stats);
  f.plan = as_global(f.plan);
  f.enc_r0 = as_global(f.enc_r0);
  f.cls_status = as_global(f.cls_status);
  f.enc_mid = as_global(f.enc_mid);
  return f;
}
template <int BATCH = kAnyCall>
__device__ __forceinline__ uint32_t field_of(const uint32_t* map, uint64_t t) {
  return BATCH == kSingle ? 0u : BATCH == kBatch ? map[t] : (map ? map[t] : 0u);
}

// Load EPL consecutive values starting at element i0 (aligned to EPL); values
// at or beyond n are zero. Returns the number of valid values.
template <typename T, int EPL>
__device__ __forceinline__ int load_run(const T* __restrict__ x, uint64_t i0, uint64_t n, T (&v)[EPL]) {
  constexpr int PER16 = 16 / sizeof(T);
  if (i0 + EPL <= n) {
    const uint4* p = reinterpret_cast<const uint4*>(x + i0);
#pragma unroll
    for (int c = 0; c < EPL / PER16; ++c) {
      const uint4 u = p[c];
      if constexpr (sizeof(T) == 4) {
        v[c * 4 + 0] = __uint_as_float(u.x);
        v[c * 4 + 1] = __uint_as_float(u.y);
        v[c * 4 + 2] = __uint_as_float(u.z);
        v[c * 4 + 3] = __uint_as_float(u.w);
      } else {
        v[c * 2 + 0] = __longlong_as_double((long long)(((uint64_t)u.y << 32) | u.x));
        v[c * 2 + 1] = __longlong_as_double((long long)(((uint64_t)u.w << 32) | u.z));
      }
    }
    return EPL;
  }
  int cnt = 0;
#pragma unroll
  for (int i = 0; i < EPL; ++i) {
    const bool ok = i0 + i < n;
    v[i] = ok ? x[i0 + i] : (T)0;
    cnt += ok ? 1 : 0;
  }
  return cnt;
}

// Load the first cnt of EPL consecutive values at x + i0 (aligned to EPL);
// the others are zero.
template <typename T, int EPL>
__device__ __forceinline__ void load_count(const T* __restrict__ x, uint32_t i0, int cnt, T (&v)[EPL]) {
  if (cnt == EPL) {
    load_run<T, EPL>(x, i0, (uint64_t)i0 + EPL, v);
    return;
  }
#pragma unroll
  for (int i = 0; i < EPL; ++i) v[i] = i < cnt ? x[i0 + i] : (T)0;
}

// Inclusive running min (MAX = false) or max over groups of G consecutive
// lanes: the group's last lane ends with the group's extremum. DPP row shifts
// for G <= 16 (no LDS), lane shuffles otherwise.
template <int G, typename U, bool MAX>
__device__ __forceinline__ U group_scan_last(U v) {
  if constexpr (G == 1) {
    return v;
  } else if constexpr (G <= 16) {
    const int lg = lane_id() & (G - 1);
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      U o;
      if constexpr (sizeof(U) == 4) {
        o = (U)dpp_shr(d, (uint32_t)v);
      } else {
        const uint32_t lo = dpp_shr(d, (uint32_t)v), hi = dpp_shr(d, (uint32_t)(v >> 32));
        o = ((U)hi << 32) | lo;
      }
      const U m = MAX ? (o > v ? o : v) : (o < v ? o : v);
      v = lg >= d ? m : v;
    }
    return v;
  } else {
    return MAX ? group_max<G, U>(v) : group_min<G, U>(v);
  }
}

// ----------------------------------------------------------------- stats ---

// Per-block totalOrder extrema (as keys) of all values over a chunk of
// kStatsChunk tiles of one field (two tiles per iteration keep more loads in
// flight), and the chunk's finite range folded into one of the field's range
// slots.
template <typename T, int B>
__device__ __forceinline__ void stats_tile(const T (&v)[Geo<T, B>::EPL], int cnt, uint64_t i0, uint64_t nblk,
                                           typename Traits<T>::U* __restrict__ stats,
                                           typename Traits<T>::U& flo, typename Traits<T>::U& fhi) {
  using U = typename Traits<T>::U;
  constexpr int EPL = Geo<T, B>::EPL, LPB = Geo<T, B>::LPB;
  U kmin = (U)~(U)0, kmax = 0;
  if (cnt == EPL) {  // every lane but the field's last partial one
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      const U k = order_key<U>(bits_of(v[i]));
      kmin = k < kmin ? k : kmin;
      kmax = k > kmax ? k : kmax;
    }
  } else {
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      const U k = order_key<U>(bits_of(v[i]));
      kmin = (i < cnt && k < kmin) ? k : kmin;
      kmax = (i < cnt && k > kmax) ? k : kmax;
    }
  }
  // the block's extrema gather in the group's last lane
  kmin = group_scan_last<LPB, U, false>(kmin);
  kmax = group_scan_last<LPB, U, true>(kmax);
  const uint64_t blk = i0 / B;
  const bool last = (threadIdx.x % LPB) == LPB - 1;
  if (last && blk < nblk) {
    // one store for the pair (8- or 16-byte aligned: the array starts 256-byte aligned)
    if constexpr (sizeof(U) == 4) {
      *reinterpret_cast<uint2*>(stats + 2 * blk) = make_uint2(kmin, kmax);
    } else {
      *reinterpret_cast<ulonglong2*>(stats + 2 * blk) = make_ulonglong2(kmin, kmax);
    }
  }
  // finite range: a block whose extrema are finite is finite throughout and
  // adds [kmin, kmax]; a block holding a NaN or an infinity (rare) adds its
  // finite values one by one, in every lane of its group
  const bool finite = kmin >= FiniteKeys<T>::LO && kmax <= FiniteKeys<T>::HI;
  if (last && finite && blk < nblk) {
    flo = kmin < flo ? kmin : flo;
    fhi = kmax > fhi ? kmax : fhi;
  }
  const uint64_t odd = __ballot(last && !finite && blk < nblk);
  const int gl = (lane_id() & ~(LPB - 1)) + LPB - 1;  // the group's last lane
  if ((odd >> gl) & 1ull) {
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      const U u = bits_of(v[i]);
      const U k = order_key<U>(u);
      const bool fin = i < cnt && is_finite_bits<T>(u);
      flo = (fin && k < flo) ? k : flo;
      fhi = (fin && k > fhi) ? k : fhi;
    }
  }
}

// Per-block totalOrder extrema (as keys) of all values over a chunk of
// kStatsChunk tiles of one field (two tiles per iteration keep more loads in
// flight), and the chunk's finite range folded into one of the field's range
// slots -- or, on the field's first use of the workspace, stored as the
// chunk's partial.
template <typename T, int B>
__device__ __forceinline__ void stats_chunk(const FieldC& f, uint64_t c, uint64_t* s_lo, uint64_t* s_hi) {
  using U = typename Traits<T>::U;
  using G = Geo<T, B>;
  constexpr int EPL = G::EPL;
  const T* x = reinterpret_cast<const T*>(f.in);
  U* stats = reinterpret_cast<U*>(f.stats);
  U flo = (U)~(U)0, fhi = 0;
  const uint64_t ntile = cdiv(f.n, (uint64_t)G::TILE);
  const uint64_t t0 = c * kStatsChunk;
  const uint64_t t1 = std::min<uint64_t>(ntile, t0 + kStatsChunk);
  for (uint64_t t = t0; t < t1; t += 2) {
    const uint64_t i0 = t * G::TILE + (uint64_t)threadIdx.x * EPL;
    const uint64_t i1 = i0 + G::TILE;
    const bool second = t + 1 < t1;
    T v0[EPL], v1[EPL];
    const int c0 = load_run<T, EPL>(x, i0, f.n, v0);
    const int c1 = second ? load_run<T, EPL>(x, i1, f.n, v1) : 0;
    stats_tile<T, B>(v0, c0, i0, f.nblk, stats, flo, fhi);
    if (second) stats_tile<T, B>(v1, c1, i1, f.nblk, stats, flo, fhi);
  }
  flo = group_min<kWave, U>(flo);
  fhi = group_max<kWave, U>(fhi);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    s_lo[w] = flo;
    s_hi[w] = fhi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t lo = s_lo[0], hi = s_hi[0];
    for (int i = 1; i < kWavesPerWG; ++i) {
      lo = s_lo[i] < lo ? s_lo[i] : lo;
      hi = s_hi[i] > hi ? s_hi[i] : hi;
    }
    if (*f.clean != kCleanWord) {
      // lo > hi: no finite value
      *reinterpret_cast<ulonglong2*>(f.parts + 2 * c) = make_ulonglong2(lo, hi);
    } else if (lo <= hi) {  // the chunk saw a finite value
      uint64_t* slot = f.range + (c % f.nslots) * (kRangeStride / 8);
      atomicMax((unsigned long long*)slot, ~(unsigned long long)lo);
      atomicMax((unsigned long long*)slot + 1, (unsigned long long)hi);
    }
  }
}

// Every extrema workgroup (of both element types) also clears its slice of
// the words that the later passes count, publish and wait on: they run after
// this pass, and nothing in it reads them. A single call and a batch take
// separate (uniform) paths, so that each reads its descriptor with scalar
// loads: one expression choosing between the kernel argument and the table
// would read it through a generic pointer.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_stats(CBatch b) {
  __shared__ uint64_t s_lo[kWavesPerWG], s_hi[kWavesPerWG];
  constexpr int DT = sizeof(T) == 4 ? 0 : 1;
  const uint64_t g = blockIdx.x;
  const uint64_t all = b.tiles_stats[0] + b.tiles_stats[1];
  for (uint64_t i = ((DT ? b.tiles_stats[0] : 0) + g) * kWG + threadIdx.x; i < b.zero_words; i += all * kWG)
    b.zero_begin[i] = 0;
  if (b.fields) {
    const FieldC f = field_at<kBatch>(b, field_of<kBatch>(b.field_stats[DT], g));
    stats_chunk<T, B>(f, g - f.base_stats, s_lo, s_hi);
  } else {
    const FieldC f = field_at<kSingle>(b, 0);
    stats_chunk<T, B>(f, g, s_lo, s_hi);
  }
}

// ----------------------------------------------------------------- range ---

__device__ __forceinline__ uint64_t bound_of(const FieldC& f, uint64_t lo, uint64_t hi) {
  const int rel = f.eb_mode == 1;
  return f.dtype == 0 ? (uint64_t)bits_of(bound_from<float>(rel, f.eb, lo, hi))
                      : (uint64_t)bits_of(bound_from<double>(rel, f.eb, lo, hi));
}

// The bound e of a field (as the bits of a T) from its parameters and, for
// the relative bound, the field's finite range (no finite value: the range
// is empty and e = 0). Every thread of classification tile t calls it.
// Range slots in use (clean): each wave folds them by itself, one per lane.
// First use: tile t = 0 folds the chunks' partials and publishes the bound
// in the counters; the other tiles wait for it (tile 0 waits on nothing, and
// a workgroup runs only once every lower-numbered one has been dispatched).
// Contains a barrier on the first-use path of tile 0.
__device__ __forceinline__ uint64_t field_bound(const FieldC& f, uint32_t t, bool clean, uint64_t nchunks,
                                               uint64_t* s_red) {
  if (f.eb_mode != 1) return bound_of(f, ~0ull, 0ull);  // absolute bound: no range needed
  const uint32_t l = lane_id();
  if (f.next_range) {
    // a shard of a larger field: the range of the whole field from the
    // shards' ranges (pairs of doubles, which hold the element values exactly)
    double lo = __builtin_inf(), hi = -__builtin_inf();
    for (uint32_t i = l; i < f.next_range; i += kWave) {
      const double a = f.ext_range[2 * i], c = f.ext_range[2 * i + 1];
      lo = a < lo ? a : lo;
      hi = c > hi ? c : hi;
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const double a = __shfl_xor(lo, d), c = __shfl_xor(hi, d);
      lo = a < lo ? a : lo;
      hi = c > hi ? c : hi;
    }
    if (!(lo <= hi) || f.eb == 0.0) return bound_of(f, ~0ull, 0ull);  // no finite value
    return f.dtype == 0 ? (uint64_t)bits_of(round_down_to<float>(f.eb * (hi - lo)))
                        : (uint64_t)bits_of(round_down_to<double>(f.eb * (hi - lo)));
  }
  if (clean) {
    uint64_t lo_inv = 0, hi = 0;
    if (l < f.nslots) {
      lo_inv = f.range[l * (kRangeStride / 8)];
      hi = f.range[l * (kRangeStride / 8) + 1];
    }
    lo_inv = group_max<kWave, uint64_t>(lo_inv);
    hi = group_max<kWave, uint64_t>(hi);
    return bound_of(f, ~lo_inv, hi);
  }
  if (t == 0) {
    uint64_t lo = ~0ull, hi = 0;
    // eight partials in flight per thread
    constexpr int U = 8;
    const ulonglong2* parts = reinterpret_cast<const ulonglong2*>(f.parts);
    for (uint64_t i0 = 0; i0 < nchunks; i0 += (uint64_t)U * kWG) {
      ulonglong2 p[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t i = i0 + (uint64_t)u * kWG + threadIdx.x;
        p[u] = i < nchunks ? parts[i] : make_ulonglong2(~0ull, 0ull);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        lo = p[u].x < lo ? p[u].x : lo;
        hi = p[u].y > hi ? p[u].y : hi;
      }
    }
    lo = group_min<kWave, uint64_t>(lo);
    hi = group_max<kWave, uint64_t>(hi);
    const int w = threadIdx.x / kWave;
    if (l == 0) {
      s_red[2 * w] = lo;
      s_red[2 * w + 1] = hi;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kWavesPerWG; ++i) {
      lo = s_red[2 * i] < lo ? s_red[2 * i] : lo;
      hi = s_red[2 * i + 1] > hi ? s_red[2 * i + 1] : hi;
    }
    const uint64_t e_bits = bound_of(f, lo, hi);
    if (threadIdx.x == 0) {
      f.ctr->e_bits = e_bits;
      __hip_atomic_store(&f.ctr->e_ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    return e_bits;
  }
  // relaxed polls (an acquiring load would invalidate caches at every poll),
  // one acquire fence once the flag is up
  uint32_t spins = 0;
  while (__hip_atomic_load(&f.ctr->e_ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
    if (++spins > kSpinLimit) {
      if (l == 0) atomicMax(&f.ctr->err, 1u);
      return 0;
    }
    __builtin_amdgcn_s_sleep(8);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return __hip_atomic_load(&f.ctr->e_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Parameters of one block from its totalOrder extrema (keys): K = -1 for a
// block with a non-finite value (stored raw), 0 for a constant block, else the
// kept bits of eq. (4). verify is false where the bound is proved a priori.
template <typename T>
struct BlockPlan {
  T mu;
  int K;
  bool verify;
};

template <typename T>
__device__ __forceinline__ BlockPlan<T> plan_block(typename Traits<T>::U kmin, typename Traits<T>::U kmax, T e) {
  using U = typename Traits<T>::U;
  BlockPlan<T> p;
  p.mu = (T)0;
  p.K = -1;
  p.verify = true;
  if (kmin < FiniteKeys<T>::LO || kmax > FiniteKeys<T>::HI) return p;
  const T mn = from_bits<T>(key_to_bits<U>(kmin));
  const T mx = from_bits<T>(key_to_bits<U>(kmax));
  int m0;
  if (classify_block<T>(mn, mx, e, p.mu, m0)) {
    p.K = 0;
    return p;
  }
  p.K = kept_bits<T>(m0);
  // A priori bound: truncation errs by < 2^p(e); the two roundings (of x - mu
  // and of mu + v') by at most 2^(p(M) - (mantissa bits - 2)) together, with
  // M = max(|mn|, |mx|). If e - 2^p(e) covers that, every value passes.
  constexpr int MANT = Traits<T>::W - 1 - Traits<T>::E;
  const U emask = FiniteKeys<T>::EXPMASK;
  const U ebits = bits_of(e);
  const U pow2_bits = (ebits & emask) ? (ebits & emask) : ((U)1 << MANT);
  const T slack = e - from_bits<T>(pow2_bits);  // exact: same binade
  const T amn = mn < (T)0 ? -mn : mn, amx = mx < (T)0 ? -mx : mx;
  const T M = amn > amx ? amn : amx;
  const bool slack_normal = slack > (T)0 && (bits_of(slack) & emask) != 0;
  p.verify = !(slack_normal && exp_of<T>(slack) >= exp_of<T>(M) - (MANT - 2));
  return p;
}

// A block's plan in one byte: 0 constant, 0xFF raw, else K with bit 7 set
// when the values must be verified.
template <typename T>
__device__ __forceinline__ uint32_t plan_byte(const BlockPlan<T>& p) {
  return p.K < 0 ? 0xFFu : p.K == 0 ? 0u : (uint32_t)p.K | (p.verify ? 0x80u : 0u);
}

// ---------------------------------------------------------------- header ---

// Header and the zero padding after the state bits, mu, K and codes sections
// of a field's stream, by the threads of one workgroup. Returns the stream
// size.
__device__ __forceinline__ uint64_t write_stream_header(const FieldC& f, uint64_t e_bits, uint64_t n_nc,
                                                        uint64_t mid_total) {
  const uint32_t w = f.dtype == 0 ? 4 : 8;
  const Sections s = sections(f.nblk, n_nc, w, f.b, mid_total);
  uint8_t* out = f.out;
  if (threadIdx.x == 0) {
    uint32_t* o32 = reinterpret_cast<uint32_t*>(out);
    uint64_t* o64 = reinterpret_cast<uint64_t*>(out);
    o32[0] = kMagic;
    o32[1] = (uint32_t)kVersion | (f.dtype << 8) | (f.eb_mode << 16) | (f.ndims << 24);
    o32[2] = f.b;
    o32[3] = 0;
    for (int d = 0; d < 4; ++d) o64[2 + d] = f.dims[d];
    o64[6] = f.n;
    o64[7] = (uint64_t)__double_as_longlong(f.eb);
    o64[8] = e_bits;
    o64[9] = f.nblk;
    o64[10] = n_nc;
    o64[11] = mid_total;
  }
  const uint64_t pads[4][2] = {{96 + cdiv(f.nblk, 8), s.mu},
                               {s.mu + f.nblk * w, s.kbytes},
                               {s.kbytes + n_nc, s.codes},
                               {s.codes + n_nc * (f.b / 4), s.mid}};
  for (int p = 0; p < 4; ++p)
    for (uint64_t i = pads[p][0] + threadIdx.x; i < pads[p][1]; i += blockDim.x) out[i] = 0;
  return s.total;
}

// The end of a field's stream, by its last encode tile once that tile's
// offset is known: the mid-byte total (the header's last field) and the
// stream size, or 0 there if a bounded wait of this compression gave up.
// (Every tile's wait ends once all tiles before it have published, which the
// last tile's own wait has seen, so no wait can give up after this.)
__device__ __forceinline__ void finish_stream(const FieldC& f, uint64_t mid_off, uint64_t mid_total) {
  reinterpret_cast<uint64_t*>(f.out)[11] = mid_total;
  const uint32_t err = __hip_atomic_load(&f.ctr->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  *f.out_size = err ? 0 : mid_off + mid_total;
}

// -------------------------------------------------------------- classify ---

// mu and the constant test of every block, the state bits, and the rank of the
// first non-constant block of every encode tile (a prefix count over tiles of
// CLS blocks, four per thread at most). The last tile writes n_nc.
template <typename T, int B>
__device__ __forceinline__ void classify_tile(const FieldC& f, uint32_t t, uint32_t* s_scan, uint32_t* s_state,
                                              uint64_t* s_base, uint64_t* s_red) {
  using U = typename Traits<T>::U;
  using G = Geo<T, B>;
  constexpr int TBLK = G::TBLK;
  constexpr int CLS = TBLK > (int)kClsMin ? TBLK : (int)kClsMin;
  constexpr int BPT = CLS / kWG;  // blocks per thread
  const U* stats = reinterpret_cast<const U*>(f.stats);
  const uint64_t nblk = f.nblk;
  const uint64_t k0 = (uint64_t)t * CLS + (uint64_t)threadIdx.x * BPT;
  static_assert(BPT == 4, "four blocks per thread");
  // a thread's blocks are consecutive and start 16-byte aligned in the
  // extrema, mu and plan arrays, so a full group moves as 16-byte words. The
  // extrema come through a buffer resource over the tile's blocks (reads
  // past the field's last block return zeros): one load form for every lane,
  // so the range slots' loads below go out before any of them is waited for
  const bool full = k0 + BPT <= nblk;
  U kmin[BPT], kmax[BPT];
  {
    const uint64_t kt = (uint64_t)t * CLS;
    const uint32_t nb_t = (uint32_t)std::min<uint64_t>(nblk - kt, (uint64_t)CLS);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<U*>(stats + 2 * kt), (short)0, (int)(nb_t * 2u * (uint32_t)sizeof(U)), 0x00020000);
    using v4u = unsigned int __attribute__((ext_vector_type(4)));
    U w[2 * BPT];
    constexpr int NQ = 2 * BPT * (int)sizeof(U) / 16;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const v4u u = __builtin_amdgcn_raw_buffer_load_b128(
          rs, (int)((uint32_t)threadIdx.x * (uint32_t)(2 * BPT * sizeof(U)) + 16u * (uint32_t)q), 0, 0);
      reinterpret_cast<v4u*>(w)[q] = u;
    }
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      kmin[i] = w[2 * i];
      kmax[i] = w[2 * i + 1];
    }
  }
  const bool clean = *f.clean == kCleanWord;
  for (int i = threadIdx.x; i < CLS / 32; i += kWG) s_state[i] = 0;
  const uint64_t nchunks = cdiv(cdiv(f.n, (uint64_t)Geo<T, B>::TILE), (uint64_t)kStatsChunk);
  const uint64_t e_bits = field_bound(f, t, clean, nchunks, s_red);
  __syncthreads();
  const T e = from_bits<T>((U)e_bits);
  if (t == 0 && threadIdx.x == 0) {
    f.ctr->e_bits = e_bits;  // read by the encode pass
    *f.out_size = kSizePending;
  }
  const uint32_t ntiles = (uint32_t)cdiv(nblk, CLS);
  T* mus = reinterpret_cast<T*>(f.out + f.mu_off);
  uint32_t cnt = 0, bits = 0;
  T mv[BPT];
  uint32_t pv = 0;  // plan bytes, block i in byte i
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const uint64_t k = k0 + i;
    mv[i] = (T)0;
    if (k < nblk) {
      const BlockPlan<T> p = plan_block<T>(kmin[i], kmax[i], e);
      mv[i] = p.mu;
      pv |= plan_byte(p) << (8 * i);
      const bool nc = p.K != 0;
      cnt += nc ? 1u : 0u;
      bits |= (nc ? 1u : 0u) << i;
    }
  }
  if (full) {
    constexpr int NQ = BPT * (int)sizeof(T) / 16;
#pragma unroll
    for (int q = 0; q < NQ; ++q) reinterpret_cast<uint4*>(mus + k0)[q] = reinterpret_cast<const uint4*>(mv)[q];
    *reinterpret_cast<uint32_t*>(f.plan + k0) = pv;
  } else {
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      if (k0 + i < nblk) {
        mus[k0 + i] = mv[i];
        f.plan[k0 + i] = (uint8_t)(pv >> (8 * i));
      }
    }
  }
  if (bits) atomicOr(&s_state[(threadIdx.x * BPT) / 32], bits << ((threadIdx.x * BPT) % 32));
  uint32_t total;
  const uint32_t ex = wg_excl_sum<uint32_t>(cnt, s_scan, total);  // has barriers
  if (threadIdx.x < kWave) {
    if (threadIdx.x == 0) lookback_publish(f.cls_status, t, total);
    const uint64_t p = lookback_resolve_n(f.cls_status, t, total, &f.ctr->err, 1u, ntiles);
    if (threadIdx.x == 0) *s_base = p;
  }
  // state bytes of this tile, never past the state section
  const uint64_t state_bytes = (nblk + 7) / 8;
  for (int i = threadIdx.x; i < CLS / 8; i += kWG) {
    const uint64_t byte = (uint64_t)t * (CLS / 8) + i;
    if (byte < state_bytes) f.out[96 + byte] = (uint8_t)(s_state[i / 4] >> (8 * (i % 4)));
  }
  __syncthreads();
  const uint64_t base = *s_base;
  // first rank of every encode tile that starts in this thread's blocks
  if ((k0 % TBLK) == 0 && k0 < nblk) f.enc_r0[k0 / TBLK] = base + ex;
  if (t == ntiles - 1) {
    // Every tile has published, so every tile has read the range slots: the
    // last one clears them for the next call and marks them clean; it also
    // writes the header (the encode pass adds the mid-byte total) and the
    // padding between the sections.
    const uint64_t n_nc = base + total;
    if (threadIdx.x == 0) f.ctr->n_nc = n_nc;
    if (threadIdx.x < kRangeSlots)
      *reinterpret_cast<ulonglong2*>(f.range + threadIdx.x * (kRangeStride / 8)) = make_ulonglong2(0, 0);
    if (threadIdx.x == 0) *f.clean = kCleanWord;
    write_stream_header(f, e_bits, n_nc, 0);
  }
}

template <typename T, int B>
__global__ __launch_bounds__(256) void k_classify(CBatch b) {
  constexpr int CLS = Geo<T, B>::TBLK > (int)kClsMin ? Geo<T, B>::TBLK : (int)kClsMin;
  __shared__ uint32_t s_scan[kWavesPerWG];
  __shared__ uint32_t s_state[CLS / 32 > 32 ? CLS / 32 : 32];
  __shared__ uint64_t s_base;
  __shared__ uint64_t s_red[2 * kWavesPerWG];
  const uint64_t g = blockIdx.x;
  const FieldC f = field_at(b, field_of(b.field_cls[Traits<T>::BYTES / 8], g));
  classify_tile<T, B>(f, (uint32_t)(g - f.base_cls), s_scan, s_state, &s_base, s_red);
}

// ---------------------------------------------------------------- encode ---

// Truncate v = x - mu to K leading bits, shifted right by s into nb whole
// bytes; when verify is set, check that every valid value reconstructs within
// e exactly. Returns false if some value fails.
template <typename T, int EPL>
__device__ __forceinline__ bool encode_try(const T (&x)[EPL], int cnt, T mu, T e, int K, bool verify,
                                           typename Traits<T>::U (&q)[EPL]) {
  using U = typename Traits<T>::U;
  const int s = shift_of(K);
  const U keep = top_bytes_mask<U>(bytes_of(K));
#pragma unroll
  for (int i = 0; i < EPL; ++i) q[i] = (U)(bits_of(x[i] - mu) >> s) & keep;
  bool ok = true;
  if (verify) {  // one branch per row, none per value
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      const T xr = mu + from_bits<T>((U)(q[i] << s));
      // bitwise on purpose: both checks, no short-circuit branch
      const bool good = (bool)((int)exact_le<T>(x[i], xr, e) & (int)exact_le<T>(xr, x[i], e));
      ok = (bool)((int)ok & ((int)good | (int)(i >= cnt)));
      // one value at a time: interleaving all of them costs registers, and
      // this path is rare
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  return ok;
}

// Appends byte strings to a lane's run of the LDS byte stream, a ring of
// bmask + 1 bytes. The ring is zeroed beforehand and every full dword is
// OR-ed in (the first and last may be shared with the neighbouring lanes), so
// the only per-value branch is the predicated store itself.
struct LanePacker {
  uint8_t* stage;
  uint32_t da;     // ring byte of the dword being filled (a multiple of 4)
  uint32_t lo, hi; // pending bytes, the next byte of the stream in the low byte of lo
  uint32_t fill;   // pending bits (< 32)
  uint32_t bmask;  // ring bytes - 1 (a power of two less one)
  __device__ __forceinline__ LanePacker(uint32_t* st, uint32_t off, uint32_t bm)
      : stage(reinterpret_cast<uint8_t*>(st)), da(off & ~3u & bm), lo(0), hi(0), fill((off & 3u) * 8u), bmask(bm) {}
  // L <= 4 bytes of sv, first byte in the low byte, bytes above L zero
  __device__ __forceinline__ void put4(uint32_t sv, int L) {
    const uint64_t sh = (uint64_t)sv << fill;
    lo |= (uint32_t)sh;
    hi |= (uint32_t)(sh >> 32);
    const uint32_t nf = fill + 8u * (uint32_t)L;  // < 64
    fill = nf & 31u;
    if (nf > 31u) {
      atomicOr(reinterpret_cast<uint32_t*>(stage + da), lo);
      da = (da + 4u) & bmask;
      lo = hi;
      hi = 0;
    }
  }
  __device__ __forceinline__ void put(uint32_t sv, int L) { put4(sv, L); }
  // L <= 8 bytes of sv at once: the 96-bit window lo, hi, x takes them at
  // bit `fill`, and up to two full dwords leave
  __device__ __forceinline__ void put(uint64_t sv, int L) {
    const uint64_t a = (uint64_t)(uint32_t)sv << fill;
    const uint64_t b = (sv >> 32) << fill;
    lo |= (uint32_t)a;
    hi |= (uint32_t)(a >> 32) | (uint32_t)b;
    const uint32_t x = (uint32_t)(b >> 32);
    const uint32_t nf = fill + 8u * (uint32_t)L;  // < 96
    fill = nf & 31u;
    if (nf > 31u) {
      atomicOr(reinterpret_cast<uint32_t*>(stage + da), lo);
      da = (da + 4u) & bmask;
      lo = hi;
      hi = x;
      if (nf > 63u) {
        atomicOr(reinterpret_cast<uint32_t*>(stage + da), lo);
        da = (da + 4u) & bmask;
        lo = hi;
        hi = 0;
      }
    }
  }
  __device__ __forceinline__ void flush() {
    if (fill > 0) atomicOr(reinterpret_cast<uint32_t*>(stage + da), lo);
  }
};

// The bytes of v after its c lowest ones (c in [0, 3]; v's string after
// dropping c leading bytes when the first byte is the low one).
__device__ __forceinline__ uint32_t drop_low_bytes(uint32_t v, uint32_t c) {
  return __builtin_amdgcn_alignbyte(0u, v, c);
}
__device__ __forceinline__ uint64_t drop_low_bytes(uint64_t v, uint32_t c) {
  const uint32_t l = (uint32_t)v, h = (uint32_t)(v >> 32);
  return ((uint64_t)__builtin_amdgcn_alignbyte(0u, h, c) << 32) | __builtin_amdgcn_alignbyte(h, l, c);
}

// Copy total staged bytes to out + [dst, dst + total). They start at the
// 16-byte word at16 of the LDS ring of mask16 + 1 such words (a power of two)
// and may wrap around its end. Whole aligned 16-byte chunks of the
// destination go out as single stores, the shared first and last chunks byte
// by byte. Chunk c of the destination starts at staged byte 16 c - a (a = dst
// mod 16, the same for every chunk), so its bytes lie in the two staged
// 16-byte words c - 1 and c (c when a = 0): every lane reads two consecutive
// 16-byte words (a wave reads a contiguous range: no LDS bank conflicts; five
// strided dword reads per chunk put 64 lanes on 8 banks) and realigns them
// with byte funnel shifts by the same amount.
__device__ __forceinline__ void copy_out(uint8_t* __restrict__ out, uint64_t dst, const uint32_t* stage,
                                         uint32_t at16, uint32_t mask16, uint32_t total) {
  const uint4* ring = reinterpret_cast<const uint4*>(stage);
  const uint32_t st = (uint32_t)(dst & 15u);
  uint8_t* base = out + (dst - st);
  const uint32_t end = st + total;
  const uint32_t nchunk = (end + 15) / 16;
  const uint32_t b = (16u - st) & 15u;  // byte of the chunk's start in the first stage word read
  const uint32_t k = b >> 2, sh = b & 3u;
  const uint32_t back = st ? 1u : 0u;
  const uint32_t bmask = mask16 * 16u + 15u;
  for (uint32_t c = threadIdx.x; c < nchunk; c += kWG) {
    const uint32_t lo = c * 16 < st ? st : c * 16;
    const uint32_t hi = c * 16 + 16 > end ? end : c * 16 + 16;
    if (lo == c * 16 && hi == c * 16 + 16) {
      // c >= 1 here whenever st > 0 (chunk 0 is then partial)
      const uint4 q0 = ring[(at16 + c - back) & mask16];
      const uint4 q1 = ring[(at16 + c - back + 1) & mask16];
      const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
      uint4 u;
      // k is the same for every lane: a uniform branch picks the words
      switch (k) {
        case 0:
          u = make_uint4(__builtin_amdgcn_alignbyte(w[1], w[0], sh), __builtin_amdgcn_alignbyte(w[2], w[1], sh),
                         __builtin_amdgcn_alignbyte(w[3], w[2], sh), __builtin_amdgcn_alignbyte(w[4], w[3], sh));
          break;
        case 1:
          u = make_uint4(__builtin_amdgcn_alignbyte(w[2], w[1], sh), __builtin_amdgcn_alignbyte(w[3], w[2], sh),
                         __builtin_amdgcn_alignbyte(w[4], w[3], sh), __builtin_amdgcn_alignbyte(w[5], w[4], sh));
          break;
        case 2:
          u = make_uint4(__builtin_amdgcn_alignbyte(w[3], w[2], sh), __builtin_amdgcn_alignbyte(w[4], w[3], sh),
                         __builtin_amdgcn_alignbyte(w[5], w[4], sh), __builtin_amdgcn_alignbyte(w[6], w[5], sh));
          break;
        default:
          u = make_uint4(__builtin_amdgcn_alignbyte(w[4], w[3], sh), __builtin_amdgcn_alignbyte(w[5], w[4], sh),
                         __builtin_amdgcn_alignbyte(w[6], w[5], sh), __builtin_amdgcn_alignbyte(w[7], w[6], sh));
          break;
      }
      *reinterpret_cast<uint4*>(base + c * 16) = u;
    } else {
      for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t bi = (at16 * 16u + i - st) & bmask;
        base[i] = (uint8_t)(stage[bi >> 2] >> ((bi & 3u) * 8u));
      }
    }
  }
}

// Clear the ring's 16-byte words that hold total bytes from word at16 on.
__device__ __forceinline__ void ring_clear(uint32_t* stage, uint32_t at16, uint32_t mask16, uint32_t total) {
  uint4* ring = reinterpret_cast<uint4*>(stage);
  const uint32_t nw = (total + 15) / 16;
  for (uint32_t i = threadIdx.x; i < nw; i += kWG) ring[(at16 + i) & mask16] = make_uint4(0, 0, 0, 0);
}

// Per-row plan of a tile's blocks as one lane sees them: K (-1 raw, 0
// constant or no block, else kept bits), whether the values need verifying,
// how many values the lane holds, and the rank of the row's block among the
// tile's non-constant ones. For float64 the four are packed into one word
// per row (K + 1 in bits 0-6, verify in bit 7, the count in bits 8-12, the
// rank from bit 13): that encoder is at its register cap and spills
// otherwise; for float32 plain fields measured faster.
template <typename T, int B, bool PACK = (sizeof(T) == 8)>
struct RowPlan;

template <typename T, int B>
struct RowPlan<T, B, false> {
  static constexpr int SUB = Geo<T, B>::SUB;
  int K_[SUB], cnt_[SUB];
  bool verify_[SUB];
  uint32_t rank_[SUB];
  __device__ __forceinline__ void set(int s, int K, bool verify, int cnt) {
    K_[s] = K;
    verify_[s] = verify;
    cnt_[s] = cnt;
  }
  __device__ __forceinline__ void set_rank(int s, uint32_t r) { rank_[s] = r; }
  __device__ __forceinline__ int K(int s) const { return K_[s]; }
  __device__ __forceinline__ bool verify(int s) const { return verify_[s]; }
  __device__ __forceinline__ int cnt(int s) const { return cnt_[s]; }
  __device__ __forceinline__ uint32_t rank(int s) const { return rank_[s]; }
};

template <typename T, int B>
struct RowPlan<T, B, true> {
  static constexpr int SUB = Geo<T, B>::SUB;
  static_assert(Geo<T, B>::EPL <= 31 && Geo<T, B>::TBLK <= (1 << 19), "packed row fields overflow");
  uint32_t meta[SUB];
  __device__ __forceinline__ void set(int s, int K, bool verify, int cnt) {
    meta[s] = (uint32_t)(K + 1) | (verify ? 0x80u : 0u) | ((uint32_t)cnt << 8);
  }
  __device__ __forceinline__ void set_rank(int s, uint32_t r) { meta[s] |= r << 13; }
  __device__ __forceinline__ int K(int s) const { return (int)(meta[s] & 0x7Fu) - 1; }
  __device__ __forceinline__ bool verify(int s) const { return (meta[s] >> 7) & 1u; }
  __device__ __forceinline__ int cnt(int s) const { return (int)((meta[s] >> 8) & 31u); }
  __device__ __forceinline__ uint32_t rank(int s) const { return meta[s] >> 13; }
};

// What a workgroup holds of one tile between its loads and its encoding.
template <typename T, int B>
struct TileIn {
  T x[Geo<T, B>::SUB][Geo<T, B>::EPL];
  T mu[Geo<T, B>::SUB];
  RowPlan<T, B> row;
  uint64_t r0;                    // rank of the tile's first non-constant block
  uint32_t field;                 // batch entry
  uint32_t tile;                  // tile within the field
  T e;                            // the field's bound and non-constant block count,
  uint64_t n_nc;                  // read with the tile so their latency hides too
};

// Loads tile t: each block's mu (from the stream) and plan byte (both left
// by the classification pass), ranks within the tile (barriers), and the
// values of its non-constant blocks (left in flight).
template <typename T, int B>
__device__ __forceinline__ void tile_load(TileIn<T, B>& in, uint32_t t, const T* __restrict__ x,
                                          const T* __restrict__ mus, const uint8_t* __restrict__ plan,
                                          const uint64_t* __restrict__ enc_r0, uint64_t n, uint64_t nblk,
                                          uint32_t* s_scan) {
  using G = Geo<T, B>;
  constexpr int EPL = G::EPL, LPB = G::LPB, TB = G::TB, SUB = G::SUB, TBLK = G::TBLK;
  const int g = threadIdx.x / LPB, lig = threadIdx.x % LPB;
  in.r0 = enc_r0[t];
  uint32_t first[SUB];
  if constexpr (sizeof(T) == 4) {
    // the tile's first block and value (wave-uniform), its block and value
    // counts; lanes index from them with 32-bit offsets. (For float64 the
    // same form measured slower: it left the encoder spilling registers.)
    const uint64_t kb = (uint64_t)t * TBLK;
    const uint32_t nblk_t = (uint32_t)std::min<uint64_t>(nblk - kb, (uint64_t)TBLK);
    const uint32_t nval_t = (uint32_t)std::min<uint64_t>(n - kb * B, (uint64_t)TBLK * B);
    const T* x_t = x + kb * B;
    const T* mus_t = mus + kb;
    const uint8_t* plan_t = plan + kb;
    // every row's mu and plan byte first, then the values: vector loads
    // return in order, so a row's plan byte read after the previous row's
    // values would wait for them (one memory latency per row)
    uint32_t pbs[SUB];
#pragma unroll
    for (int s = 0; s < SUB; ++s) {
      const uint32_t lk = (uint32_t)(s * TB + g);
      in.mu[s] = (T)0;
      pbs[s] = 0;
      if (lk < nblk_t) {
        in.mu[s] = mus_t[lk];
        pbs[s] = plan_t[lk];
      }
    }
    // The values through a buffer resource over the tile's values (to the
    // field's end): reads past its range return zeros without touching
    // memory, so lanes of constant blocks (sent far past it) and a short
    // block's run past the field's end need no branch. With one load form
    // for every lane no lane's loads wait on another's (two forms writing
    // the same registers made every row wait for all loads before it).
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(x_t), (short)0, (int)(nval_t * sizeof(T)), 0x00020000);
    using v4u = unsigned int __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int s = 0; s < SUB; ++s) {
      const uint32_t lk = (uint32_t)(s * TB + g);
      const bool inb = lk < nblk_t;
      const uint32_t pb = pbs[s];
      const int K = pb == 0xFFu ? -1 : (int)(pb & 0x7Fu);
      // values from this lane's first one to the tile's end (constant blocks load none)
      const int rem = (int)nval_t - (int)(lk * B) - lig * EPL;
      const int cnt = (inb && K != 0) ? (rem < 0 ? 0 : (rem > EPL ? EPL : rem)) : 0;
      in.row.set(s, K, (pb & 0x80u) != 0 && pb != 0xFFu, cnt);
      const uint32_t off = cnt > 0 ? (lk * B + (uint32_t)(lig * EPL)) * 4u : 0x40000000u;
#pragma unroll
      for (int c = 0; c < EPL / 4; ++c) {
        const v4u u = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off + 16u * (uint32_t)c), 0, 0);
        in.x[s][4 * c + 0] = __uint_as_float(u.x);
        in.x[s][4 * c + 1] = __uint_as_float(u.y);
        in.x[s][4 * c + 2] = __uint_as_float(u.z);
        in.x[s][4 * c + 3] = __uint_as_float(u.w);
      }
      first[s] = (lig == 0 && K != 0) ? 1u : 0u;
    }
  } else {
    uint32_t pbs[SUB];  // as above: every row's plan byte before any value
#pragma unroll
    for (int s = 0; s < SUB; ++s) {
      const uint64_t k = (uint64_t)t * TBLK + (uint64_t)s * TB + g;
      in.mu[s] = (T)0;
      pbs[s] = 0;
      if (k < nblk) {
        in.mu[s] = mus[k];
        pbs[s] = plan[k];
      }
    }
#pragma unroll
    for (int s = 0; s < SUB; ++s) {
      const uint64_t k = (uint64_t)t * TBLK + (uint64_t)s * TB + g;
      const uint32_t pb = pbs[s];
      const int K = pb == 0xFFu ? -1 : (int)(pb & 0x7Fu);
      const uint64_t nk = (k < nblk && K != 0) ? std::min<uint64_t>((uint64_t)B, n - k * B) : 0;
      const int cnt = (int)((uint64_t)lig * EPL >= nk ? 0 : std::min<uint64_t>(EPL, nk - (uint64_t)lig * EPL));
      in.row.set(s, K, (pb & 0x80u) != 0 && pb != 0xFFu, cnt);
      load_run<T, EPL>(x, k * B + (uint64_t)lig * EPL, k * B + nk, in.x[s]);
      first[s] = (lig == 0 && K != 0) ? 1u : 0u;
    }
  }
  uint32_t tot[SUB], rank[SUB];
  wg_excl_scan_multi<SUB>(first, rank, tot, s_scan);
  // the group's first lane counted its block; the others see it counted
#pragma unroll
  for (int s = 0; s < SUB; ++s) in.row.set_rank(s, rank[s] - ((lig != 0 && in.row.K(s) != 0) ? 1u : 0u));
}

// Bytes of the encoder's LDS ring: the least power of two that holds a
// tile's worst case (every value stored whole).
template <typename T, int B>
constexpr uint32_t enc_ring_bytes() {
  constexpr uint32_t worst = (uint32_t)(Geo<T, B>::TILE * Geo<T, B>::SUB * (int)sizeof(T));
  uint32_t r = 16;
  while (r < worst) r *= 2;
  return r;
}

// The encode pass for the tiles of element type T: persistent workgroups take
// tickets from the kTicketClasses counters of this type; ticket i of class c
// is global tile kTicketClasses * i + c, global tiles running over the fields
// of this type in order.
//
// A workgroup stages each tile's mid bytes in an LDS ring (a power of two of
// at least one tile's worst case) and leaves it there, pending, while it
// encodes its next tile behind it; only then does it resolve the pending
// tile's offset in the mid section and copy it out. By then the tiles before
// it have long published their sizes, so the look-back finds them without
// waiting, and its latency overlaps the next tile's loads. When a tile's
// bytes would reach the pending tile's, the pending one is written out first
// (incompressible tiles: no overlap, as with one stage).
template <typename T, int B, int BATCH>
__device__ __forceinline__ void encode_pass(const CBatch& b, uint32_t* s_scan, uint32_t* s_tile, uint64_t* s_base,
                                            uint64_t* s_end, uint32_t* s_stage) {
  using U = typename Traits<T>::U;
  using G = Geo<T, B>;
  constexpr int EPL = G::EPL, LPB = G::LPB, SUB = G::SUB;
  constexpr int BYTES = Traits<T>::BYTES;
  constexpr uint32_t RING = enc_ring_bytes<T, B>();
  constexpr uint32_t MASK16 = RING / 16 - 1;
  constexpr int DT = sizeof(T) == 4 ? 0 : 1;
  const uint64_t ntiles = b.tiles_enc[DT];
  if (ntiles == 0) return;
  // A single call's workgroup 0 is the scan wave of the tiles' mid-byte
  // offsets (the others wait on one status word each); a batch's tiles, of
  // many fields, resolve their offsets by look-back.
  if constexpr (BATCH == kSingle) {
    if (blockIdx.x == 0) {
      if (threadIdx.x < kWave) {
        const FieldC f = field_at<BATCH>(b, 0);
        scan_wave<16>(f.enc_mid, ntiles, &f.ctr->err, 1u);
      }
      return;
    }
  }
  const uint32_t wid = BATCH == kSingle ? blockIdx.x - 1 : blockIdx.x;
  const uint32_t cls = wid % kTicketClasses;
  uint32_t* ticket = b.tickets + (DT * kTicketClasses + cls) * 64;
  const int lig = threadIdx.x % LPB;

  auto claim = [&]() -> uint64_t {
    if (threadIdx.x == 0) *s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint64_t v = (uint64_t)*s_tile * kTicketClasses + cls;
    __syncthreads();
    return v;
  };
  auto load = [&](TileIn<T, B>& in, uint64_t gt) {
    const uint32_t fi = field_of<BATCH>(b.field_enc[DT], gt);
    const FieldC f = field_at<BATCH>(b, fi);
    in.field = fi;
    in.tile = (uint32_t)(gt - f.base_enc);
    in.e = from_bits<T>((U)f.ctr->e_bits);
    in.n_nc = f.ctr->n_nc;
    tile_load<T, B>(in, in.tile, reinterpret_cast<const T*>(f.in), reinterpret_cast<const T*>(f.out + f.mu_off),
                    f.plan, f.enc_r0, f.n, f.nblk, s_scan);
  };

  for (uint32_t i = threadIdx.x; i <= MASK16; i += kWG) reinterpret_cast<uint4*>(s_stage)[i] = make_uint4(0, 0, 0, 0);
  uint64_t gt = claim();
  if (gt >= ntiles) return;
  TileIn<T, B> cur;
  load(cur, gt);
  // a single call's last tile leaves its stream end to after the loop, where
  // nothing else is live (written in the loop, it made the loop spill); the
  // mid-byte total waits in LDS
  if (threadIdx.x == 0) *s_end = ~0ull;

  // the pending tile (same in every lane): encoded into the ring from byte
  // p_at (16-byte aligned), its offset not yet resolved
  bool pend = false;
  uint32_t p_tile = 0, p_field = 0, p_bytes = 0, p_at = 0;
  uint32_t at = 0;  // ring byte of the current tile's start (16-byte aligned)
  // Resolve the pending tile's offset, copy it out and clear its ring bytes.
  // A single call's tile waits on its own status word, which the scan wave
  // publishes; a batch's walks back by look-back, one status word per lane a
  // round (status loads go to the device's coherence point, and wider
  // windows measured slower).
  auto flush = [&](uint64_t first_poll) {
    const FieldC fp = field_at<BATCH>(b, p_field);
    if constexpr (BATCH == kSingle) {
      if (threadIdx.x == 0) *s_base = scan_wait(fp.enc_mid, p_tile, p_bytes, &fp.ctr->err, 1u, first_poll);
    } else if (threadIdx.x < kWave) {
      // the predecessor's word was read before the next tile's loads: when
      // it already holds its inclusive prefix (the common case by now), that
      // is this tile's offset, published as the look-back would
      const uint64_t w0 = __shfl(first_poll, 0);
      uint64_t p;
      if (p_tile > 0 && (w0 >> 62) == 2) {
        p = w0 & kValueMask;
        if (threadIdx.x == 0) status_store(fp.enc_mid + p_tile, kFlagIncl | ((p + p_bytes) & kValueMask));
      } else {
        p = lookback_resolve<1>(fp.enc_mid, p_tile, p_bytes, &fp.ctr->err, 1u);
      }
      if (threadIdx.x == 0) *s_base = p;
    }
    __syncthreads();
    const uint64_t base = *s_base;
    const uint64_t mid = sections(fp.nblk, fp.ctr->n_nc, BYTES, B, 0).mid;
    // the output holds the worst case (every block raw; the caller's capacity
    // is checked against it): an offset past it can only come from a failed
    // wait, which has raised the error already
    if (mid + base + p_bytes <= sections(fp.nblk, fp.nblk, BYTES, B, fp.n * BYTES).total)
      copy_out(fp.out, mid + base, s_stage, p_at / 16, MASK16, p_bytes);
    if (p_tile == cdiv(fp.nblk, G::TBLK) - 1) {
      // the field's last tile ends the mid section: its total (the last
      // header field) and the stream size
      if (threadIdx.x == 0) {
        if constexpr (BATCH == kSingle)
          *s_end = base + p_bytes;
        else
          fp.ctr->mid_total = base + p_bytes;  // for the finishing pass
      }
    }
    __syncthreads();
    ring_clear(s_stage, p_at / 16, MASK16, p_bytes);
    pend = false;
  };

  for (;;) {
    const FieldC f = field_at<BATCH>(b, cur.field);
    const uint32_t t = cur.tile;
    const T e = cur.e;
    const Sections sec = sections(f.nblk, cur.n_nc, BYTES, B, 0);
    uint8_t* out = f.out;
    uint64_t* mid_status = f.enc_mid;
    // the tile's K bytes, codes and mu values from their first (the same in
    // every lane); rows index them with 32-bit offsets
    uint8_t* const kb_t = out + sec.kbytes + cur.r0;
    uint8_t* const cd_t = out + sec.codes + cur.r0 * (B / 4);
    T* const mus_t = reinterpret_cast<T*>(out + f.mu_off) + (uint64_t)t * G::TBLK;
    // Row by row: encode with error control (K0, then one more mantissa bit,
    // then raw; every lane votes, lanes without a coded block vote yes), codes
    // and byte counts, the row's offsets, K bytes and codes, and the staged
    // mid bytes, so that only one row's words are live at a time.
    uint32_t tile_bytes = 0;
#pragma unroll
    for (int s = 0; s < SUB; ++s) {
      if constexpr (sizeof(T) == 4) {
        // the flush's barrier orders the cleared words before this row's
        // stores
        if (pend && tile_bytes + (uint32_t)(G::TILE * BYTES) > RING - ((p_bytes + 15u) & ~15u)) flush(0);
      }
      U q[EPL];
      int K = cur.row.K(s);
      // a wave whose blocks of this row are all constant (or past the end)
      // stores nothing: it skips to the row's offset scan, which every wave
      // joins (the vote is wave-uniform, so the branch is too). Only the
      // 64-bit words pay enough per row for the skip to win; for float32 it
      // measured no faster and the branch is left out.
      const bool live = sizeof(T) == 4 || __ballot(K != 0) != 0;
      const int cnt_s = cur.row.cnt(s);
      bool raw = false;
      int nb = 0;
      uint32_t codes = 0, lb = 0;
      const bool coded = K > 0;
      // Without a short block (the last of a field) in the wave, no value
      // needs a validity test: constant and absent blocks encode as zero
      // words that keep nothing (K = 0: no kept bytes, no codes), raw blocks
      // keep every byte with code 0.
      const bool whole = __ballot(K != 0 && cnt_s != EPL) == 0;
      if (live) {
        bool ok = encode_try<T, EPL>(cur.x[s], coded ? cnt_s : 0, cur.mu[s], e, K, coded && cur.row.verify(s), q);
        if (!group_all<LPB>(ok)) {  // only coded blocks can fail
          const int K1 = kept_bits<T>(K - Traits<T>::KMIN + 1);
          bool ok1 = false;
          if (K1 != K) ok1 = encode_try<T, EPL>(cur.x[s], cnt_s, cur.mu[s], e, K1, true, q);
          K = group_all<LPB>(ok1) ? K1 : -1;
        }
        raw = K < 0;
        if (raw) {  // byte-swapped here, so that every string below is byte_swap(q) less its ci low bytes
#pragma unroll
          for (int i = 0; i < EPL; ++i) q[i] = byte_swap(bits_of(cur.x[s][i]));
        }
        nb = raw ? BYTES : (K > 0 ? bytes_of(K) : 0);
        U prev = lane_before<LPB, U>(q[EPL - 1]);
        prev = lig == 0 ? (U)0 : prev;
        // leading identical bytes capped at min(3, nb) (0 for raw blocks); a
        // zero difference counts all bytes, which the cap turns into the cap
        // as well. The cap is at most 24 bits, so a 64-bit word's high half
        // decides it.
        const uint32_t cap8 = raw ? 0u : 8u * (uint32_t)(nb < 3 ? nb : 3);
        auto code_of = [&](U z) -> uint32_t {
          const uint32_t lz = sizeof(U) == 8 ? lead_zero_bits((uint32_t)((uint64_t)z >> 32)) : lead_zero_bits(z);
          return (lz < cap8 ? lz : cap8) >> 3;
        };
        uint32_t csum = 0;
        if (whole) {
#pragma unroll
          for (int i = 0; i < EPL; ++i) {
            const uint32_t ci = code_of(q[i] ^ prev);
            codes |= ci << (2 * (EPL - 1 - i));
            csum += ci;
            prev = q[i];
          }
        } else {
#pragma unroll
          for (int i = 0; i < EPL; ++i) {
            const uint32_t ci = i < cnt_s ? code_of(q[i] ^ prev) : 0u;
            codes |= ci << (2 * (EPL - 1 - i));
            csum += ci;
            prev = q[i];
          }
        }
        // stored bytes of the lane: nb per valid value less the identical ones
        lb = (uint32_t)(nb * cnt_s) - csum;
      }
      uint32_t rtot;
      const uint32_t ex = wg_excl_sum<uint32_t>(lb, s_scan, rtot);
      // the ring from this tile's start up to the pending tile's must hold
      // the row (the condition is the same in every lane). For float64 rows
      // (16 KiB) the check takes the row's own size; float32 rows check
      // their largest size before the row, where the flush's code does not
      // meet the row's live registers (checked here, the float32 encoder
      // spilled).
      if constexpr (sizeof(T) == 8) {
        if (pend && tile_bytes + rtot > RING - ((p_bytes + 15u) & ~15u)) {
          flush(0);
          __syncthreads();  // the cleared words before this row's stores
        }
      }
      if (K != 0) {
        const uint32_t r = cur.row.rank(s);  // within the tile
        if (lig == 0) {
          kb_t[r] = raw ? kRawK : (uint8_t)K;
          if (coded && raw) mus_t[(uint32_t)(s * G::TB) + threadIdx.x / LPB] = (T)0;
        }
        uint8_t* cdst = cd_t + (r * (uint32_t)(B / 4) + (uint32_t)lig * (EPL / 4));
        if constexpr (EPL == 8) {
          const uint16_t wv = (uint16_t)(((codes >> 8) & 0xFFu) | ((codes & 0xFFu) << 8));
          *reinterpret_cast<uint16_t*>(cdst) = wv;
        } else {
#pragma unroll
          for (int j = 0; j < EPL / 4; ++j) cdst[j] = (uint8_t)(codes >> (8 * (EPL / 4 - 1 - j)));
        }
      }
      // stage the kept bytes of each value, most significant first: q holds
      // only its top nb bytes, so after the byte swap the value's string is
      // byte_swap(q) without its ci low bytes, zero bytes above it
      if (live) {
        LanePacker pk(s_stage, at + tile_bytes + ex, RING - 1);
        if (whole) {
#pragma unroll
          for (int i = 0; i < EPL; ++i) {
            const int ci = (int)((codes >> (2 * (EPL - 1 - i))) & 3u);
            pk.put(drop_low_bytes(byte_swap(q[i]), (uint32_t)ci), nb - ci);
          }
        } else {
#pragma unroll
          for (int i = 0; i < EPL; ++i) {
            const int ci = (int)((codes >> (2 * (EPL - 1 - i))) & 3u);
            const bool valid = i < cnt_s;
            const U sv = valid ? drop_low_bytes(byte_swap(q[i]), (uint32_t)ci) : (U)0;
            pk.put(sv, valid ? nb - ci : 0);
          }
        }
        pk.flush();
      }
      tile_bytes += rtot;
    }
    if (threadIdx.x == 0) lookback_publish(mid_status, t, tile_bytes);
    const uint32_t f_cur = cur.field;

    // the next tile's loads go out while the pending tile's offset is
    // resolved. A single call reads the pending tile's offset word before
    // them: vector loads return in order, so a read issued after the tile's
    // loads would wait for all of them
    gt = claim();  // its barriers also order the staging before the copy-out
    const bool more = gt < ntiles;
    uint64_t first_poll = 0;
    if constexpr (BATCH == kSingle) {
      if (pend && threadIdx.x == 0) first_poll = status_load(field_at<BATCH>(b, p_field).enc_mid + p_tile);
    } else {  // a batch: the predecessor's word, for the look-back's shortcut
      if (pend && threadIdx.x == 0 && p_tile > 0)
        first_poll = status_load(field_at<BATCH>(b, p_field).enc_mid + p_tile - 1);
    }
    if (more) load(cur, gt);
    if (pend) flush(first_poll);
    pend = true;
    p_tile = t;
    p_field = f_cur;
    p_bytes = tile_bytes;
    p_at = at;
    at = (at + ((tile_bytes + 15u) & ~15u)) & (RING - 1);
    if (!more) break;
  }
  flush(0);
  if constexpr (BATCH == kSingle) {
    if (threadIdx.x == 0 && *s_end != ~0ull) {
      const FieldC f = field_at<BATCH>(b, 0);
      finish_stream(f, sections(f.nblk, f.ctr->n_nc, BYTES, B, 0).mid, *s_end);
    }
  }
}

template <typename T, int B, int BATCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Geo<T, B>::ENC_WAVES))) void k_encode(
    CBatch b) {
  using G = Geo<T, B>;
  __shared__ uint32_t s_scan[G::SUB * kWavesPerWG];
  __shared__ uint32_t s_tile;
  __shared__ uint64_t s_base, s_end;
  __shared__ __align__(16) uint32_t s_stage[enc_ring_bytes<T, B>() / 4];
  encode_pass<T, B, BATCH>(b, s_scan, &s_tile, &s_base, &s_end, s_stage);
}

// --------------------------------------------------------------- finalize ---

// The finishing pass of a batch, one workgroup a field (a single call
// finishes its stream in the encode pass and needs this pass only when it has
// no values): a field with values gets its mid-byte total and stream size;
// a field without values has no extrema, classification or encode tiles and
// gets its whole header (the bound from an empty range) and size.
__global__ void k_finalize(CBatch b) {
  const FieldC f = field_at(b, blockIdx.x);
  if (f.nblk != 0) {
    if (threadIdx.x == 0) {
      const uint32_t w = f.dtype == 0 ? 4 : 8;
      finish_stream(f, sections(f.nblk, f.ctr->n_nc, w, f.b, 0).mid, f.ctr->mid_total);
    }
    return;
  }
  const int rel = f.eb_mode == 1;
  const uint64_t e_bits = f.dtype == 0 ? (uint64_t)bits_of(bound_from<float>(rel, f.eb, ~0ull, 0ull))
                                       : (uint64_t)bits_of(bound_from<double>(rel, f.eb, ~0ull, 0ull));
  const uint64_t total = write_stream_header(f, e_bits, 0, 0);
  if (threadIdx.x == 0) *f.out_size = total;
}

// ---------------------------------------------------------------- launch ---

template <int B>
hipError_t launch_compress_b(const CBatch& b, const CLaunchGeom& g, hipStream_t stream, TimerHook hook) {
  auto run = [&](const char* name, auto&& fn) {
    if (hook) hook(name, stream, 1);
    fn();
    if (hook) hook(name, stream, 0);
  };
  if (b.tiles_stats[0] + b.tiles_stats[1] > 0) {
    if (b.tiles_stats[0]) run("k_stats", [&] { k_stats<float, B><<<(uint32_t)b.tiles_stats[0], 256, 0, stream>>>(b); });
    if (b.tiles_stats[1]) run("k_stats", [&] { k_stats<double, B><<<(uint32_t)b.tiles_stats[1], 256, 0, stream>>>(b); });
    if (b.tiles_cls[0]) run("k_classify", [&] { k_classify<float, B><<<(uint32_t)b.tiles_cls[0], 256, 0, stream>>>(b); });
    if (b.tiles_cls[1]) run("k_classify", [&] { k_classify<double, B><<<(uint32_t)b.tiles_cls[1], 256, 0, stream>>>(b); });
    for (int dt = 0; dt < 2; ++dt) {
      if (!b.tiles_enc[dt]) continue;
      // at least one workgroup per ticket class: tiles of a class without one
      // would never be encoded (and every later tile would wait for them)
      const uint64_t want = std::max<uint64_t>(g.encode_wgs[dt], kTicketClasses);
      const uint32_t genc = (uint32_t)std::min<uint64_t>(b.tiles_enc[dt], want);
      const bool batch = b.fields != nullptr;
      // a single call adds workgroup 0, its scan wave
      if (dt == 0 && !batch)
        run("k_encode", [&] { k_encode<float, B, kSingle><<<genc + 1, 256, 0, stream>>>(b); });
      else if (dt == 0)
        run("k_encode", [&] { k_encode<float, B, kBatch><<<genc, 256, 0, stream>>>(b); });
      else if (!batch)
        run("k_encode", [&] { k_encode<double, B, kSingle><<<genc + 1, 256, 0, stream>>>(b); });
      else
        run("k_encode", [&] { k_encode<double, B, kBatch><<<genc, 256, 0, stream>>>(b); });
    }
  }
  // batches finish their streams here; a single call only without values
  if (b.fields != nullptr || b.any_empty) run("k_finalize", [&] { k_finalize<<<b.nfields, 64, 0, stream>>>(b); });
  return hipGetLastError();
}

hipError_t launch_compress(const CBatch& b, uint32_t block, const CLaunchGeom& g, hipStream_t stream,
                           TimerHook hook) {
  switch (block) {
    case 8: return launch_compress_b<8>(b, g, stream, hook);
    case 16: return launch_compress_b<16>(b, g, stream, hook);
    case 32: return launch_compress_b<32>(b, g, stream, hook);
    case 64: return launch_compress_b<64>(b, g, stream, hook);
    case 128: return launch_compress_b<128>(b, g, stream, hook);
    case 256: return launch_compress_b<256>(b, g, stream, hook);
    case 512: return launch_compress_b<512>(b, g, stream, hook);
    case 1024: return launch_compress_b<1024>(b, g, stream, hook);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace szx
