// szx_device.hpp -- device-side building blocks of the SZx kernels for gfx950.
//
// Element traits, IEEE-754 totalOrder keys, the exact "a - c <= e" decision,
// the bit budget of eq. (4) with the byte shift of eq. (5), wave/group scans,
// the workgroup-wide scan, and the decoupled look-back that chains tiles of a
// single-pass device-wide prefix sum (Sec. V-B: the output offset of each
// block is the prefix sum of the bytes of the blocks before it).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "szx_layout.hpp"

namespace szx {

// A pointer read from a field descriptor in memory is typed generic, so every
// access through it would compile to flat instructions (which wait on both
// the vector-memory and the LDS counters). Descriptors only hold device
// memory: re-read the pointer's bits as a global-memory pointer, so that the
// compiler infers global accesses through it.
template <typename P>
__device__ __forceinline__ P as_global(const P& member) {
  const uint64_t raw = *reinterpret_cast<const uint64_t*>(&member);
  return (P)(__attribute__((address_space(1))) char*)raw;
}

constexpr int kWave = 64;
constexpr int kWG = 256;
constexpr int kWavesPerWG = kWG / kWave;
constexpr uint32_t kHeaderBytes = 96;
constexpr uint32_t kMagic = 0x4D585A53u;  // "SZXM" little-endian
constexpr uint8_t kVersion = 1;
constexpr uint8_t kRawK = 0xFF;

template <typename T>
struct Traits;

template <>
struct Traits<float> {
  using U = uint32_t;
  static constexpr int W = 32;     // bits per value
  static constexpr int E = 8;      // exponent bits
  static constexpr int BIAS = 127;
  static constexpr int BYTES = 4;
  static constexpr int KMIN = 1 + E;
};

template <>
struct Traits<double> {
  using U = uint64_t;
  static constexpr int W = 64;
  static constexpr int E = 11;
  static constexpr int BIAS = 1023;
  static constexpr int BYTES = 8;
  static constexpr int KMIN = 1 + E;
};

// Launch geometry that depends only on the block size b: each lane owns EPL
// consecutive values, LPB lanes share one block, a 256-thread workgroup tile
// holds TB whole blocks. It changes no output byte.
// A tile is SUB such rows of TB blocks: about TARGET bytes of input (and at
// least 8 blocks, so that a tile owns whole bytes of the state bits). The
// encoder's tiles are large, so that the per-tile costs of its prefix sums
// are rare; the decoder's are half that size, so that more workgroups fit a
// compute unit (its tiles wait on nothing).
constexpr int geo_sub(int tile_bytes, int tb, int target) {
  int s = target / tile_bytes;
  s = s < 1 ? 1 : s;
  while (tb * s < 8) s *= 2;
  return s;
}

template <typename T, int B, int TARGET = (int)kEncodeTileBytes>
struct Geo {
  static constexpr int EPL = B >= 512 ? B / 64 : 8;
  static constexpr int LPB = B / EPL;  // 1..64, divides 64
  static constexpr int TB = kWG / LPB;
  static constexpr int TILE = TB * B;  // values per row
  static constexpr int SUB = geo_sub(TILE * (int)sizeof(T), TB, TARGET);
  static constexpr int TBLK = TB * SUB;  // blocks per tile
  // waves per SIMD the encoder is held to (its LDS stage holds a tile's
  // output: 4 workgroups of a 32 KiB stage fit the 160 KiB of LDS, one of a
  // 64 KiB stage leaves room for 2)
  static constexpr int ENC_WAVES = TILE * SUB * (int)sizeof(T) > 40000 ? 2 : 4;
  static_assert(LPB >= 1 && LPB <= 64 && (64 % LPB) == 0, "group must fit a wave");
  static_assert(TBLK % 8 == 0, "a tile owns whole state bytes");
};

// Decoder tiles (each a whole number of them per encode tile).
template <typename T, int B>
using GeoD = Geo<T, B, (int)kDecodeTileBytes>;

__device__ __forceinline__ uint32_t bits_of(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint64_t bits_of(double v) { return (uint64_t)__double_as_longlong(v); }
__device__ __forceinline__ float float_from(uint32_t u) { return __uint_as_float(u); }
__device__ __forceinline__ double double_from(uint64_t u) { return __longlong_as_double((long long)u); }

template <typename T>
__device__ __forceinline__ T from_bits(typename Traits<T>::U u);
template <>
__device__ __forceinline__ float from_bits<float>(uint32_t u) { return float_from(u); }
template <>
__device__ __forceinline__ double from_bits<double>(uint64_t u) { return double_from(u); }

// Unsigned key whose order is IEEE-754 totalOrder (-0 < +0): flip all bits of
// negatives, set the sign bit of non-negatives.
template <typename U>
__device__ __forceinline__ U order_key(U u) {
  constexpr U sign = (U)1 << (sizeof(U) * 8 - 1);
  return (u & sign) ? (U)~u : (U)(u | sign);
}
template <typename U>
__device__ __forceinline__ U key_to_bits(U k) {
  constexpr U sign = (U)1 << (sizeof(U) * 8 - 1);
  return (k & sign) ? (U)(k & ~sign) : (U)~k;
}

// Keys of -max finite and +max finite: a block is all-finite iff its key range
// lies inside [kLo, kHi].
template <typename T>
struct FiniteKeys {
  using U = typename Traits<T>::U;
  static constexpr U EXPMASK = (((U)1 << Traits<T>::E) - 1) << (Traits<T>::W - 1 - Traits<T>::E);
  static constexpr U SIGN = (U)1 << (Traits<T>::W - 1);
  static constexpr U MAXF = EXPMASK - 1;          // largest finite magnitude pattern
  static constexpr U HI = MAXF | SIGN;            // key of +max
  static constexpr U LO = (U)~(MAXF | SIGN);      // key of -max
};

template <typename T>
__device__ __forceinline__ bool is_finite_bits(typename Traits<T>::U u) {
  return (u & FiniteKeys<T>::EXPMASK) != FiniteKeys<T>::EXPMASK;
}

// Exact decision of (a - c) <= e for finite a, c, e whose difference does not
// overflow. s = fl(a - c) lies on the same side of e as the exact difference
// whenever s != e (rounding is monotone); when s == e the rounding error,
// recovered exactly by Knuth's TwoSum, decides.
template <typename T>
__device__ __forceinline__ bool exact_le(T a, T c, T e) {
  const T nb = -c;
  const T s = a + nb;
  if (s < e) return true;
  if (s > e) return false;
  const T bv = s - a;
  const T av = s - bv;
  const T t = (a - av) + (nb - bv);
  return t <= (T)0;
}

// p(y) of eq. (4): unbiased exponent of |y|, with zero and subnormals at the
// smallest normal exponent.
template <typename T>
__device__ __forceinline__ int exp_of(T y) {
  using U = typename Traits<T>::U;
  const U u = bits_of(y);
  int f = (int)((u >> (Traits<T>::W - 1 - Traits<T>::E)) & ((1u << Traits<T>::E) - 1));
  f = f < 1 ? 1 : f;
  return f - Traits<T>::BIAS;
}

// Largest T value <= ed, for ed >= 0 (possibly +inf).
template <typename T>
__device__ __forceinline__ T round_down_to(double ed);
template <>
__device__ __forceinline__ float round_down_to<float>(double ed) {
  if (!(ed > 0.0)) return 0.0f;
  if (__builtin_isinf(ed)) return 3.40282346638528859812e+38f;
  float f = __double2float_rn(ed);
  if (__builtin_isinf(f)) return 3.40282346638528859812e+38f;
  while ((double)f > ed) f = __uint_as_float(__float_as_uint(f) - 1u);
  return f;
}
template <>
__device__ __forceinline__ double round_down_to<double>(double ed) {
  if (!(ed > 0.0)) return 0.0;
  if (__builtin_isinf(ed)) return 1.79769313486231570815e+308;
  return ed;
}

// Bound e from the parameters and, for REL, the global finite range (keys;
// lo > hi means no finite value was seen).
template <typename T>
__device__ __forceinline__ T bound_from(int rel, double eb, uint64_t klo, uint64_t khi) {
  using U = typename Traits<T>::U;
  double ed;
  if (!rel) {
    ed = eb;
  } else if (klo > khi || eb == 0.0) {
    ed = 0.0;
  } else {
    const T gmin = from_bits<T>(key_to_bits<U>((U)klo));
    const T gmax = from_bits<T>(key_to_bits<U>((U)khi));
    const double range = (double)gmax - (double)gmin;
    ed = eb * range;
  }
  return round_down_to<T>(ed);
}

// Kept leading bits K = min(W, 1 + E + m) (eq. (4) read as a count of kept
// bits: sign, exponent and m mantissa bits), its right shift s (eq. (5)) and
// the number of whole bytes nb = (K + s) / 8.
__device__ __forceinline__ int shift_of(int K) { return (8 - (K & 7)) & 7; }
__device__ __forceinline__ int bytes_of(int K) { return (K + shift_of(K)) >> 3; }

template <typename T>
__device__ __forceinline__ int kept_bits(int m) {
  const int k = 1 + Traits<T>::E + m;
  return k > Traits<T>::W ? Traits<T>::W : k;
}

// Mid-range and constant test of one block from its totalOrder extrema.
// Returns true for a constant block. m0 receives the mantissa budget of eq. (4)
// for a non-constant one.
template <typename T>
__device__ __forceinline__ bool classify_block(T mn, T mx, T e, T& mu, int& m0) {
  mu = (T)0.5 * mn + (T)0.5 * mx;
  if (exact_le<T>(mx, mu, e) && exact_le<T>(mu, mn, e)) {
    m0 = 0;
    return true;
  }
  T r1 = mx - mu;
  T r2 = mn - mu;
  r1 = r1 < (T)0 ? -r1 : r1;
  r2 = r2 < (T)0 ? -r2 : r2;
  const T r = r1 > r2 ? r1 : r2;
  const int m = exp_of<T>(r) - exp_of<T>(e);
  m0 = m < 0 ? 0 : m;
  return false;
}

// Mask of the top nb bytes of a word.
template <typename U>
__device__ __forceinline__ U top_bytes_mask(int nb) {
  constexpr int W = sizeof(U) * 8;
  return nb >= W / 8 ? (U)~(U)0 : (nb <= 0 ? (U)0 : (U) ~(((U)1 << (W - 8 * nb)) - 1));
}


// Leading zero bits of z; any value >= the width for z = 0 (callers cap it).
__device__ __forceinline__ uint32_t lead_zero_bits(uint32_t z) { return (uint32_t)__clz((int)z); }
__device__ __forceinline__ uint32_t lead_zero_bits(uint64_t z) { return (uint32_t)__clzll((long long)z); }

__device__ __forceinline__ uint32_t byte_swap(uint32_t v) { return __builtin_bswap32(v); }
__device__ __forceinline__ uint64_t byte_swap(uint64_t v) { return __builtin_bswap64(v); }

// ---------------------------------------------------------------- scans ----

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Inclusive sum of 32-bit values over the 64 lanes of a wave with DPP: row
// shifts by 1, 2, 4, 8 within each row of 16 lanes, then the last lane of
// rows 0 and 2 added to rows 1 and 3 (row_bcast:15) and the last lane of row 1
// to rows 2 and 3 (row_bcast:31). Lanes without a source add 0. No LDS.
__device__ __forceinline__ uint32_t wave_incl_sum_u32(uint32_t v) {
  int x = (int)v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return (uint32_t)x;
}

// Lane i - d within each row of 16 lanes (row_shr:d, d in {1, 2, 4, 8});
// the first d lanes of a row get 0.
__device__ __forceinline__ uint32_t dpp_shr(int d, uint32_t v) {
  switch (d) {
    case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
    case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);
    case 4: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
    default: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);
  }
}

// The value of the previous lane within groups of G <= 16 lanes (row_shr:1;
// the first lane of each row of 16 gets 0, other group starts get their
// neighbour, which callers replace).
__device__ __forceinline__ uint32_t lane_before_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
}
template <int G, typename U>
__device__ __forceinline__ U lane_before(U v) {
  if constexpr (G <= 16) {
    if constexpr (sizeof(U) == 4) {
      return (U)lane_before_u32((uint32_t)v);
    } else {
      const uint32_t lo = lane_before_u32((uint32_t)v);
      const uint32_t hi = lane_before_u32((uint32_t)(v >> 32));
      return ((U)hi << 32) | lo;
    }
  } else {
    return __shfl_up(v, 1, G);
  }
}

// Inclusive sum over groups of G consecutive lanes (G a power of two <= 64).
template <int G, typename V>
__device__ __forceinline__ V group_incl_sum(V v) {
  if constexpr (G == 64 && sizeof(V) == 4) return (V)wave_incl_sum_u32((uint32_t)v);
  const int lg = lane_id() & (G - 1);
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    const V t = __shfl_up(v, d, G);
    if (lg >= d) v += t;
  }
  return v;
}

// Minimum and maximum over groups of G consecutive lanes (all lanes of a
// group end with the group's value).
template <int G, typename U>
__device__ __forceinline__ U group_min(U v) {
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    const U o = __shfl_xor(v, d, G);
    v = o < v ? o : v;
  }
  return v;
}
template <int G, typename U>
__device__ __forceinline__ U group_max(U v) {
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    const U o = __shfl_xor(v, d, G);
    v = o > v ? o : v;
  }
  return v;
}

template <int G, typename V>
__device__ __forceinline__ V group_sum(V v) {
#pragma unroll
  for (int d = 1; d < G; d <<= 1) v += __shfl_xor(v, d, G);
  return v;
}

template <int G>
__device__ __forceinline__ bool group_all(bool p) {
  const uint64_t m = __ballot(p);
  if (G == 64) return m == ~0ull;
  const int base = lane_id() & ~(G - 1);
  const uint64_t gm = ((G == 64) ? ~0ull : ((1ull << G) - 1)) << base;
  return (m & gm) == gm;
}

// Exclusive prefix sum over the 256 threads of a workgroup (thread order).
// `scratch` holds kWavesPerWG entries. Returns the exclusive prefix; `total`
// receives the workgroup total. Contains barriers: call from all threads.
template <typename V>
__device__ __forceinline__ V wg_excl_sum(V v, V* scratch, V& total) {
  const V inc = group_incl_sum<kWave, V>(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) scratch[w] = inc;
  __syncthreads();
  V before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kWavesPerWG; ++i) {
    const V s = scratch[i];
    before += (i < w) ? s : (V)0;
    all += s;
  }
  __syncthreads();
  total = all;
  return before + inc - v;
}

// S exclusive prefix sums over the 256 threads at once, laid end to end: the
// prefix of value s of a thread counts all values s' < s of every thread, then
// value s of the threads before it. tot[s] receives the total of value s.
// `scratch` holds S * kWavesPerWG entries. Contains barriers.
template <int S>
__device__ __forceinline__ void wg_excl_scan_multi(const uint32_t (&v)[S], uint32_t (&excl)[S],
                                                   uint32_t (&tot)[S], uint32_t* scratch) {
  uint32_t inc[S];
#pragma unroll
  for (int s = 0; s < S; ++s) inc[s] = group_incl_sum<kWave, uint32_t>(v[s]);
  const int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) {
#pragma unroll
    for (int s = 0; s < S; ++s) scratch[s * kWavesPerWG + w] = inc[s];
  }
  __syncthreads();
  uint32_t running = 0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerWG; ++i) {
      const uint32_t x = scratch[s * kWavesPerWG + i];
      before += (i < w) ? x : 0u;
      all += x;
    }
    excl[s] = running + before + inc[s] - v[s];
    tot[s] = all;
    running += all;
  }
  __syncthreads();
}

// ------------------------------------------------------ decoupled look-back -

// A tile's status word: flag in the top two bits (0 = not yet published,
// 1 = aggregate of the tile alone, 2 = inclusive prefix), value below.
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagIncl = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 18;

// The flag and the value share one 64-bit word, so a reader never needs any
// other memory of the writer: relaxed device-scope atomics are enough. (An
// acquire/release pair would add a write-back or an invalidation of the L2 of
// the XCD at every publish and every poll.)
// Status words live in device memory: the accesses are typed global, so that
// a look-back compiled out of line (its pointer generic) does not poll with
// flat instructions.
typedef __attribute__((address_space(1))) uint64_t global_u64;
__device__ __forceinline__ void status_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store((global_u64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t status_load(const uint64_t* p) {
  return __hip_atomic_load((global_u64*)const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-wide exclusive prefix sums over tiles (decoupled look-back). A tile
// first publishes its own aggregate, then resolves its exclusive prefix from
// its predecessors' words and publishes its inclusive prefix. A tile waits
// only on lower-numbered tiles; every tile is taken by a running workgroup
// in increasing order within its ticket class and publishes its aggregate
// before it waits on anything, so every wait ends. Waits are bounded all the
// same: on exhaustion err is raised to err_code and the partial prefix is
// returned.
__device__ __forceinline__ void lookback_publish(uint64_t* status, uint32_t t, uint64_t agg) {
  status_store(status + t, (t == 0 ? kFlagIncl : kFlagAgg) | (agg & kValueMask));
}

// Called by all 64 lanes of one wave after lookback_publish; returns the same
// exclusive prefix in every lane.
template <int R = 4>  // status words per lane per round: a window of 64 R tiles
__device__ __noinline__ uint64_t lookback_resolve(uint64_t* status, uint32_t t, uint64_t agg,
                                                  uint32_t* err, uint32_t err_code) {
  const int lane = lane_id();
  if (t == 0) return 0;
  uint64_t excl = 0;
  int64_t base = (int64_t)t - 1;
  uint32_t spins = 0;
  for (;;) {
    uint64_t w[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int64_t j = base - (k * kWave + lane);
      w[k] = j >= 0 ? status_load(status + j) : (kFlagIncl | 0ull);
    }
    bool done = false, retry = false;
    int consumed = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if (done || retry) continue;
      const uint64_t flag = w[k] >> 62;
      const uint64_t incl = __ballot(flag == 2);
      const uint64_t inval = __ballot(flag == 0);
      const int first = incl ? (int)__ffsll((long long)incl) - 1 : 64;
      const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1);
      if (inval & need) {
        retry = true;
        continue;
      }
      uint64_t v = lane <= first ? (w[k] & kValueMask) : 0ull;
      excl += group_sum<kWave, uint64_t>(v);
      if (first < 64)
        done = true;
      else
        ++consumed;
    }
    if (done) break;
    base -= (int64_t)consumed * kWave;
    if (retry) {
      if (++spins > kSpinLimit) {
        if (lane == 0) atomicMax(err, err_code);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  if (lane == 0) status_store(status + t, kFlagIncl | ((excl + agg) & kValueMask));
  return excl;
}

// Prefix sums over tiles kept by one scan wave, for a pass whose tiles are
// many and in flight all at once: the tiles only publish their aggregates;
// the scan wave reads them in tile order, 64 R words a round, and publishes
// every tile's inclusive prefix as soon as all earlier tiles have published,
// so a tile's own wait is one status word. (A decoupled look-back walks back
// through every tile still in flight, one window per round and per tile.)
// The scan wave waits only on tiles that running workgroups hold, and its
// waits are bounded like the others: on exhaustion err is raised and it
// stops, and the tiles still waiting give up on their own bounds.
template <int R>
__device__ __noinline__ void scan_wave(uint64_t* status, uint64_t ntiles, uint32_t* err, uint32_t err_code) {
  const int lane = lane_id();
  uint64_t first = 0, run = 0;
  uint32_t spins = 0;
  while (first < ntiles) {
    uint64_t w[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint64_t j = first + (uint64_t)(k * kWave + lane);
      w[k] = j < ntiles ? status_load(status + j) : 0ull;
    }
    uint64_t adv = 0;
    bool stop = false;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if (stop) continue;
      // the published words from the window's start, consecutively
      const uint64_t pub = __ballot((w[k] >> 62) != 0);
      const int c = pub == ~0ull ? 64 : (int)__ffsll((long long)~pub) - 1;
      const uint64_t v = lane < c ? (w[k] & kValueMask) : 0ull;
      const uint64_t incl = run + group_incl_sum<kWave, uint64_t>(v);
      if (lane < c) status_store(status + first + adv + lane, kFlagIncl | (incl & kValueMask));
      run = __shfl(incl, 63);
      adv += (uint64_t)c;
      stop = c < 64;
    }
    first += adv;
    if (adv == 0) {
      if (++spins > kSpinLimit) {
        if (lane == 0) atomicMax(err, err_code);
        return;
      }
      __builtin_amdgcn_s_sleep(2);
    } else {
      spins = 0;
    }
  }
}

// A tile's exclusive prefix once the scan wave has published its inclusive
// one (one lane polls; the value is the inclusive prefix less the tile's own
// aggregate). Bounded: on exhaustion err is raised and 0 is returned.
__device__ __forceinline__ uint64_t scan_wait(const uint64_t* status, uint32_t t, uint64_t agg, uint32_t* err,
                                              uint32_t err_code, uint64_t first = 0) {
  // `first`: the word as read earlier by the caller (0: not read)
  if ((first >> 62) == 2) return ((first & kValueMask) - agg) & kValueMask;
  uint32_t spins = 0;
  for (;;) {
    const uint64_t w = status_load(status + t);
    if ((w >> 62) == 2) return ((w & kValueMask) - agg) & kValueMask;
    if (++spins > kSpinLimit) {
      atomicMax(err, err_code);
      return 0;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// The look-back with its window sized to the tiles of the scan: every status
// load is a transaction at the device's coherence point, so where many tiles
// are in flight a window of 64 (one word per lane) costs less than fewer,
// wider rounds; where few are, a window of 256 covers them in one round.
__device__ __forceinline__ uint64_t lookback_resolve_n(uint64_t* status, uint32_t t, uint64_t agg, uint32_t* err,
                                                       uint32_t err_code, uint64_t ntiles) {
  return ntiles > 512 ? lookback_resolve<1>(status, t, agg, err, err_code)
                      : lookback_resolve<4>(status, t, agg, err, err_code);
}

}  // namespace szx
