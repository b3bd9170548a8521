// szx_compress.hip -- compression kernels of the SZx method for gfx950.
//
// Pipeline of one sz_compress call (all on the caller's stream):
//   k_init      clear counters and the tile status words of the scans
//   k_stats     per-block totalOrder min/max (Alg. 1 "compute mu_k" needs both)
//               and, for the relative bound, the global finite range
//   k_classify  bound e, mid-range mu and constant test per block (Alg. 1),
//               state bits and mu section, list of non-constant blocks through
//               a single-pass prefix count
//   k_encode    per non-constant block: normalise, keep K bits (eq. (4)),
//               shift (eq. (5)), verify the bound, 2-bit leading-byte codes and
//               mid bytes; the tile's output offset comes from a single-pass
//               prefix sum over tiles (Sec. V-B); bytes are packed in LDS and
//               leave in aligned 16-byte stores
//   k_finalize  header, section padding, stream size
#include <algorithm>

#include "szx_device.hpp"
#include "szx_launch.hpp"

namespace szx {

// ------------------------------------------------------------------ init ---

__global__ __launch_bounds__(256) void k_init(Counters* ctr, uint64_t* st1, uint64_t n1,
                                              uint64_t* st2, uint64_t n2, uint32_t* status) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1 + n2; i += stride) {
    if (i < n1)
      st1[i] = 0;
    else
      st2[i - n1] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctr->err = 0;
    ctr->klo = ~0ull;
    ctr->khi = 0;
    ctr->n_nc = 0;
    ctr->mid_total = 0;
    ctr->e_bits = 0;
    if (status) *status = 0;
  }
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

// ----------------------------------------------------------------- stats ---

// Per-block totalOrder extrema (as keys) of all values, and per workgroup the
// finite range (keys; lo > hi when the workgroup saw no finite value) into
// part[2 * blockIdx.x], part[2 * blockIdx.x + 1]. Two tiles per iteration keep
// more loads in flight.
template <typename T, int B>
__device__ __forceinline__ void stats_tile(const T (&v)[Geo<T, B>::EPL], int cnt, uint64_t i0, uint64_t nblk,
                                           typename Traits<T>::U* __restrict__ stats,
                                           typename Traits<T>::U& flo, typename Traits<T>::U& fhi) {
  using U = typename Traits<T>::U;
  constexpr int EPL = Geo<T, B>::EPL, LPB = Geo<T, B>::LPB;
  U kmin = (U)~(U)0, kmax = 0;
#pragma unroll
  for (int i = 0; i < EPL; ++i) {
    const U u = bits_of(v[i]);
    const U k = order_key<U>(u);
    const bool ok = i < cnt;
    kmin = (ok && k < kmin) ? k : kmin;
    kmax = (ok && k > kmax) ? k : kmax;
    const bool fin = ok && is_finite_bits<T>(u);
    flo = (fin && k < flo) ? k : flo;
    fhi = (fin && k > fhi) ? k : fhi;
  }
  kmin = group_min<LPB, U>(kmin);
  kmax = group_max<LPB, U>(kmax);
  const uint64_t blk = i0 / B;
  if ((threadIdx.x % LPB) == 0 && blk < nblk) {
    stats[2 * blk] = kmin;
    stats[2 * blk + 1] = kmax;
  }
}

template <typename T, int B>
__global__ __launch_bounds__(256) void k_stats(const T* __restrict__ x, uint64_t n, uint64_t nblk,
                                               typename Traits<T>::U* __restrict__ stats,
                                               uint64_t* __restrict__ part) {
  using U = typename Traits<T>::U;
  using G = Geo<T, B>;
  constexpr int EPL = G::EPL;
  __shared__ U s_lo[kWavesPerWG], s_hi[kWavesPerWG];
  U flo = (U)~(U)0, fhi = 0;
  const uint64_t ntile = cdiv(n, (uint64_t)G::TILE);
  const uint64_t step = gridDim.x;
  for (uint64_t t = blockIdx.x; t < ntile; t += 2 * step) {
    const uint64_t i0 = t * G::TILE + (uint64_t)threadIdx.x * EPL;
    const uint64_t i1 = i0 + step * G::TILE;
    const bool second = t + step < ntile;
    T v0[EPL], v1[EPL];
    const int c0 = load_run<T, EPL>(x, i0, n, v0);
    const int c1 = second ? load_run<T, EPL>(x, i1, n, v1) : 0;
    stats_tile<T, B>(v0, c0, i0, nblk, stats, flo, fhi);
    if (second) stats_tile<T, B>(v1, c1, i1, nblk, stats, flo, fhi);
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
    U lo = s_lo[0], hi = s_hi[0];
    for (int i = 1; i < kWavesPerWG; ++i) {
      lo = s_lo[i] < lo ? s_lo[i] : lo;
      hi = s_hi[i] > hi ? s_hi[i] : hi;
    }
    // widen to 64 bits keeping "no finite value" as lo > hi
    part[2 * blockIdx.x] = lo > hi ? ~0ull : (uint64_t)lo;
    part[2 * blockIdx.x + 1] = lo > hi ? 0ull : (uint64_t)hi;
  }
}

// -------------------------------------------------------------- classify ---

template <typename T>
__global__ __launch_bounds__(256) void k_classify(const typename Traits<T>::U* __restrict__ stats,
                                                  uint8_t* __restrict__ out, uint32_t* __restrict__ rec,
                                                  uint64_t* cls_status, Counters* ctr, uint64_t nblk,
                                                  uint64_t mu_off, int rel, double eb,
                                                  const uint64_t* __restrict__ part, uint32_t nparts) {
  using U = typename Traits<T>::U;
  __shared__ uint32_t s_scan[kWavesPerWG];
  __shared__ uint64_t s_base;
  __shared__ uint64_t s_lo[kWavesPerWG], s_hi[kWavesPerWG];
  // global finite range from the per-workgroup partials of k_stats
  uint64_t lo = ~0ull, hi = 0;
  if (rel) {
    for (uint32_t i = threadIdx.x; i < nparts; i += kWG) {
      const uint64_t a = part[2 * i], b = part[2 * i + 1];
      lo = a < lo ? a : lo;
      hi = b > hi ? b : hi;
    }
    lo = group_min<kWave, uint64_t>(lo);
    hi = group_max<kWave, uint64_t>(hi);
    if (lane_id() == 0) {
      s_lo[threadIdx.x / kWave] = lo;
      s_hi[threadIdx.x / kWave] = hi;
    }
    __syncthreads();
    lo = s_lo[0];
    hi = s_hi[0];
    for (int i = 1; i < kWavesPerWG; ++i) {
      lo = s_lo[i] < lo ? s_lo[i] : lo;
      hi = s_hi[i] > hi ? s_hi[i] : hi;
    }
  }
  const T e = bound_from<T>(rel, eb, lo, hi);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctr->klo = lo;
    ctr->khi = hi;
    ctr->e_bits = (uint64_t)bits_of(e);
  }
  const uint32_t ntiles = (uint32_t)cdiv(nblk, kClsTile);
  T* mus = reinterpret_cast<T*>(out + mu_off);
  {
    const uint32_t t = blockIdx.x;
    const uint64_t k = (uint64_t)t * kClsTile + threadIdx.x;
    bool nc = false;
    if (k < nblk) {
      const U kmin = stats[2 * k], kmax = stats[2 * k + 1];
      T mu = (T)0;
      if (kmin < FiniteKeys<T>::LO || kmax > FiniteKeys<T>::HI) {
        nc = true;  // a non-finite value: the block is stored raw, mu = +0
      } else {
        const T mn = from_bits<T>(key_to_bits<U>(kmin));
        const T mx = from_bits<T>(key_to_bits<U>(kmax));
        int m0;
        nc = !classify_block<T>(mn, mx, e, mu, m0);
      }
      mus[k] = mu;
    }
    // state bits: one 64-bit word per wave, written when it covers a block
    const uint64_t word = __ballot(nc);
    const uint64_t first = (uint64_t)t * kClsTile + (threadIdx.x & ~63u);
    if (lane_id() == 0 && first < nblk)
      *reinterpret_cast<uint64_t*>(out + 96 + first / 8) = word;
    uint32_t total;
    const uint32_t ex = wg_excl_sum<uint32_t>(nc ? 1u : 0u, s_scan, total);
    if (threadIdx.x < kWave) {
      const uint64_t p = lookback_excl(cls_status, t, total, &ctr->err, 1u);
      if (threadIdx.x == 0) s_base = p;
    }
    __syncthreads();
    const uint64_t base = s_base;
    if (nc) rec[base + ex] = (uint32_t)k;
    if (t == ntiles - 1 && threadIdx.x == 0) ctr->n_nc = base + total;
  }
}

// ---------------------------------------------------------------- encode ---

// Truncate v = x - mu to K leading bits, shifted right by s into nb whole
// bytes, and check that every valid value reconstructs within e exactly.
template <typename T, int EPL>
__device__ __forceinline__ bool encode_try(const T (&x)[EPL], int cnt, T mu, T e, int K,
                                           typename Traits<T>::U (&q)[EPL]) {
  using U = typename Traits<T>::U;
  const int s = shift_of(K);
  const U keep = top_bytes_mask<U>(bytes_of(K));
  bool ok = true;
#pragma unroll
  for (int i = 0; i < EPL; ++i) {
    const T v = x[i] - mu;
    const U qi = (U)(bits_of(v) >> s) & keep;
    const T xr = mu + from_bits<T>((U)(qi << s));
    const bool good = exact_le<T>(x[i], xr, e) && exact_le<T>(xr, x[i], e);
    ok = ok && (good || i >= cnt);
    q[i] = qi;
  }
  return ok;
}

// OR a string of L <= sizeof(U) bytes (first byte in the low byte of sv) into
// the LDS byte stream at byte offset off.
__device__ __forceinline__ void lds_put(uint32_t* stage, uint32_t off, uint32_t sv) {
  const uint32_t d = off >> 2, sh = (off & 3u) * 8u;
  const uint32_t lo = sv << sh;
  const uint32_t hi = sh ? (sv >> (32u - sh)) : 0u;
  if (lo) atomicOr(stage + d, lo);
  if (hi) atomicOr(stage + d + 1, hi);
}
__device__ __forceinline__ void lds_put(uint32_t* stage, uint32_t off, uint64_t sv) {
  const uint32_t d = off >> 2, sh = (off & 3u) * 8u;
  const uint64_t lo = sv << sh;
  const uint32_t hi = sh ? (uint32_t)(sv >> (64u - sh)) : 0u;
  if ((uint32_t)lo) atomicOr(stage + d, (uint32_t)lo);
  if ((uint32_t)(lo >> 32)) atomicOr(stage + d + 1, (uint32_t)(lo >> 32));
  if (hi) atomicOr(stage + d + 2, hi);
}

template <typename U>
__device__ __forceinline__ U low_bytes_mask(int L) {
  return L >= (int)sizeof(U) ? (U)~(U)0 : (U)(((U)1 << (8 * L)) - 1);
}

// Copy the staged bytes [0, st + total) to dst_base + [st, st + total), where
// dst_base is 16-byte aligned: whole 16-byte chunks as single stores, the
// shared first and last chunks byte by byte.
__device__ __forceinline__ void copy_out(uint8_t* __restrict__ dst_base, const uint32_t* stage,
                                         uint32_t st, uint32_t total) {
  const uint32_t end = st + total;
  const uint32_t nchunk = (end + 15) / 16;
  for (uint32_t c = threadIdx.x; c < nchunk; c += kWG) {
    const uint32_t lo = c * 16 < st ? st : c * 16;
    const uint32_t hi = c * 16 + 16 > end ? end : c * 16 + 16;
    if (lo == c * 16 && hi == c * 16 + 16) {
      const uint4 u = reinterpret_cast<const uint4*>(stage)[c];
      *reinterpret_cast<uint4*>(dst_base + c * 16) = u;
    } else {
      for (uint32_t i = lo; i < hi; ++i) dst_base[i] = (uint8_t)(stage[i >> 2] >> ((i & 3u) * 8u));
    }
  }
}

template <typename T, int B>
__global__ __launch_bounds__(256) void k_encode(const T* __restrict__ x, uint8_t* __restrict__ out,
                                                const typename Traits<T>::U* __restrict__ stats,
                                                const uint32_t* __restrict__ rec, uint64_t* enc_status,
                                                Counters* ctr, uint64_t n, uint64_t nblk, uint64_t mu_off) {
  using U = typename Traits<T>::U;
  using G = Geo<T, B>;
  constexpr int EPL = G::EPL, LPB = G::LPB, TB = G::TB;
  constexpr int BYTES = Traits<T>::BYTES;
  constexpr int STAGE_WORDS = (G::TILE * BYTES + 16) / 4 + 4;
  __shared__ uint32_t s_scan[kWavesPerWG];
  __shared__ uint64_t s_base;
  __shared__ __align__(16) uint32_t s_stage[STAGE_WORDS];

  const uint64_t n_nc = ctr->n_nc;
  const T e = from_bits<T>((U)ctr->e_bits);
  const Sections sec = sections(nblk, n_nc, BYTES, B, 0);
  const uint32_t ntiles = (uint32_t)cdiv(n_nc, TB);
  T* mus = reinterpret_cast<T*>(out + mu_off);
  const int g = threadIdx.x / LPB, lig = threadIdx.x % LPB;

  {
    const uint32_t t = blockIdx.x;
    if (t >= ntiles) return;  // the grid covers every block; fewer are non-constant

    const uint64_t r = (uint64_t)t * TB + g;
    const bool active = r < n_nc;
    const uint64_t k = active ? rec[r] : 0;
    const uint64_t nk = active ? ((n - k * B) < (uint64_t)B ? (n - k * B) : (uint64_t)B) : 0;
    const int cnt = (int)((uint64_t)lig * EPL >= nk ? 0 : (nk - (uint64_t)lig * EPL > (uint64_t)EPL ? EPL : nk - (uint64_t)lig * EPL));
    T xv[EPL];
    load_run<T, EPL>(x, k * B + (uint64_t)lig * EPL, k * B + nk, xv);

    // block parameters from the extrema
    int K = -1;  // -1: raw
    T mu = (T)0;
    if (active) {
      const U kmin = stats[2 * k], kmax = stats[2 * k + 1];
      if (!(kmin < FiniteKeys<T>::LO || kmax > FiniteKeys<T>::HI)) {
        const T mn = from_bits<T>(key_to_bits<U>(kmin));
        const T mx = from_bits<T>(key_to_bits<U>(kmax));
        int m0;
        classify_block<T>(mn, mx, e, mu, m0);
        K = kept_bits<T>(m0);
      }
    }
    // error control: K0, then one more bit, then raw (all lanes take part in
    // the votes; inactive and raw groups vote yes)
    U q[EPL];
    bool ok = encode_try<T, EPL>(xv, K > 0 ? cnt : 0, mu, e, K > 0 ? K : Traits<T>::W, q);
    bool pass = group_all<LPB>(ok);
    if (K > 0 && !pass) {
      const int K1 = kept_bits<T>(K - Traits<T>::KMIN + 1);
      if (K1 != K) {
        ok = encode_try<T, EPL>(xv, cnt, mu, e, K1, q);
        K = K1;
      } else {
        ok = false;
      }
    } else {
      ok = true;
    }
    pass = group_all<LPB>(ok);
    if (!pass) K = -1;

    // codes and per-value byte counts
    const bool raw = K < 0;
    const int nb = raw ? 0 : bytes_of(K);
    U prev = __shfl_up(q[EPL - 1], 1, LPB);
    if (lig == 0) prev = 0;
    uint32_t codes = 0;  // EPL codes, 2 bits each, first value most significant
    int c[EPL];
    uint32_t lane_bytes = 0;
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      int ci = same_lead_bytes(q[i], prev);
      ci = ci > 3 ? 3 : ci;
      ci = ci > nb ? nb : ci;
      ci = (raw || i >= cnt) ? 0 : ci;
      c[i] = ci;
      codes |= (uint32_t)ci << (2 * (EPL - 1 - i));
      prev = q[i];
      lane_bytes += i < cnt ? (raw ? BYTES : nb - ci) : 0;
    }
    uint32_t tile_bytes;
    const uint32_t lane_off = wg_excl_sum<uint32_t>(lane_bytes, s_scan, tile_bytes);

    // zero the staging area while wave 0 resolves the tile's output offset
    for (int i = threadIdx.x; i < STAGE_WORDS / 4; i += kWG)
      reinterpret_cast<uint4*>(s_stage)[i] = make_uint4(0, 0, 0, 0);
    if (threadIdx.x < kWave) {
      const uint64_t p = lookback_excl(enc_status, t, tile_bytes, &ctr->err, 1u);
      if (threadIdx.x == 0) s_base = p;
    }
    __syncthreads();
    const uint64_t base = s_base;
    const uint64_t gdst = sec.mid + base;
    const uint32_t st = (uint32_t)(gdst & 15u);

    if (active) {
      if (lig == 0) {
        out[sec.kbytes + r] = raw ? kRawK : (uint8_t)K;
        if (raw) mus[k] = (T)0;
      }
      // this lane's codes: EPL/4 bytes, first value in the top bits of the first byte
      uint8_t* cdst = out + sec.codes + r * (B / 4) + (uint64_t)lig * (EPL / 4);
      if constexpr (EPL == 8) {
        const uint16_t wv = (uint16_t)(((codes >> 8) & 0xFFu) | ((codes & 0xFFu) << 8));
        *reinterpret_cast<uint16_t*>(cdst) = wv;
      } else {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) cdst[j] = (uint8_t)(codes >> (8 * (EPL / 4 - 1 - j)));
      }
    }
    // stage the kept bytes of each value, most significant first
    uint32_t off = st + lane_off;
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      if (i < cnt) {
        if (raw) {
          lds_put(s_stage, off, (U)bits_of(xv[i]));
          off += BYTES;
        } else {
          const int L = nb - c[i];
          if (L > 0) {
            const U img = byte_swap(q[i]);
            const U sv = (U)(img >> (8 * c[i])) & low_bytes_mask<U>(L);
            lds_put(s_stage, off, sv);
          }
          off += L;
        }
      }
    }
    __syncthreads();
    copy_out(out + (gdst - st), s_stage, st, tile_bytes);
    if (t == ntiles - 1 && threadIdx.x == 0) ctr->mid_total = base + tile_bytes;
  }
}

// --------------------------------------------------------------- finalize ---

struct HeaderArgs {
  uint32_t dtype, eb_mode, ndims, b;
  uint64_t dims[4];
  uint64_t n, nblk;
  double eb;
  uint32_t w;
};

__global__ void k_finalize(uint8_t* __restrict__ out, uint64_t* out_size, const Counters* ctr,
                           HeaderArgs h) {
  const uint64_t n_nc = ctr->n_nc, mid_total = ctr->mid_total;
  const Sections s = sections(h.nblk, n_nc, h.w, h.b, mid_total);
  if (threadIdx.x == 0) {
    uint32_t* o32 = reinterpret_cast<uint32_t*>(out);
    uint64_t* o64 = reinterpret_cast<uint64_t*>(out);
    o32[0] = kMagic;
    o32[1] = (uint32_t)kVersion | (h.dtype << 8) | (h.eb_mode << 16) | (h.ndims << 24);
    o32[2] = h.b;
    o32[3] = 0;
    for (int d = 0; d < 4; ++d) o64[2 + d] = h.dims[d];
    o64[6] = h.n;
    o64[7] = (uint64_t)__double_as_longlong(h.eb);
    o64[8] = ctr->e_bits;
    o64[9] = h.nblk;
    o64[10] = n_nc;
    o64[11] = mid_total;
    *out_size = ctr->err ? 0 : s.total;
  }
  // zero padding: after the state words, after mu, after K, after codes
  const uint64_t pads[4][2] = {{96 + 8 * cdiv(h.nblk, 64), s.mu},
                               {s.mu + h.nblk * h.w, s.kbytes},
                               {s.kbytes + n_nc, s.codes},
                               {s.codes + n_nc * (h.b / 4), s.mid}};
  for (int p = 0; p < 4; ++p)
    for (uint64_t i = pads[p][0] + threadIdx.x; i < pads[p][1]; i += blockDim.x) out[i] = 0;
}

// ---------------------------------------------------------------- launch ---

template <typename T, int B>
hipError_t launch_compress_t(const Job& j, const CompressLaunch& L, TimerHook hook) {
  using U = typename Traits<T>::U;
  using G = Geo<T, B>;
  const WsLayout W = ws_layout(j.nblk, j.w, j.b);
  Counters* ctr = reinterpret_cast<Counters*>(L.ws + W.counters);
  U* stats = reinterpret_cast<U*>(L.ws + W.stats);
  uint32_t* rec = reinterpret_cast<uint32_t*>(L.ws + W.rec);
  uint64_t* cls_st = reinterpret_cast<uint64_t*>(L.ws + W.cls_status);
  uint64_t* enc_st = reinterpret_cast<uint64_t*>(L.ws + W.enc_status);
  uint64_t* part = reinterpret_cast<uint64_t*>(L.ws + W.range_part);
  const uint64_t ncls = cdiv(j.nblk, kClsTile) + 1;
  const uint64_t nenc = cdiv(j.nblk, G::TB) + 1;
  const Sections sec0 = sections(j.nblk, 0, j.w, j.b, 0);

  auto run = [&](const char* name, auto&& fn) {
    if (hook) hook(name, L.stream, 1);
    fn();
    if (hook) hook(name, L.stream, 0);
  };
  {
    const uint32_t grid = (uint32_t)std::min<uint64_t>(cdiv(ncls + nenc, 256), 1024);
    run("k_init", [&] { k_init<<<grid, 256, 0, L.stream>>>(ctr, cls_st, ncls, enc_st, nenc, nullptr); });
  }
  if (j.nblk > 0) {
    const uint64_t ntile = cdiv(j.n, (uint64_t)G::TILE);
    const uint32_t grid = (uint32_t)std::min<uint64_t>(ntile, std::min<uint64_t>(kMaxRangeParts, (uint64_t)L.n_cu * 4));
    run("k_stats", [&] {
      k_stats<T, B><<<grid, 256, 0, L.stream>>>((const T*)L.in, j.n, j.nblk, stats, part);
    });
    const uint32_t gcls = (uint32_t)cdiv(j.nblk, kClsTile);
    run("k_classify", [&] {
      k_classify<T><<<gcls, 256, 0, L.stream>>>(stats, L.out, rec, cls_st, ctr, j.nblk, sec0.mu,
                                                j.eb_mode == 1 ? 1 : 0, j.eb, part, grid);
    });
    const uint32_t genc = (uint32_t)cdiv(j.nblk, G::TB);
    run("k_encode", [&] {
      k_encode<T, B><<<genc, 256, 0, L.stream>>>((const T*)L.in, L.out, stats, rec, enc_st, ctr, j.n,
                                                  j.nblk, sec0.mu);
    });
  }
  HeaderArgs h;
  h.dtype = j.dtype;
  h.eb_mode = j.eb_mode;
  h.ndims = j.ndims;
  h.b = j.b;
  for (int d = 0; d < 4; ++d) h.dims[d] = j.dims[d];
  h.n = j.n;
  h.nblk = j.nblk;
  h.eb = j.eb;
  h.w = j.w;
  run("k_finalize", [&] { k_finalize<<<1, 64, 0, L.stream>>>(L.out, L.out_size, ctr, h); });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_compress_dt(const Job& j, const CompressLaunch& L, TimerHook hook) {
  switch (j.b) {
    case 8: return launch_compress_t<T, 8>(j, L, hook);
    case 16: return launch_compress_t<T, 16>(j, L, hook);
    case 32: return launch_compress_t<T, 32>(j, L, hook);
    case 64: return launch_compress_t<T, 64>(j, L, hook);
    case 128: return launch_compress_t<T, 128>(j, L, hook);
    case 256: return launch_compress_t<T, 256>(j, L, hook);
    case 512: return launch_compress_t<T, 512>(j, L, hook);
    case 1024: return launch_compress_t<T, 1024>(j, L, hook);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_compress(const Job& j, const CompressLaunch& L, TimerHook hook) {
  return j.dtype == 0 ? launch_compress_dt<float>(j, L, hook) : launch_compress_dt<double>(j, L, hook);
}

}  // namespace szx
