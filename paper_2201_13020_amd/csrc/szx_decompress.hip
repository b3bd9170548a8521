// szx_decompress.hip -- decompression kernel of the SZx method for gfx950.
//
// One persistent kernel over tiles of consecutive blocks, tiles taken in
// workgroup order (tile t = workgroup t). Per tile:
//   1. state bits -> the tile's non-constant blocks; a device-wide prefix count
//      (decoupled look-back) gives their ranks, hence their K byte and codes;
//   2. per value, the count of stored mid bytes (kept bytes minus the leading
//      bytes the 2-bit code says are shared); a second device-wide prefix sum
//      gives the tile's first mid byte ("a parallel prefix-scan is applied
//      before retrieving the mid-bytes", Sec. V-B);
//   3. the tile's mid bytes are staged in LDS with aligned 16-byte loads;
//   4. leading bytes: byte j of value i is the stored byte j of the nearest
//      value i' <= i whose code stores byte j (Sec. V-B, index propagation).
//      This is one inclusive scan over (code, top bytes) pairs with the
//      associative operator (c_a, S_a) . (c_b, S_b) = (min(c_a, c_b),
//      (S_a & top(c_b)) | S_b);
//   5. x' = mu + (q' << s); constant blocks are filled with mu, raw blocks
//      copied.
// Every read of the stream is bounded by in_bytes; a malformed stream sets
// *status = SZ_ECORRUPT and leaves no buffer.
#include <algorithm>

#include "szx_device.hpp"
#include "szx_launch.hpp"

namespace szx {

constexpr uint32_t kStatusCorrupt = 3;  // SZ_ECORRUPT
constexpr uint32_t kStatusDevice = 4;   // SZ_EDEVICE: a bounded wait gave up

struct DecodeArgs {
  const uint8_t* in;
  uint64_t in_bytes;
  uint8_t* out;
  uint32_t* status;
  Counters* ctr;
  uint64_t* rank_st;
  uint64_t* mid_st;
  uint64_t n, nblk;
  uint32_t dtype, ndims;
  uint64_t dims[4];
};

__global__ __launch_bounds__(256) void k_dinit(Counters* ctr, uint64_t* st1, uint64_t n1, uint32_t* status) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1; i += stride) st1[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *status = 0;
  }
}

__device__ __forceinline__ uint64_t rd64(const uint8_t* p) { return *reinterpret_cast<const uint64_t*>(p); }
__device__ __forceinline__ uint32_t rd32(const uint8_t* p) { return *reinterpret_cast<const uint32_t*>(p); }

// Mask of the top c bytes of the 24-bit leading field kept in bits 31..8.
__device__ __forceinline__ uint32_t lead_mask(uint32_t c) {
  return c == 0 ? 0u : (c == 1 ? 0xFF000000u : (c == 2 ? 0xFFFF0000u : 0xFFFFFF00u));
}

// Composition of two leading-byte transforms packed as (S in bits 31..8, c in
// bits 1..0): first `a`, then `b`.
__device__ __forceinline__ uint32_t lead_compose(uint32_t a, uint32_t b) {
  const uint32_t ca = a & 3u, cb = b & 3u;
  const uint32_t s = ((a & 0xFFFFFF00u) & lead_mask(cb)) | (b & 0xFFFFFF00u);
  return s | (ca < cb ? ca : cb);
}

template <typename U>
__device__ __forceinline__ uint32_t top24(U q) {
  return (uint32_t)(q >> (sizeof(U) * 8 - 32)) & 0xFFFFFF00u;
}
template <typename U>
__device__ __forceinline__ U from_top24(uint32_t t) {
  return (U)t << (sizeof(U) * 8 - 32);
}

// Read L <= sizeof(U) bytes at byte offset off of the staged stream; the first
// byte lands in the low byte of the result.
__device__ __forceinline__ uint32_t lds_get32(const uint32_t* stage, uint32_t off) {
  const uint32_t d = off >> 2, sh = (off & 3u) * 8u;
  const uint64_t v = (uint64_t)stage[d] | ((uint64_t)stage[d + 1] << 32);
  return (uint32_t)(v >> sh);
}
__device__ __forceinline__ uint64_t lds_get64(const uint32_t* stage, uint32_t off) {
  const uint32_t d = off >> 2, sh = (off & 3u) * 8u;
  const uint64_t lo = (uint64_t)stage[d] | ((uint64_t)stage[d + 1] << 32);
  const uint64_t hi = stage[d + 2];
  return sh ? ((lo >> sh) | (hi << (64u - sh))) : lo;
}
template <typename U>
__device__ __forceinline__ U lds_get(const uint32_t* stage, uint32_t off);
template <>
__device__ __forceinline__ uint32_t lds_get<uint32_t>(const uint32_t* stage, uint32_t off) {
  return lds_get32(stage, off);
}
template <>
__device__ __forceinline__ uint64_t lds_get<uint64_t>(const uint32_t* stage, uint32_t off) {
  return lds_get64(stage, off);
}

template <typename U>
__device__ __forceinline__ U low_mask(int L) {
  return L >= (int)sizeof(U) ? (U)~(U)0 : (U)(((U)1 << (8 * L)) - 1);
}

template <typename T, int EPL>
__device__ __forceinline__ void store_run(T* __restrict__ y, uint64_t i0, int cnt, const T (&v)[EPL]) {
  if (cnt == EPL) {
    constexpr int PER16 = 16 / sizeof(T);
    uint4* p = reinterpret_cast<uint4*>(y + i0);
#pragma unroll
    for (int c = 0; c < EPL / PER16; ++c) {
      uint4 u;
      if constexpr (sizeof(T) == 4) {
        u.x = __float_as_uint(v[c * 4 + 0]);
        u.y = __float_as_uint(v[c * 4 + 1]);
        u.z = __float_as_uint(v[c * 4 + 2]);
        u.w = __float_as_uint(v[c * 4 + 3]);
      } else {
        const uint64_t a = (uint64_t)__double_as_longlong(v[c * 2 + 0]);
        const uint64_t b = (uint64_t)__double_as_longlong(v[c * 2 + 1]);
        u.x = (uint32_t)a;
        u.y = (uint32_t)(a >> 32);
        u.z = (uint32_t)b;
        u.w = (uint32_t)(b >> 32);
      }
      p[c] = u;
    }
  } else {
#pragma unroll
    for (int i = 0; i < EPL; ++i)
      if (i < cnt) y[i0 + i] = v[i];
  }
}

template <typename T, int B>
__global__ __launch_bounds__(256) void k_decode(DecodeArgs a) {
  using U = typename Traits<T>::U;
  using G = Geo<T, B>;
  constexpr int EPL = G::EPL, LPB = G::LPB, TB = G::TB;
  constexpr int BYTES = Traits<T>::BYTES;
  constexpr int STAGE_WORDS = (G::TILE * BYTES + 32) / 4 + 4;
  __shared__ uint32_t s_scan[kWavesPerWG];
  __shared__ uint64_t s_r0, s_m0;
  __shared__ __align__(16) uint32_t s_stage[STAGE_WORDS];

  // header checks, identical in every workgroup
  const uint8_t* in = a.in;
  bool hdr_ok = a.in_bytes >= kHeaderBytes;
  uint64_t n_nc = 0, mid_total = 0;
  Sections sec = sections(a.nblk, 0, BYTES, B, 0);
  if (hdr_ok) {
    const uint32_t w1 = rd32(in + 4);
    hdr_ok = rd32(in) == kMagic && (w1 & 0xFFu) == kVersion && ((w1 >> 8) & 0xFFu) == a.dtype &&
             ((w1 >> 16) & 0xFFu) <= 1 && ((w1 >> 24) & 0xFFu) == a.ndims && rd32(in + 8) == (uint32_t)B &&
             rd64(in + 48) == a.n && rd64(in + 72) == a.nblk;
    for (int d = 0; d < 4; ++d) hdr_ok = hdr_ok && rd64(in + 16 + 8 * d) == a.dims[d];
    n_nc = rd64(in + 80);
    mid_total = rd64(in + 88);
    hdr_ok = hdr_ok && n_nc <= a.nblk && mid_total <= a.n * BYTES;
    if (hdr_ok) {
      sec = sections(a.nblk, n_nc, BYTES, B, mid_total);
      hdr_ok = sec.total <= a.in_bytes;
    }
  }
  if (!hdr_ok) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(a.status, kStatusCorrupt);
    return;
  }

  const uint32_t ntiles = (uint32_t)cdiv(a.nblk, TB);
  const int g = threadIdx.x / LPB, lig = threadIdx.x % LPB;
  const int lane = lane_id();
  const T* mus = reinterpret_cast<const T*>(in + sec.mu);
  T* y = reinterpret_cast<T*>(a.out);

  {
    const uint32_t t = blockIdx.x;
    if (t >= ntiles) return;
    bool bad = false;

    const uint64_t k = (uint64_t)t * TB + g;
    const bool inb = k < a.nblk;
    const bool nc = inb && ((in[sec.state + (k >> 3)] >> (k & 7)) & 1u);
    const uint64_t nk = inb ? std::min<uint64_t>((uint64_t)B, a.n - k * B) : 0;
    const int cnt = (int)((uint64_t)lig * EPL >= nk ? 0 : std::min<uint64_t>(EPL, nk - (uint64_t)lig * EPL));

    // 1. ranks of the tile's non-constant blocks
    uint32_t tile_nc;
    const uint32_t rank_in_tile = wg_excl_sum<uint32_t>((lig == 0 && nc) ? 1u : 0u, s_scan, tile_nc);
    const uint32_t grp_rank = __shfl(rank_in_tile, lane - lig);
    if (threadIdx.x < kWave) {
      const uint64_t p = lookback_excl(a.rank_st, t, tile_nc, a.status, kStatusDevice);
      if (threadIdx.x == 0) s_r0 = p;
    }
    __syncthreads();
    const uint64_t r = s_r0 + grp_rank;
    if (t == ntiles - 1 && threadIdx.x == 0 && s_r0 + tile_nc != n_nc) bad = true;
    const bool have = nc && r < n_nc;
    bad = bad || (nc && r >= n_nc);

    // 2. per-value byte counts
    int K = have ? (int)in[sec.kbytes + r] : 0;
    const bool raw = have && K == kRawK;
    if (have && !raw && (K < Traits<T>::KMIN || K > Traits<T>::W)) {
      bad = true;
      K = 0;
    }
    const bool coded = have && !raw && K != 0;
    const int nb = coded ? bytes_of(K) : 0;
    uint32_t cw = 0;  // this lane's EPL codes, first value in the top bits
    if (coded) {
      const uint8_t* cp = in + sec.codes + r * (B / 4) + (uint64_t)lig * (EPL / 4);
#pragma unroll
      for (int j = 0; j < EPL / 4; ++j) cw = (cw << 8) | cp[j];
    }
    int c[EPL];
    uint32_t lane_bytes = 0;
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      int ci = (int)((cw >> (2 * (EPL - 1 - i))) & 3u);
      if (ci > nb) {
        bad = bad || (coded && i < cnt);
        ci = nb;
      }
      c[i] = ci;
      lane_bytes += i < cnt ? (raw ? BYTES : (coded ? nb - ci : 0)) : 0;
    }
    uint32_t tile_bytes;
    const uint32_t lane_off = wg_excl_sum<uint32_t>(lane_bytes, s_scan, tile_bytes);
    if (threadIdx.x < kWave) {
      const uint64_t p = lookback_excl(a.mid_st, t, tile_bytes, a.status, kStatusDevice);
      if (threadIdx.x == 0) s_m0 = p;
    }
    __syncthreads();
    const uint64_t m0 = s_m0;
    if (m0 + tile_bytes > mid_total) bad = true;
    if (t == ntiles - 1 && threadIdx.x == 0 && m0 + tile_bytes != mid_total) bad = true;

    // 3. stage the tile's mid bytes, aligned as in the stream
    const uint64_t src = sec.mid + m0;
    const uint32_t st = (uint32_t)(src & 15u);
    const uint64_t src0 = src - st;
    {
      const uint32_t nchunk = (st + tile_bytes + 15) / 16;
      for (uint32_t ch = threadIdx.x; ch < nchunk; ch += kWG) {
        const uint64_t gpos = src0 + (uint64_t)ch * 16;
        uint4 u = make_uint4(0, 0, 0, 0);
        if (gpos + 16 <= a.in_bytes) {
          u = *reinterpret_cast<const uint4*>(in + gpos);
        } else {
          uint32_t wv[4] = {0, 0, 0, 0};
          for (int bq = 0; bq < 16; ++bq)
            if (gpos + bq < a.in_bytes) wv[bq >> 2] |= (uint32_t)in[gpos + bq] << ((bq & 3) * 8);
          u = make_uint4(wv[0], wv[1], wv[2], wv[3]);
        }
        reinterpret_cast<uint4*>(s_stage)[ch] = u;
      }
    }
    __syncthreads();

    // 4. values
    const T mu = inb ? mus[k] : (T)0;
    T v[EPL];
    if (!nc || !have) {
#pragma unroll
      for (int i = 0; i < EPL; ++i) v[i] = mu;
    } else if (raw) {
      uint32_t off = st + lane_off;
#pragma unroll
      for (int i = 0; i < EPL; ++i) {
        v[i] = from_bits<T>(lds_get<U>(s_stage, off));
        off += i < cnt ? BYTES : 0;
      }
    } else {
      const int s = shift_of(K > 0 ? K : Traits<T>::W);
      uint32_t off = st + lane_off;
      U q0[EPL];
      uint32_t cmin[EPL];
      U run = 0;
      uint32_t cm = 3;
#pragma unroll
      for (int i = 0; i < EPL; ++i) {
        const int L = i < cnt ? nb - c[i] : 0;
        U sv = 0;
        if (L > 0) sv = (U)(lds_get<U>(s_stage, off) & low_mask<U>(L)) << (8 * c[i]);
        off += L;
        const U stored = byte_swap(sv);
        // invalid trailing values act as the identity (keep all, add nothing)
        const int ci = i < cnt ? c[i] : 3;
        run = (run & top_bytes_mask<U>(ci)) | stored;
        cm = (uint32_t)ci < cm ? (uint32_t)ci : cm;
        q0[i] = run;
        cmin[i] = cm;
      }
      // carry of the leading bytes from the lanes before this one in the block
      uint32_t pk = top24<U>(run) | cm;
#pragma unroll
      for (int d = 1; d < LPB; d <<= 1) {
        const uint32_t o = __shfl_up(pk, d, LPB);
        if (lig >= d) pk = lead_compose(o, pk);
      }
      uint32_t carry = __shfl_up(pk, 1, LPB) & 0xFFFFFF00u;
      if (lig == 0) carry = 0;
      const U cfull = from_top24<U>(carry);
#pragma unroll
      for (int i = 0; i < EPL; ++i) {
        const U qi = q0[i] | (cfull & top_bytes_mask<U>((int)cmin[i]));
        v[i] = mu + from_bits<T>((U)(qi << s));
      }
    }
    if (cnt > 0) store_run<T, EPL>(y, k * B + (uint64_t)lig * EPL, cnt, v);
    if (__ballot(bad) != 0 && lane == 0) atomicMax(a.status, kStatusCorrupt);
  }
}

// ---------------------------------------------------------------- launch ---

template <typename T, int B>
hipError_t launch_decompress_t(const Job& j, const DecompressLaunch& L, TimerHook hook) {
  using G = Geo<T, B>;
  const WsLayout W = ws_layout(j.nblk, j.w, j.b);
  Counters* ctr = reinterpret_cast<Counters*>(L.ws + W.counters);
  uint64_t* rank_st = reinterpret_cast<uint64_t*>(L.ws + W.dec_rank);
  const uint64_t ntile = cdiv(j.nblk, G::TB) + 1;
  // dec_rank and dec_mid are adjacent pieces of the workspace: clear both
  const uint64_t nclear = (W.total - W.dec_rank) / 8;
  auto run = [&](const char* name, auto&& fn) {
    if (hook) hook(name, L.stream, 1);
    fn();
    if (hook) hook(name, L.stream, 0);
  };
  {
    const uint32_t grid = (uint32_t)std::min<uint64_t>(cdiv(nclear, 256), 1024);
    run("k_dinit", [&] { k_dinit<<<grid ? grid : 1, 256, 0, L.stream>>>(ctr, rank_st, nclear, L.status); });
  }
  DecodeArgs a;
  a.in = (const uint8_t*)L.in;
  a.in_bytes = L.in_bytes;
  a.out = (uint8_t*)L.out;
  a.status = L.status;
  a.ctr = ctr;
  a.rank_st = rank_st;
  a.mid_st = reinterpret_cast<uint64_t*>(L.ws + W.dec_mid);
  a.n = j.n;
  a.nblk = j.nblk;
  a.dtype = j.dtype;
  a.ndims = j.ndims;
  for (int d = 0; d < 4; ++d) a.dims[d] = j.dims[d];
  (void)ntile;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, cdiv(j.nblk, G::TB));
  run("k_decode", [&] { k_decode<T, B><<<grid, 256, 0, L.stream>>>(a); });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_decompress_dt(const Job& j, const DecompressLaunch& L, TimerHook hook) {
  switch (j.b) {
    case 8: return launch_decompress_t<T, 8>(j, L, hook);
    case 16: return launch_decompress_t<T, 16>(j, L, hook);
    case 32: return launch_decompress_t<T, 32>(j, L, hook);
    case 64: return launch_decompress_t<T, 64>(j, L, hook);
    case 128: return launch_decompress_t<T, 128>(j, L, hook);
    case 256: return launch_decompress_t<T, 256>(j, L, hook);
    case 512: return launch_decompress_t<T, 512>(j, L, hook);
    case 1024: return launch_decompress_t<T, 1024>(j, L, hook);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_decompress(const Job& j, const DecompressLaunch& L, TimerHook hook) {
  return j.dtype == 0 ? launch_decompress_dt<float>(j, L, hook) : launch_decompress_dt<double>(j, L, hook);
}

}  // namespace szx
