// szx_decompress.hip -- decompression kernels of the SZx method for gfx950.
//
// Two kernels per call:
//   k_dindex  over tiles of consecutive blocks: state bits give each tile's
//             non-constant blocks and their ranks (hence their K byte and
//             codes) -- the population count of the state bits before the
//             tile for the first 256 tiles, a light single-pass prefix count
//             after them; workgroup 0 first clears the status words that the
//             prefix sums use (a gate holds the others); per value the number of
//             stored mid bytes is the kept bytes minus the leading bytes its
//             2-bit code shares, and a second light prefix sum gives the first
//             mid byte of every decode tile (Sec. V-B locates the mid bytes by
//             a prefix sum of these counts before they are read).
//   k_decode  every decode tile on its own, no waiting: it stages its mid bytes
//             in LDS with aligned 16-byte loads, resolves leading bytes -- byte
//             j of value i is the stored byte j of the nearest value i' <= i
//             whose code stores byte j (Sec. V-B, index propagation) -- with one
//             inclusive scan over (code, top bytes) pairs under the associative
//             operator (c_a, S_a) . (c_b, S_b) = (min(c_a, c_b),
//             (S_a & top(c_b)) | S_b), and writes x' = mu + (q' << s);
//             constant blocks get mu, raw blocks their stored bytes.
// Every read of the stream is bounded by in_bytes; a malformed stream sets
// *status = SZ_ECORRUPT and no access leaves the given buffers.
#include <algorithm>

#include "szx_device.hpp"
#include "szx_launch.hpp"

namespace szx {

constexpr uint32_t kStatusCorrupt = 3;  // SZ_ECORRUPT
constexpr uint32_t kStatusDevice = 4;   // SZ_EDEVICE: a bounded wait gave up
constexpr uint32_t kDirectRankTiles = 256;  // index tiles that count their first rank directly

// Field of a call, or of a batch entry (a copy with its pointers typed as
// global memory).
__device__ __forceinline__ FieldD field_at(const DBatch& b, uint32_t fi) {
  FieldD f = b.fields ? b.fields[fi] : b.one;
  f.in = as_global(f.in);
  f.out = as_global(f.out);
  f.status = as_global(f.status);
  f.index = as_global(f.index);
  f.rank_st = as_global(f.rank_st);
  f.mid_st = as_global(f.mid_st);
  return f;
}
__device__ __forceinline__ uint32_t dfield_of(const uint32_t* map, uint64_t t) { return map ? map[t] : 0u; }

// Only for calls without index tiles (every field empty): their status words.
__global__ __launch_bounds__(256) void k_dinit(DBatch b) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t nf = b.fields ? b.nfields : 1;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += stride) *field_at(b, (uint32_t)i).status = 0;
}

// ---------------------------------------------------------------- gate ---
// The index pass's status words and every field's status word must be zero
// before any index tile publishes or reports an error, and no launch of its
// own clears them. Workgroup 0 of the call's first index launch (dispatched
// first) clears them and then stores the call's token in the go word; every
// other workgroup waits for the token before its first publish or report
// (its stream loads are already out). The second index launch of a mixed
// batch finds the token there and clears nothing. The token changes with
// every call: the last decode launch advances the epoch it comes from, when
// no index tile reads it any more.
__device__ __forceinline__ uint64_t gate_token(const DBatch& b) {
  return status_load(as_global(b.gate) + kGateEpochWord) ^ kGateKey;
}

__device__ __forceinline__ void gate_open(const DBatch& b, int* s_flag) {
  uint64_t* gate = as_global(b.gate);
  if (threadIdx.x == 0) *s_flag = status_load(gate + kGateGoWord) != gate_token(b);
  __syncthreads();
  if (!*s_flag) return;  // the same in every thread
  for (uint64_t i = threadIdx.x; i < b.zero_words; i += kWG) status_store(as_global(b.zero_begin) + i, 0);
  const uint32_t nf = b.fields ? b.nfields : 1u;
  for (uint32_t i = threadIdx.x; i < nf; i += kWG)
    __hip_atomic_store((__attribute__((address_space(1))) uint32_t*)field_at(b, i).status, 0u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  // every wave's stores are performed before the barrier (a release only: an
  // acquire would also drop this XCD's L2)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) status_store(gate + kGateGoWord, gate_token(b));
}

// Every workgroup but 0 waits for the token before its first publish or
// error report. Its later reads of the cleared words are device-scope atomic
// loads issued after the token is seen, so they need no fence (a fence here
// would drop the XCD's L2 for every tile). Workgroup 0 opens the gate right
// after its descriptor and header loads (a store ahead of them would keep the
// compiler from making them scalar loads), while the others load their state
// bits.
__device__ __forceinline__ void gate_wait(const DBatch& b, uint32_t* status) {
  if (blockIdx.x == 0) return;
  if (threadIdx.x == 0) {
    const uint64_t* go = as_global(b.gate) + kGateGoWord;
    const uint64_t tok = gate_token(b);
    uint32_t spins = 0;
    while (status_load(go) != tok) {
      if (++spins > kSpinLimit) {
        atomicMax(status, kStatusDevice);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
}

__device__ __forceinline__ uint64_t rd64(const uint8_t* p) { return *reinterpret_cast<const uint64_t*>(p); }
__device__ __forceinline__ uint32_t rd32(const uint8_t* p) { return *reinterpret_cast<const uint32_t*>(p); }

// Mask of the top c bytes (c in [0, 3]) of the 24-bit leading field kept in
// bits 31..8, branch-free: the field's mask shifted left by 8 (3 - c).
__device__ __forceinline__ uint32_t lead_mask(uint32_t c) { return 0xFFFFFF00u << (8u * (3u - c)); }

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

// The top c bytes of a word, from s8 = 8 c (c in [0, 3]): the complement of
// the all-ones word shifted right by s8.
template <typename U>
__device__ __forceinline__ U top_bytes_of(uint32_t s8) {
  return (U)~((U)~(U)0 >> s8);
}

// Bytes of a decode tile's LDS stage: the tile's mid bytes at most (a value
// stores at most its width), the 15-byte misalignment of their start and the
// round-up to whole 16-byte chunks, then room for the unguarded reads of a
// lane: it starts at most at the end of all stored bytes, advances at most a
// word per value before its last read, and a read takes up to 12 bytes.
template <typename T, int B>
constexpr int dec_stage_words() {
  using G = GeoD<T, B>;
  return (G::TILE * G::SUB * (int)sizeof(T) + 32 + G::EPL * (int)sizeof(T) + 16) / 4;
}

// Previous lane's value within groups of G lanes (lanes with lig < d get
// garbage, which callers discard): DPP row shifts for G <= 16.
template <int G, int D>
__device__ __forceinline__ uint32_t lane_up(uint32_t v) {
  if constexpr (G <= 16) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 + D, 0xF, 0xF, false);  // row_shr:D
  } else {
    return __shfl_up(v, D, G);
  }
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
      if constexpr (sizeof(T) == 4) {
        // streamed past the caches: the values are not read again here, and
        // the field's other passes keep the cache. (Each store of a wave
        // covers 16 bytes of every 32; float64 lanes, 16 of every 64, ran
        // four times slower this way and keep ordinary stores.)
        using v4u = unsigned int __attribute__((ext_vector_type(4)));
        const v4u nv = {u.x, u.y, u.z, u.w};
        __builtin_nontemporal_store(nv, reinterpret_cast<v4u*>(p + c));
      } else {
        p[c] = u;
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < EPL; ++i)
      if (i < cnt) y[i0 + i] = v[i];
  }
}

// Header of the stream, checked against the caller's expectations; identical
// in every workgroup.
struct StreamInfo {
  bool ok;
  uint64_t n_nc, mid_total;
  Sections sec;
};

template <int BYTES, int B>
__device__ __forceinline__ StreamInfo read_header(const FieldD& a) {
  StreamInfo h;
  const uint8_t* in = a.in;
  h.ok = a.in_bytes >= kHeaderBytes;
  h.n_nc = 0;
  h.mid_total = 0;
  h.sec = sections(a.nblk, 0, BYTES, B, 0);
  if (h.ok) {
    const uint32_t w1 = rd32(in + 4);
    h.ok = rd32(in) == kMagic && (w1 & 0xFFu) == kVersion && ((w1 >> 8) & 0xFFu) == a.dtype &&
           ((w1 >> 16) & 0xFFu) <= 1 && ((w1 >> 24) & 0xFFu) == a.ndims && rd32(in + 8) == (uint32_t)B &&
           rd64(in + 48) == a.n && rd64(in + 72) == a.nblk;
    for (int d = 0; d < 4; ++d) h.ok = h.ok && rd64(in + 16 + 8 * d) == a.dims[d];
    h.n_nc = rd64(in + 80);
    h.mid_total = rd64(in + 88);
    h.ok = h.ok && h.n_nc <= a.nblk && h.mid_total <= a.n * BYTES;
    if (h.ok) {
      h.sec = sections(a.nblk, h.n_nc, BYTES, B, h.mid_total);
      h.ok = h.sec.total <= a.in_bytes;
    }
  }
  return h;
}

// A block's code bytes as words of 16 codes (b = 8: one half word in the
// low 16 bits), read through a buffer resource at byte offset off (reads past
// its range return zeros). A block's codes start 16-byte aligned (the codes
// section is, and each block holds b / 4 bytes), so from b = 64 on they load
// as 16-byte words.
template <int B>
struct BlockCodes {
  static constexpr uint32_t NW = B >= 16 ? B / 16 : 1;
  uint32_t raw[NW];
};
template <int B>
__device__ __forceinline__ void load_codes(__amdgpu_buffer_rsrc_t rs, uint32_t off, BlockCodes<B>& c) {
  using v4u = unsigned int __attribute__((ext_vector_type(4)));
  if constexpr (B >= 64) {
#pragma unroll
    for (uint32_t q = 0; q < BlockCodes<B>::NW / 4; ++q) {
      const v4u u = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off + 16u * q), 0, 0);
      c.raw[4 * q + 0] = u.x;
      c.raw[4 * q + 1] = u.y;
      c.raw[4 * q + 2] = u.z;
      c.raw[4 * q + 3] = u.w;
    }
  } else if constexpr (B >= 16) {
#pragma unroll
    for (uint32_t j = 0; j < BlockCodes<B>::NW; ++j)
      c.raw[j] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(off + 4u * j), 0, 0);
  } else {
    c.raw[0] = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)off, 0, 0);
  }
}

// Mid bytes of one non-constant block of nk values with K byte Kb and codes
// c; raises bad for a K outside [1 + E, W] or a code above the kept bytes.
template <typename T, int B>
__device__ __forceinline__ uint32_t block_mid_bytes(const BlockCodes<B>& c, uint32_t Kb, uint32_t nk, bool& bad) {
  constexpr int BYTES = Traits<T>::BYTES;
  if (Kb == kRawK) return nk * BYTES;
  if ((int)Kb < Traits<T>::KMIN || (int)Kb > Traits<T>::W) {
    bad = true;
    return 0;
  }
  const uint32_t nb = (uint32_t)bytes_of((int)Kb);
  uint32_t sum = 0, over = 0;
  // b/4 code bytes, 4 codes per byte, first value in the top bits
#pragma unroll
  for (uint32_t j = 0; j < BlockCodes<B>::NW; ++j) {
    uint32_t w;
    if constexpr (B >= 16) {
      w = __builtin_bswap32(c.raw[j]);
    } else {
      const uint32_t h2 = c.raw[0] & 0xFFFFu;
      w = ((h2 & 0xFFu) << 24) | ((h2 >> 8) << 16);
    }
    const uint32_t first = 16 * j;  // value index of the top code of w
    if (first >= nk) w = 0;
    else if (nk - first < 16) w &= ~0u << (2 * (16 - (nk - first)));  // codes past the block end
    sum += __popc(w & 0x55555555u) + 2u * __popc(w & 0xAAAAAAAAu);
    over |= w & (w >> 1) & 0x55555555u;  // a code of 3
  }
  if (nb == 2 && over) bad = true;
  return nk * nb - sum;
}

// Per tile of CLS blocks (four per thread): ranks of the non-constant blocks
// and mid bytes, each through a light single-pass prefix sum; writes the first
// rank and first mid byte of every decode tile in it.
template <typename T, int B>
__device__ __forceinline__ void dindex_tile(const DBatch& b, const FieldD& a, uint32_t t, uint32_t* s_scan,
                                            uint64_t* s_r0p, uint64_t* s_m0p, int* s_flag) {
  using G = Geo<T, B>;  // classification tiles follow the encode geometry
  constexpr int BYTES = Traits<T>::BYTES;
  constexpr int TBLK = G::TBLK;
  constexpr int CLS = TBLK > (int)kClsMin ? TBLK : (int)kClsMin;
  constexpr int BPT = CLS / kWG;
  static_assert(GeoD<T, B>::TBLK % BPT == 0, "every decode tile starts at some thread's first block");
  uint64_t& s_r0 = *s_r0p;
  uint64_t& s_m0 = *s_m0p;
  const StreamInfo h = read_header<BYTES, B>(a);
  if (blockIdx.x == 0) gate_open(b, s_flag);
  if (!h.ok) {
    gate_wait(b, a.status);
    if (t == 0 && threadIdx.x == 0) atomicMax(a.status, kStatusCorrupt);
    return;
  }
  const uint32_t ntiles = (uint32_t)cdiv(a.nblk, CLS);
  const uint8_t* in = a.in;
  const uint64_t k0 = (uint64_t)t * CLS + (uint64_t)threadIdx.x * BPT;
  bool bad = false;
  // a thread's blocks share one state byte (BPT divides 8): one load
  static_assert(8 % BPT == 0, "a thread's state bits lie in one byte");
  const uint32_t sbyte = k0 < a.nblk ? (uint32_t)in[h.sec.state + (k0 >> 3)] : 0u;
  uint32_t ncb = 0, cnt = 0;
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const uint64_t k = k0 + i;
    const bool nc = k < a.nblk && ((sbyte >> ((uint32_t)(k0 & 7) + i)) & 1u);
    ncb |= (nc ? 1u : 0u) << i;
    cnt += nc ? 1u : 0u;
  }
  // A tile whose preceding state bits are few (the first kDirectRankTiles
  // tiles: at most 32 KiB of them) counts its first rank directly, as the
  // population count of those bits (16-byte words from a 16-byte aligned
  // section, all loads issued at once), and publishes it as inclusive; later
  // tiles chain by look-back and stop at those words.
  const bool direct = t < kDirectRankTiles;
  uint32_t pop = 0;
  if (direct) {
    constexpr uint32_t W16 = kDirectRankTiles * (CLS / 8) / 16 / kWG;  // words per thread, at most
    const uint32_t n16 = t * (CLS / 8) / 16;
    // a buffer resource over exactly those bytes: words past it read zero,
    // so every lane issues the same loads (no branch, no waits between them)
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(in + h.sec.state), (short)0, (int)(n16 * 16u), 0x00020000);
    using v4u = unsigned int __attribute__((ext_vector_type(4)));
    v4u u[W16];
#pragma unroll
    for (uint32_t j = 0; j < W16; ++j) u[j] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)((threadIdx.x + j * kWG) * 16u), 0, 0);
#pragma unroll
    for (uint32_t j = 0; j < W16; ++j) pop += __popc(u[j].x) + __popc(u[j].y) + __popc(u[j].z) + __popc(u[j].w);
  }
  const uint32_t v2[2] = {cnt, pop};
  uint32_t ex2[2], tot2[2];
  wg_excl_scan_multi<2>(v2, ex2, tot2, s_scan);
  const uint32_t rex = ex2[0], tnc = tot2[0];
  gate_wait(b, a.status);
  if (direct) {
    if (threadIdx.x == 0) status_store(a.rank_st + t, kFlagIncl | (((uint64_t)tot2[1] + tnc) & kValueMask));
    if (threadIdx.x == 0) s_r0 = tot2[1];
  } else if (threadIdx.x < kWave) {
    if (threadIdx.x == 0) lookback_publish(a.rank_st, t, tnc);
    const uint64_t p = lookback_resolve_n(a.rank_st, t, tnc, a.status, kStatusDevice, ntiles);
    if (threadIdx.x == 0) s_r0 = p;
  }
  __syncthreads();
  const uint64_t R0 = s_r0;
  // The K bytes and codes of the tile's ranks [R0, R0 + tnc) that the
  // stream holds, through buffer resources over just those bytes (32-bit
  // offsets from the tile's first rank; reads past them return zeros): every
  // load of the thread goes out before any of them is used.
  const uint64_t have_nc = h.n_nc > R0 ? std::min<uint64_t>(h.n_nc - R0, (uint64_t)tnc) : 0;
  const __amdgpu_buffer_rsrc_t rk_ = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t*>(in + h.sec.kbytes + R0), (short)0, (int)have_nc, 0x00020000);
  const __amdgpu_buffer_rsrc_t rc_ = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t*>(in + h.sec.codes + R0 * (B / 4)), (short)0, (int)(have_nc * (B / 4)), 0x00020000);
  uint32_t kbv[BPT];
  BlockCodes<B> cv[BPT];
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    // this block's rank from the tile's first: rex plus the thread's
    // non-constant blocks before it (constant blocks read far past the range)
    const uint32_t rl = rex + (uint32_t)__popc(ncb & ((1u << i) - 1u));
    const bool live = (ncb >> i) & 1u;
    kbv[i] = __builtin_amdgcn_raw_buffer_load_b8(rk_, live ? (int)rl : 0x40000000, 0, 0);
    // up to b = 128 (32 code bytes a block); larger blocks load theirs as
    // they are counted, which keeps their registers in bounds
    if constexpr (B <= 128) load_codes<B>(rc_, live ? rl * (uint32_t)(B / 4) : 0x40000000u, cv[i]);
  }
  uint32_t mid = 0;
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const uint64_t k = k0 + i;
    if ((ncb >> i) & 1u) {
      const uint32_t rl = rex + (uint32_t)__popc(ncb & ((1u << i) - 1u));
      if ((uint64_t)rl < have_nc) {
        const uint32_t nk = (uint32_t)std::min<uint64_t>((uint64_t)B, a.n - k * B);
        if constexpr (B > 128) load_codes<B>(rc_, rl * (uint32_t)(B / 4), cv[i]);
        mid += block_mid_bytes<T, B>(cv[i], kbv[i], nk, bad);
      } else {
        bad = true;
      }
    }
  }
  uint32_t tmid;
  const uint32_t mex = wg_excl_sum<uint32_t>(mid, s_scan, tmid);
  if (threadIdx.x < kWave) {
    if (threadIdx.x == 0) lookback_publish(a.mid_st, t, tmid);
    const uint64_t p = lookback_resolve_n(a.mid_st, t, tmid, a.status, kStatusDevice, ntiles);
    if (threadIdx.x == 0) s_m0 = p;
  }
  __syncthreads();
  const uint64_t M0 = s_m0;
  constexpr int DTBLK = GeoD<T, B>::TBLK;  // index entries per decode tile
  if ((k0 % DTBLK) == 0 && k0 < a.nblk) {
    a.index[2 * (k0 / DTBLK)] = R0 + rex;
    a.index[2 * (k0 / DTBLK) + 1] = M0 + mex;
  }
  if (t == ntiles - 1 && threadIdx.x == 0) {
    if (R0 + tnc != h.n_nc || M0 + tmid != h.mid_total) bad = true;
    // the end of the last decode tile
    a.index[2 * cdiv(a.nblk, DTBLK)] = h.n_nc;
    a.index[2 * cdiv(a.nblk, DTBLK) + 1] = h.mid_total;
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicMax(a.status, kStatusCorrupt);
}

template <typename T, int B>
__global__ __launch_bounds__(256) void k_dindex(DBatch b) {
  __shared__ uint32_t s_scan[2 * kWavesPerWG];
  __shared__ uint64_t s_r0, s_m0;
  __shared__ int s_flag;
  const uint64_t g = blockIdx.x;
  const FieldD f = field_at(b, dfield_of(b.field_idx[Traits<T>::BYTES / 8], g));
  dindex_tile<T, B>(b, f, (uint32_t)(g - f.base_idx), s_scan, &s_r0, &s_m0, &s_flag);
}

template <typename T, int B>
__device__ __forceinline__ void decode_tile(const FieldD& a, uint32_t t, uint32_t* s_scan, uint32_t* s_stage) {
  using U = typename Traits<T>::U;
  using G = GeoD<T, B>;
  constexpr int EPL = G::EPL, LPB = G::LPB, TB = G::TB, SUB = G::SUB, TBLK = G::TBLK;
  constexpr int BYTES = Traits<T>::BYTES;

  const StreamInfo h = read_header<BYTES, B>(a);
  if (!h.ok) return;  // k_dindex reported it
  const uint32_t ntiles = (uint32_t)cdiv(a.nblk, TBLK);
  if (t >= ntiles) return;
  const uint8_t* in = a.in;
  const int g = threadIdx.x / LPB, lig = threadIdx.x % LPB;
  const int lane = lane_id();
  const T* mus = reinterpret_cast<const T*>(in + h.sec.mu);
  T* y = reinterpret_cast<T*>(a.out);
  bool bad = false;

  // the tile's mid bytes: [m0, m1) of the mid section, staged as soon as known
  const uint64_t r0 = a.index[2 * t];
  const uint64_t m0 = a.index[2 * t + 1];
  uint64_t m1 = a.index[2 * t + 3];
  if (m1 < m0 || m1 - m0 > (uint64_t)G::TILE * SUB * BYTES) {
    bad = true;
    m1 = m0;
  }
  const uint32_t tile_bytes = (uint32_t)(m1 - m0);
  const uint64_t src = h.sec.mid + m0;
  const uint32_t st = (uint32_t)(src & 15u);
  {
    // 64-bit positions stay with the tile (wave-uniform); lanes use 32-bit
    // offsets from them
    const uint64_t src0 = src - st;
    const uint8_t* base = in + src0;
    const uint64_t left = a.in_bytes > src0 ? a.in_bytes - src0 : 0;
    const uint32_t avail = (uint32_t)std::min<uint64_t>(left, 0xFFFFFFFFull);
    const uint32_t nchunk = (st + tile_bytes + 15) / 16;
    // every chunk of this thread's loads first, then the one chunk that
    // holds the stream's end byte by byte (no read past in_bytes), then the
    // stores to LDS: loads return in order, so a store waiting on its chunk
    // between loads would hold back the next chunk's load
    constexpr uint32_t NCH = ((15u + (uint32_t)(G::TILE * G::SUB * BYTES) + 15u) / 16u + kWG - 1u) / kWG;
    uint4 u[NCH];
#pragma unroll
    for (uint32_t j = 0; j < NCH; ++j) {
      const uint32_t ch = threadIdx.x + j * kWG;
      u[j] = make_uint4(0, 0, 0, 0);
      if (ch < nchunk && ch * 16 + 16 <= avail) u[j] = *reinterpret_cast<const uint4*>(base + ch * 16);
    }
#pragma unroll
    for (uint32_t j = 0; j < NCH; ++j) {
      const uint32_t ch = threadIdx.x + j * kWG;
      if (ch < nchunk && ch * 16 + 16 > avail) {
        const uint32_t off = ch * 16;
        uint32_t wv[4] = {0, 0, 0, 0};
        for (uint32_t bq = 0; bq < 16; ++bq)
          if (off + bq < avail) wv[bq >> 2] |= (uint32_t)base[off + bq] << ((bq & 3) * 8);
        u[j] = make_uint4(wv[0], wv[1], wv[2], wv[3]);
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < NCH; ++j) {
      const uint32_t ch = threadIdx.x + j * kWG;
      if (ch < nchunk) reinterpret_cast<uint4*>(s_stage)[ch] = u[j];
    }
  }

  // the tile's first block and value (wave-uniform), its block and value
  // counts; lanes index from them with 32-bit offsets
  const uint64_t kb = (uint64_t)t * TBLK;
  const uint32_t nblk_t = (uint32_t)std::min<uint64_t>(a.nblk - kb, (uint64_t)TBLK);
  const uint32_t nval_t = (uint32_t)std::min<uint64_t>(a.n - kb * B, (uint64_t)TBLK * B);
  const uint8_t* state_t = in + h.sec.state + (kb >> 3);  // a tile owns whole state bytes
  const T* mus_t = mus + kb;
  T* y_t = y + kb * B;

  // ranks of the tile's non-constant blocks, their K bytes and codes
  bool nc[SUB];
  int cnt[SUB];
  uint32_t first_of[SUB];
  T mu[SUB];
  // every row's state byte and mu load before any is used (loads return in
  // order: a row's loads issued after the previous row's use would wait)
  uint32_t sbyte[SUB];
#pragma unroll
  for (int s = 0; s < SUB; ++s) {
    const uint32_t lk = (uint32_t)(s * TB + g);
    sbyte[s] = 0;
    mu[s] = (T)0;
    if (lk < nblk_t) {
      sbyte[s] = state_t[lk >> 3];
      mu[s] = mus_t[lk];
    }
  }
#pragma unroll
  for (int s = 0; s < SUB; ++s) {
    const uint32_t lk = (uint32_t)(s * TB + g);
    const bool inb = lk < nblk_t;
    nc[s] = inb && ((sbyte[s] >> (lk & 7)) & 1u);
    // values from this lane's first one to the tile's end
    const int rem = (int)nval_t - (int)(lk * B) - lig * EPL;
    cnt[s] = inb ? (rem < 0 ? 0 : (rem > EPL ? EPL : rem)) : 0;
    first_of[s] = (lig == 0 && nc[s]) ? 1u : 0u;
  }
  uint32_t rk[SUB], rtot[SUB];
  wg_excl_scan_multi<SUB>(first_of, rk, rtot, s_scan);
  int Ks[SUB];       // kept bits; -1 raw; 0 constant or unusable
  uint32_t cw[SUB];  // this lane's EPL codes, first value in the top bits
  uint32_t nbytes[SUB];
  // ranks from r0 on, 32-bit within the tile
  const uint32_t nnc_t = (uint32_t)std::min<uint64_t>(h.n_nc > r0 ? h.n_nc - r0 : 0, (uint64_t)TBLK);
  const uint8_t* kbytes_t = in + h.sec.kbytes + r0;
  const uint8_t* codes_t = in + h.sec.codes + r0 * (B / 4);
  // every row's K byte and codes first (loads return in order: a row's
  // loads issued after the previous row's use would wait on them)
  uint32_t kraw[SUB], craw[SUB];
#pragma unroll
  for (int s = 0; s < SUB; ++s) {
    const uint32_t rl = rk[s] - ((lig != 0 && nc[s]) ? 1u : 0u);
    const bool have = nc[s] && rl < nnc_t;
    kraw[s] = have ? (uint32_t)kbytes_t[rl] : 0u;
    craw[s] = 0;
    if (have) {  // loaded beside K, used only for a coded block
      const uint8_t* cp = codes_t + rl * (B / 4) + (uint32_t)lig * (EPL / 4);
      if constexpr (EPL == 8) {
        craw[s] = *reinterpret_cast<const uint16_t*>(cp);  // byte order fixed below
      } else {
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) c = (c << 8) | cp[j];
        craw[s] = c;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < SUB; ++s) {
    // the group's first lane counted its block; the others see it counted
    const uint32_t rl = rk[s] - ((lig != 0 && nc[s]) ? 1u : 0u);
    const bool have = nc[s] && rl < nnc_t;
    bad = bad || (nc[s] && rl >= nnc_t);
    int K = (int)kraw[s];
    if (K == kRawK) {
      K = -1;
    } else if (have && (K < Traits<T>::KMIN || K > Traits<T>::W)) {
      bad = true;
      K = 0;
    }
    const int nb = K > 0 ? bytes_of(K) : 0;
    uint32_t c = craw[s];
    if constexpr (EPL == 8) c = ((c & 0xFFu) << 8) | (c >> 8);
    // stored bytes of the lane: nb per live value less its code. Codes of
    // values past the end are cleared; a code above nb marks the stream bad
    // and its row is then read as if all codes were 0, which keeps every
    // offset within the stage.
    const int cn = cnt[s];
    uint32_t lb = 0;
    if (K > 0) {
      c &= (uint32_t)(((1ull << (2 * cn)) - 1) << (2 * (EPL - cn)));
      const uint32_t hi = c & 0xAAAAAAAAu, lo = c & 0x55555555u;
      const bool over = (nb == 1 && hi != 0) || (nb == 2 && (lo & (hi >> 1)) != 0);
      bad = bad || over;
      c = over ? 0u : c;
      lb = (uint32_t)(nb * cn) - (uint32_t)(__popc(c & 0x55555555u) + 2 * __popc(c & 0xAAAAAAAAu));
    } else {
      c = 0;
      lb = K < 0 ? (uint32_t)(BYTES * cn) : 0u;
    }
    Ks[s] = K;
    cw[s] = c;
    nbytes[s] = lb;
  }
  uint32_t off[SUB], tot[SUB];
  wg_excl_scan_multi<SUB>(nbytes, off, tot, s_scan);  // its barriers also cover the staging
  uint32_t sum = 0;
#pragma unroll
  for (int s = 0; s < SUB; ++s) sum += tot[s];
  if (sum != tile_bytes) bad = true;

  // values, row by row
#pragma unroll
  for (int s = 0; s < SUB; ++s) {
    const int K = Ks[s];
    T v[EPL];
    uint32_t o = st + off[s];
    // Reads of the stage go unguarded: a lane starts at most at the end of
    // the tile's stored bytes and advances at most a word per value, which
    // the stage's size allows for. Values past the end of a short block read
    // whatever lies there and are not stored; being last in their lane and
    // block, they only reach other such values.
    if (K == 0) {  // constant: mu
#pragma unroll
      for (int i = 0; i < EPL; ++i) v[i] = mu[s];
    } else if (K < 0) {  // raw: the stored words
#pragma unroll
      for (int i = 0; i < EPL; ++i) v[i] = from_bits<T>(lds_get<U>(s_stage, o + (uint32_t)(i * BYTES)));
    } else {
      const int nb = bytes_of(K);
      const int sh = shift_of(K);
      const U keep = top_bytes_mask<U>(nb);
      U q0[EPL];
      uint32_t cmin[EPL];
      U run = 0;
      uint32_t cm = 3;
#pragma unroll
      for (int i = 0; i < EPL; ++i) {
        // ci <= nb here (checked above), so the value stores nb - ci bytes
        const uint32_t ci = (cw[s] >> (2 * (EPL - 1 - i))) & 3u;
        const uint32_t s8 = ci << 3;
        // the word at o holds this value's stored bytes, then whatever
        // follows; after the shift and byte swap those land below the kept
        // bytes, where `keep` clears them at the end (ci <= 3: shift < 32)
        const U got = lds_get<U>(s_stage, o);
        o += (uint32_t)nb - ci;
        const U stored = byte_swap((U)(got << s8));
        run = (run & top_bytes_of<U>(s8)) | stored;
        cm = ci < cm ? ci : cm;
        q0[i] = run;
        cmin[i] = cm;
      }
      // carry of the leading bytes from the lanes before this one in the
      // block; bytes below the kept ones never reach a kept byte (every mask
      // here keeps at most the top min(3, nb) bytes of a live value)
      uint32_t pk = top24<U>(run) | cm;
      {
        uint32_t o2 = lane_up<LPB, 1>(pk);
        pk = lig >= 1 ? lead_compose(o2, pk) : pk;
        if constexpr (LPB > 2) {
          o2 = lane_up<LPB, 2>(pk);
          pk = lig >= 2 ? lead_compose(o2, pk) : pk;
        }
        if constexpr (LPB > 4) {
          o2 = lane_up<LPB, 4>(pk);
          pk = lig >= 4 ? lead_compose(o2, pk) : pk;
        }
        if constexpr (LPB > 8) {
          o2 = lane_up<LPB, 8>(pk);
          pk = lig >= 8 ? lead_compose(o2, pk) : pk;
        }
        if constexpr (LPB > 16) {
          o2 = __shfl_up(pk, 16, LPB);
          pk = lig >= 16 ? lead_compose(o2, pk) : pk;
        }
        if constexpr (LPB > 32) {
          o2 = __shfl_up(pk, 32, LPB);
          pk = lig >= 32 ? lead_compose(o2, pk) : pk;
        }
      }
      uint32_t carry = LPB > 1 ? lane_up<LPB, 1>(pk) & 0xFFFFFF00u : 0u;
      carry = lig == 0 ? 0u : carry;
      const U cfull = from_top24<U>(carry);
#pragma unroll
      for (int i = 0; i < EPL; ++i) {
        const U qi = (q0[i] | (cfull & top_bytes_of<U>(cmin[i] << 3))) & keep;
        v[i] = mu[s] + from_bits<T>((U)(qi << sh));
      }
    }
    if constexpr (sizeof(T) == 8 && SUB == 1) {
      // float64 tiles of one row: the values pass through the stage so that
      // every store of a wave covers 1 KiB of the row without gaps and can
      // stream past the caches. Value i of thread L (row value L EPL + i)
      // sits at stage slot i kWG + L: the writes of a wave fill consecutive
      // slots (no bank conflicts; lane-major slots put 64 lanes on two banks)
      __syncthreads();  // every lane is done with the staged mid bytes
      T* sv = reinterpret_cast<T*>(s_stage);
#pragma unroll
      for (int i = 0; i < EPL; ++i) sv[i * kWG + threadIdx.x] = v[i];
      __syncthreads();
      using v4u = unsigned int __attribute__((ext_vector_type(4)));
      for (uint32_t c = threadIdx.x; c < (uint32_t)G::TILE / 2; c += kWG) {
        const uint32_t i0 = 2 * c;  // row values i0 and i0 + 1 (EPL is even)
        const uint32_t slot = (i0 % EPL) * kWG + i0 / EPL;
        if (i0 + 2 <= nval_t) {
          const uint64_t a = (uint64_t)__double_as_longlong(sv[slot]);
          const uint64_t b = (uint64_t)__double_as_longlong(sv[slot + kWG]);
          const v4u nv = {(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
          __builtin_nontemporal_store(nv, reinterpret_cast<v4u*>(y_t + i0));
        } else if (i0 < nval_t) {
          y_t[i0] = sv[slot];
        }
      }
    } else {
      if (cnt[s] > 0) store_run<T, EPL>(y_t, (uint32_t)((s * TB + g) * B + lig * EPL), cnt[s], v);
    }
  }
  if (__ballot(bad) != 0 && lane == 0) atomicMax(a.status, kStatusCorrupt);
}

template <typename T, int B>
__global__ __launch_bounds__(256) void k_decode(DBatch b) {
  using G = GeoD<T, B>;
  __shared__ uint32_t s_scan[G::SUB * kWavesPerWG];
  __shared__ __align__(16) uint32_t s_stage[dec_stage_words<T, B>()];
  const uint64_t g = blockIdx.x;
  const FieldD f = field_at(b, dfield_of(b.field_dec[Traits<T>::BYTES / 8], g));
  decode_tile<T, B>(f, (uint32_t)(g - f.base_dec), s_scan, s_stage);
  // the call's last decode launch advances the gate's epoch (no index tile
  // reads it any more); at the end, so that no load comes after the atomic
  if (g == 0 && threadIdx.x == 0 && (sizeof(T) == 8 || b.tiles_dec[1] == 0))
    __hip_atomic_fetch_add((__attribute__((address_space(1))) uint64_t*)(as_global(b.gate) + kGateEpochWord), 1ull,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- launch ---

template <int B>
hipError_t launch_decompress_b(const DBatch& b, hipStream_t stream, TimerHook hook) {
  auto run = [&](const char* name, auto&& fn) {
    if (hook) hook(name, stream, 1);
    fn();
    if (hook) hook(name, stream, 0);
  };
  // the index pass clears what it needs itself (its gate); a call without
  // index tiles only has status words to set
  if (b.tiles_idx[0] + b.tiles_idx[1] == 0) {
    const uint64_t nf = b.fields ? b.nfields : 1;
    const uint32_t gi = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cdiv(nf, 256), 1024));
    run("k_dinit", [&] { k_dinit<<<gi, 256, 0, stream>>>(b); });
  }
  if (b.tiles_idx[0]) run("k_dindex", [&] { k_dindex<float, B><<<(uint32_t)b.tiles_idx[0], 256, 0, stream>>>(b); });
  if (b.tiles_idx[1]) run("k_dindex", [&] { k_dindex<double, B><<<(uint32_t)b.tiles_idx[1], 256, 0, stream>>>(b); });
  if (b.tiles_dec[0]) run("k_decode", [&] { k_decode<float, B><<<(uint32_t)b.tiles_dec[0], 256, 0, stream>>>(b); });
  if (b.tiles_dec[1]) run("k_decode", [&] { k_decode<double, B><<<(uint32_t)b.tiles_dec[1], 256, 0, stream>>>(b); });
  return hipGetLastError();
}

hipError_t launch_decompress(const DBatch& b, uint32_t block, hipStream_t stream, TimerHook hook) {
  switch (block) {
    case 8: return launch_decompress_b<8>(b, stream, hook);
    case 16: return launch_decompress_b<16>(b, stream, hook);
    case 32: return launch_decompress_b<32>(b, stream, hook);
    case 64: return launch_decompress_b<64>(b, stream, hook);
    case 128: return launch_decompress_b<128>(b, stream, hook);
    case 256: return launch_decompress_b<256>(b, stream, hook);
    case 512: return launch_decompress_b<512>(b, stream, hook);
    case 1024: return launch_decompress_b<1024>(b, stream, hook);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace szx
