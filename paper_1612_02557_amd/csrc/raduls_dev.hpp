// raduls_dev.hpp -- device-side building blocks shared by the sort kernels.
//
// Records are rec_bytes = 4*RW bytes; the key is the little-endian unsigned
// integer of the first key_bytes bytes (paper, Sec. 1: keys are strings of
// base-R digits; Sec. 4: key followed by data).  A key is held as two 64-bit
// words (lo = bytes 0..7, hi = bytes 8..15), masked to key_bytes.
//
// Digits are taken most significant first.  A bucket carries `bit`, the
// number of leading key bits already resolved; its next digit of width d is
// floor(key / 2^(KB - bit - d)) mod 2^d with KB = 8*key_bytes (the paper's
// current_byte, Sec. 3.2-3.4, generalised to bit positions so that a bucket
// can skip bits that all its keys share).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "raduls_plan.hpp"

namespace rd {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));

constexpr int WG = 256;         // threads of every sort workgroup
constexpr int NWAVES = WG / 64; // wavefronts per workgroup

struct Key {
  uint64_t lo, hi;
};

template <int RW>
struct Rec {
  uint32_t w[RW];
};

// ---- record access --------------------------------------------------------

template <int RW>
__device__ __forceinline__ Rec<RW> load_rec(const uint8_t* __restrict__ base, uint64_t i) {
  Rec<RW> r;
  const uint8_t* p = base + i * (uint64_t)(RW * 4);
  if constexpr (RW % 4 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 4; j++) {
      v4u v = reinterpret_cast<const v4u*>(p)[j];
      r.w[4 * j + 0] = v.x; r.w[4 * j + 1] = v.y; r.w[4 * j + 2] = v.z; r.w[4 * j + 3] = v.w;
    }
  } else if constexpr (RW % 2 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 2; j++) {
      v2u v = reinterpret_cast<const v2u*>(p)[j];
      r.w[2 * j + 0] = v.x; r.w[2 * j + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < RW; j++) r.w[j] = reinterpret_cast<const uint32_t*>(p)[j];
  }
  return r;
}

template <int RW>
__device__ __forceinline__ void store_rec(uint8_t* __restrict__ base, uint64_t i, const Rec<RW>& r,
                                          bool nt) {
  uint8_t* p = base + i * (uint64_t)(RW * 4);
  if constexpr (RW % 4 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 4; j++) {
      v4u v = {r.w[4 * j + 0], r.w[4 * j + 1], r.w[4 * j + 2], r.w[4 * j + 3]};
      v4u* q = reinterpret_cast<v4u*>(p) + j;
      if (nt) __builtin_nontemporal_store(v, q); else *q = v;
    }
  } else if constexpr (RW % 2 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 2; j++) {
      v2u v = {r.w[2 * j + 0], r.w[2 * j + 1]};
      v2u* q = reinterpret_cast<v2u*>(p) + j;
      if (nt) __builtin_nontemporal_store(v, q); else *q = v;
    }
  } else {
#pragma unroll
    for (int j = 0; j < RW; j++) {
      uint32_t* q = reinterpret_cast<uint32_t*>(p) + j;
      if (nt) __builtin_nontemporal_store(r.w[j], q); else *q = r.w[j];
    }
  }
}

// LDS copies of records (word arrays, record i at words [i*RW, i*RW+RW)).
template <int RW>
__device__ __forceinline__ void lds_put(uint32_t* s, uint32_t i, const Rec<RW>& r) {
  uint32_t* p = s + i * RW;
  if constexpr (RW % 4 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 4; j++)
      reinterpret_cast<v4u*>(p)[j] = v4u{r.w[4 * j], r.w[4 * j + 1], r.w[4 * j + 2], r.w[4 * j + 3]};
  } else if constexpr (RW % 2 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 2; j++) reinterpret_cast<v2u*>(p)[j] = v2u{r.w[2 * j], r.w[2 * j + 1]};
  } else {
#pragma unroll
    for (int j = 0; j < RW; j++) p[j] = r.w[j];
  }
}

template <int RW>
__device__ __forceinline__ Rec<RW> lds_get(const uint32_t* s, uint32_t i) {
  Rec<RW> r;
  const uint32_t* p = s + i * RW;
  if constexpr (RW % 4 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 4; j++) {
      v4u v = reinterpret_cast<const v4u*>(p)[j];
      r.w[4 * j] = v.x; r.w[4 * j + 1] = v.y; r.w[4 * j + 2] = v.z; r.w[4 * j + 3] = v.w;
    }
  } else if constexpr (RW % 2 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 2; j++) {
      v2u v = reinterpret_cast<const v2u*>(p)[j];
      r.w[2 * j] = v.x; r.w[2 * j + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < RW; j++) r.w[j] = p[j];
  }
  return r;
}

// Buffer access to a range of records: a resource over the range's bytes
// (wave-uniform base), one VGPR offset per thread and the record slot in the
// scalar offset, so that holding many records costs no address registers;
// offsets past the range read 0 and their stores are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t job_rsrc(const uint8_t* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(base), (short)0, (int)bytes, 0x00020000);
}

template <int RW>
__device__ __forceinline__ Rec<RW> buf_load_rec(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  Rec<RW> r;
  if constexpr (RW % 4 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 4; j++) {
      const v4u v = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff + 16 * j, (int)soff, 0));
      r.w[4 * j] = v.x; r.w[4 * j + 1] = v.y; r.w[4 * j + 2] = v.z; r.w[4 * j + 3] = v.w;
    }
  } else if constexpr (RW % 2 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 2; j++) {
      const v2u v = __builtin_bit_cast(v2u, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff + 8 * j, (int)soff, 0));
      r.w[2 * j] = v.x; r.w[2 * j + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < RW; j++) r.w[j] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff + 4 * j, (int)soff, 0);
  }
  return r;
}

template <int RW>
__device__ __forceinline__ void buf_store_rec(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, const Rec<RW>& r) {
  if constexpr (RW % 4 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 4; j++) {
      const v4u v = {r.w[4 * j], r.w[4 * j + 1], r.w[4 * j + 2], r.w[4 * j + 3]};
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned int, v), rs,
                                             (int)voff + 16 * j, (int)soff, 0);
    }
  } else if constexpr (RW % 2 == 0) {
#pragma unroll
    for (int j = 0; j < RW / 2; j++) {
      const v2u v = {r.w[2 * j], r.w[2 * j + 1]};
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned int, v), rs,
                                            (int)voff + 8 * j, (int)soff, 0);
    }
  } else {
#pragma unroll
    for (int j = 0; j < RW; j++) __builtin_amdgcn_raw_buffer_store_b32(r.w[j], rs, (int)voff + 4 * j, (int)soff, 0);
  }
}

__device__ __forceinline__ uint32_t uniform32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  return (uint64_t)uniform32((uint32_t)x) | ((uint64_t)uniform32((uint32_t)(x >> 32)) << 32);
}

// ---- keys and digits ------------------------------------------------------

struct KeyFmt {
  uint64_t mlo, mhi;  // masks keeping key bytes only
  uint32_t kbits;     // 8 * key_bytes
};

__host__ __device__ inline KeyFmt make_keyfmt(uint32_t key_bytes) {
  KeyFmt f;
  f.kbits = 8 * key_bytes;
  f.mlo = key_bytes >= 8 ? ~0ull : ((1ull << (8 * key_bytes)) - 1);
  f.mhi = key_bytes <= 8 ? 0ull : (key_bytes >= 16 ? ~0ull : ((1ull << (8 * (key_bytes - 8))) - 1));
  return f;
}

template <int RW>
__device__ __forceinline__ Key rec_key(const Rec<RW>& r, const KeyFmt& f) {
  uint64_t lo = r.w[0];
  if constexpr (RW > 1) lo |= (uint64_t)r.w[1] << 32;
  uint64_t hi = 0;
  if constexpr (RW > 2) hi = r.w[2];
  if constexpr (RW > 3) hi |= (uint64_t)r.w[3] << 32;
  return Key{lo & f.mlo, hi & f.mhi};
}

// ---- key-only loads ------------------------------------------------------
// Key-only loads (the histogram needs no payload).
template <int RW>
__device__ __forceinline__ Key load_key(const uint8_t* __restrict__ base, uint64_t i, const KeyFmt& f) {
  const uint8_t* q = base + i * (uint64_t)(RW * 4);
  uint64_t lo = 0, hi = 0;
  if constexpr (RW % 2 == 0) {
    v2u a = reinterpret_cast<const v2u*>(q)[0];
    lo = a.x | ((uint64_t)a.y << 32);
    if constexpr (RW >= 4) {
      if (f.mhi) {
        v2u b = reinterpret_cast<const v2u*>(q)[1];
        hi = b.x | ((uint64_t)b.y << 32);
      }
    }
  } else {
    const uint32_t* u = reinterpret_cast<const uint32_t*>(q);
    lo = u[0];
    if constexpr (RW > 1) lo |= (uint64_t)u[1] << 32;
    if constexpr (RW > 2) { if (f.mhi) hi = u[2]; }
    if constexpr (RW > 3) { if (f.mhi) hi |= (uint64_t)u[3] << 32; }
  }
  return Key{lo & f.mlo, hi & f.mhi};
}

// The key of a record through a buffer resource (record at voff + soff);
// WIDE: keys may be longer than 8 bytes (else the high word is not loaded).
template <int RW, bool WIDE = true>
__device__ __forceinline__ Key buf_load_key(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, const KeyFmt& f) {
  uint64_t lo = 0, hi = 0;
  if constexpr (RW % 2 == 0) {
    const v2u a = __builtin_bit_cast(v2u, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
    lo = a.x | ((uint64_t)a.y << 32);
    if constexpr (RW >= 4 && WIDE) {
      if (f.mhi) {
        const v2u b = __builtin_bit_cast(v2u, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff + 8, (int)soff, 0));
        hi = b.x | ((uint64_t)b.y << 32);
      }
    }
  } else {
    lo = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, 0);
    if constexpr (RW > 1) lo |= (uint64_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff + 4, (int)soff, 0) << 32;
    if constexpr (RW > 2 && WIDE) {
      if (f.mhi) hi = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff + 8, (int)soff, 0);
    }
    if constexpr (RW > 3 && WIDE) {
      if (f.mhi) hi |= (uint64_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff + 12, (int)soff, 0) << 32;
    }
  }
  return Key{lo & f.mlo, WIDE ? (hi & f.mhi) : 0ull};
}

__device__ __forceinline__ uint64_t shr128_lo(Key k, uint32_t s) {
  if (s >= 64) return k.hi >> (s - 64);
  if (s == 0) return k.lo;
  return (k.lo >> s) | (k.hi << (64 - s));
}

// Digit of width d whose lowest bit is `shift` (d <= 16).  Keys of at most
// 64 bits (the key format is the same for the whole launch) need one shift.
__device__ __forceinline__ uint32_t key_digit(Key k, uint32_t shift, uint32_t mask, const KeyFmt& f) {
  if (f.kbits <= 64) return (uint32_t)(k.lo >> shift) & mask;
  return (uint32_t)shr128_lo(k, shift) & mask;
}

__device__ __forceinline__ bool key_less(Key a, Key b) {
  return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

// Number of leading bits (of the KB-bit key) shared by all keys whose XOR
// with a reference key OR-accumulates to v.  v == 0 means all keys equal.
__device__ __forceinline__ uint32_t common_prefix_bits(Key v, uint32_t kbits) {
  uint32_t lz;
  if (v.hi) lz = __clzll(v.hi);
  else if (v.lo) lz = 64 + __clzll(v.lo);
  else return kbits;
  return lz - (128 - kbits);
}

// ---- wavefront helpers ----------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  uint32_t l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Lanes of the wave (among `active`) holding the same digit value v (d bits):
// per bit, the lanes whose bit agrees with this lane's (the ballot, or its
// complement where this lane's bit is 0: ballot XOR (bit - 1)).
template <uint32_t D>
__device__ __forceinline__ uint64_t match_digit_n(uint32_t v, uint64_t active) {
  uint64_t peers = active;
#pragma unroll
  for (uint32_t b = 0; b < D; b++) {
    const uint32_t bit = (v >> b) & 1u;
    peers &= __ballot(bit) ^ ((uint64_t)bit - 1ull);
  }
  return peers;
}
__device__ __forceinline__ uint64_t match_digit(uint32_t v, uint32_t d, uint64_t active) {
  if (d == 8) return match_digit_n<8>(v, active);
  uint64_t peers = active;
  for (uint32_t b = 0; b < d; b++) {
    const uint32_t bit = (v >> b) & 1u;
    peers &= __ballot(bit) ^ ((uint64_t)bit - 1ull);
  }
  return peers;
}

// Stable rank among equal digits, in two steps so that the LDS round trips
// of several rounds overlap.  rank_issue: the lanes holding digit v in this
// round ("peers") elect their lowest lane, which adds the peer count to the
// wave's running counter wc[v] and keeps the old value; rank_finish: every
// peer reads its leader's old value, so rank = (digit v in earlier rounds) +
// (peers in lower lanes).  Rounds must be issued in order.
struct RankPart {
  uint32_t old;    // counter before this round (leader lanes)
  uint32_t info;   // lower 16 bits: peers below this lane; upper: leader lane
};

__device__ __forceinline__ RankPart rank_issue(uint32_t* wc, uint32_t v, uint32_t d, bool valid) {
  uint64_t active = __ballot(valid);
  uint64_t peers = match_digit(v, d, active);
  uint32_t lane = __lane_id();
  uint32_t leader = valid ? (uint32_t)(__ffsll((long long)peers) - 1) : lane;
  uint32_t old = 0;
  if (valid && leader == lane) old = atomicAdd(&wc[v], (uint32_t)__popcll(peers));
  uint64_t below = lane == 0 ? 0ull : (peers & (~0ull >> (64 - lane)));
  return RankPart{old, (uint32_t)__popcll(below) | (leader << 16)};
}

__device__ __forceinline__ uint32_t rank_finish(RankPart r) {
  uint32_t base = __shfl(r.old, (int)(r.info >> 16));
  return base + (r.info & 0xFFFFu);
}

// The same with the round's state in one register: the counter's old value
// (valid in the leader lane, below 2^16) | peers below this lane << 16 |
// leader lane << 24.
__device__ __forceinline__ uint32_t rank_issue32(uint32_t* wc, uint32_t v, uint32_t d, bool valid) {
  const uint64_t active = __ballot(valid);
  const uint64_t peers = match_digit(v, d, active);
  const uint32_t lane = __lane_id();
  const uint32_t leader = valid ? (uint32_t)(__ffsll((long long)peers) - 1) : lane;
  uint32_t old = 0;
  if (valid && leader == lane) old = atomicAdd(&wc[v], (uint32_t)__popcll(peers));
  const uint64_t below = lane == 0 ? 0ull : (peers & (~0ull >> (64 - lane)));
  return old | ((uint32_t)__popcll(below) << 16) | (leader << 24);
}

__device__ __forceinline__ uint32_t rank_finish32(uint32_t x) {
  const uint32_t base = (uint32_t)__shfl((int)x, (int)(x >> 24)) & 0xFFFFu;
  return base + ((x >> 16) & 0xFFu);
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x |= __shfl_xor(x, o);
  return x;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Exclusive prefix sum over a wave (Hillis-Steele on 64 lanes).
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t* total) {
  uint32_t l = lane_id();
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(inc, o);
    if (l >= (uint32_t)o) inc += y;
  }
  *total = __shfl(inc, 63);
  return inc - x;
}

// Block-wide exclusive scan of `count` uint32 values in LDS (in place),
// count <= 16 * WG.  Uses `tmp` (NWAVES words of LDS).  Returns the total.
// Two barriers: every thread adds up the wave totals before its own.
__device__ __forceinline__ uint32_t block_excl_scan_lds(uint32_t* a, uint32_t count, uint32_t* tmp) {
  const uint32_t t = threadIdx.x;
  const uint32_t per = (count + WG - 1) / WG;  // contiguous run per thread
  uint32_t lo = min(count, t * per), hi = min(lo + per, count);
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; i++) s += a[i];
  uint32_t wtot;
  uint32_t ex = wave_excl_scan(s, &wtot);
  if (lane_id() == 0) tmp[t / 64] = wtot;
  __syncthreads();
  uint32_t base = 0, total = 0;
#pragma unroll
  for (uint32_t w = 0; w < NWAVES; w++) {
    const uint32_t x = tmp[w];
    base += w < t / 64 ? x : 0u;
    total += x;
  }
  uint32_t run = base + ex;
  for (uint32_t i = lo; i < hi; i++) { uint32_t c = a[i]; a[i] = run; run += c; }
  __syncthreads();
  return total;
}

// ---- bucket descriptors ---------------------------------------------------

// Tiny bucket (2..63 records) packed into one word:
//   begin (40 bits) | count (6) << 40 | in-tmp (1) << 46 | bit (8) << 47
__device__ __forceinline__ uint64_t pack_tiny(uint64_t begin, uint32_t count, uint32_t tmp, uint32_t bit) {
  return begin | ((uint64_t)count << 40) | ((uint64_t)tmp << 46) | ((uint64_t)bit << 47);
}

// ---- finishing jobs ---------------------------------------------------------

// Index bits of a job of m >= 2 records.
__device__ __forceinline__ uint32_t index_bits(uint64_t m) { return 64u - (uint32_t)__clzll(m - 1); }

// Key bits a finishing job of the register kernel keeps below its digit when
// `bit` leading bits are resolved (its keys share them): what is left after
// the FIN_DIGIT_BITS digit.  With the index bits they must fit the
// composite (64 bits, or 128 for keys above 8 bytes).
__device__ __forceinline__ bool fin_fits(uint64_t m, uint32_t bit, uint32_t kbits) {
  const uint32_t rem = kbits - bit;
  const uint32_t below = rem > FIN_DIGIT_BITS ? rem - FIN_DIGIT_BITS : 0u;
  return below + index_bits(m) <= fin_comp_bits(kbits);
}

// Can a bucket (or a group of consecutive children) of m records with `bit`
// resolved bits be a finishing job of the plan's job kernel?
__device__ __forceinline__ bool job_ok(const Plan& p, uint64_t m, uint32_t bit, uint32_t kbits) {
  if (m <= TINY_MAX || bit >= kbits) return false;
  if (!p.fin_max) return m <= p.c_fin;
  return m <= p.fin_max && fin_fits(m, bit, kbits);
}

// Largest finishing job whose keys share `bit` leading bits.
__device__ __forceinline__ uint64_t job_cap(const Plan& p, uint32_t bit, uint32_t kbits) {
  if (!p.fin_max) return p.c_fin;
  const uint32_t rem = kbits - bit;
  const uint32_t below = rem > FIN_DIGIT_BITS ? rem - FIN_DIGIT_BITS : 0u;
  const uint32_t ibmax = fin_comp_bits(kbits) - below;  // at least 12
  return ibmax >= 32 ? (uint64_t)p.fin_max : min((uint64_t)p.fin_max, 1ull << ibmax);
}

// ---- look-back status words ----------------------------------------------
// epoch (22 bits) << 42 | flag (2) << 40 | value (40): flag 1 = the tile's own
// count (aggregate), flag 2 = the count of this and all earlier tiles of the
// bucket (inclusive prefix).  A word whose epoch is not the current level's
// is a leftover of an earlier level and reads as not ready.
constexpr uint32_t LB_EPOCH_SHIFT = 42;
constexpr uint64_t LB_AGG = 1ull << 40;
constexpr uint64_t LB_INC = 2ull << 40;
constexpr uint64_t LB_FLAGS = 3ull << 40;
constexpr uint64_t LB_VAL = (1ull << 40) - 1;

__device__ __forceinline__ uint64_t atomic_load_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Index of the list entry whose tile range holds `tile`: largest b with
// start[b] <= tile, b < nb (start is non-decreasing).
__device__ __forceinline__ uint32_t find_entry(const uint64_t* start, uint32_t nb, uint64_t tile) {
  uint32_t lo = 0, hi = nb;  // answer in [lo, hi)
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (start[mid] <= tile) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace rd
