// k_small.hip -- single-workgroup work: the bucket queue (paper, Sec. 3.4:
// small bins are handed out from a shared queue, largest first, and each is
// processed by one thread) and the finishing sorts of Sec. 3.5.
//
// A persistent grid takes buckets from the queue, largest size class first.
// A bucket larger than the LDS finishing capacity gets a one-workgroup radix
// pass (RADIX); its children are routed: at most 32 records -> one wavefront
// ranks them (RANK, the insertion-sort slot of Sec. 3.5); up to the LDS
// capacity -> the scheduler picks LSD, BITONIC or (one more) RADIX; larger ->
// the workgroup's own depth-first stack.  Small finishes run per wavefront
// (four at a time), larger ones use the whole workgroup.  Every procedure is
// stable, so the output does not depend on which one runs.
#include "raduls_dev.hpp"
#include "raduls_kernels.hpp"
#include "sched_dev.hpp"

namespace rd {

constexpr uint32_t RB = 256;          // radix of one-workgroup passes (d_block <= 8)
constexpr uint32_t MAX_ROUNDS = 16;   // LDS finishing capacity <= 16 * WG records
constexpr uint32_t WAVE_MAX = 256;    // largest bucket a wavefront finishes
constexpr uint32_t EMAX = WAVE_MAX / 64;

// child codes
constexpr uint32_t C_NONE = 0, C_WRANK = 1, C_WLSD = 2, C_WBIT = 3, C_GLSD = 4, C_GBIT = 5,
                   C_GRADIX = 6, C_PUSH = 7, C_GCOPY = 8, C_CF = 9;

struct SmallShared {
  uint32_t hist[RB];
  uint32_t run[RB];
  uint32_t wcnt[NWAVES * RB];
  uint32_t toff[RB + 1];
  uint32_t tcnt[RB];
  uint32_t scan_tmp[NWAVES + 1];
  uint64_t vary[2 * NWAVES];
  // child lists of up to two nested radix passes
  uint32_t cbase[2][RB];
  uint32_t ccnt[2][RB];
  uint32_t ccode[2][RB];
  uint32_t wlist[2][RB];
  uint32_t glist[2][RB];
  uint32_t wn[2], gn[2], wnext[2];
  uint32_t cbit[2];
  uint32_t cR[2];
  uint32_t ctmp[2];
  uint64_t cbegin[2];
  uint64_t cparent[2];
  uint32_t sp;
  uint32_t bcast;
  uint32_t decisions;
  Bucket item;
};

struct Ctx {
  Plan p;
  Work w;
  uint8_t* rec0;
  uint8_t* rec1;
  KeyFmt kf;
  SmallShared* S;
  uint32_t* dyn;     // dynamic LDS
  Bucket* stack;
  uint32_t ws;       // wavefront finishing capacity for this record size
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

template <int RW>
__device__ __forceinline__ Key lds_key(const uint32_t* stage, uint32_t i, const KeyFmt& f) {
  const uint32_t* q = stage + i * RW;
  uint64_t lo = q[0];
  if constexpr (RW > 1) lo |= (uint64_t)q[1] << 32;
  uint64_t hi = 0;
  if constexpr (RW > 2) hi = q[2];
  if constexpr (RW > 3) hi |= (uint64_t)q[3] << 32;
  return Key{lo & f.mlo, hi & f.mhi};
}

__device__ __forceinline__ uint32_t ctz128(Key v) {
  return v.lo ? (uint32_t)__builtin_ctzll(v.lo) : 64u + (uint32_t)__builtin_ctzll(v.hi);
}
__device__ __forceinline__ uint32_t bitlen128(Key v) {
  return v.hi ? 128u - (uint32_t)__clzll(v.hi) : (v.lo ? 64u - (uint32_t)__clzll(v.lo) : 0u);
}
// bits [s, s + n) of a 128-bit value as the low bits of a 128-bit result
__device__ __forceinline__ Key shr128(Key k, uint32_t s) {
  if (s == 0) return k;
  if (s >= 128) return Key{0, 0};
  if (s >= 64) return Key{k.hi >> (s - 64), 0};
  return Key{(k.lo >> s) | (k.hi << (64 - s)), k.hi >> s};
}
__device__ __forceinline__ Key shl128(Key k, uint32_t s) {
  if (s == 0) return k;
  if (s >= 64) return Key{0, k.lo << (s - 64)};
  return Key{k.lo << s, (k.hi << s) | (k.lo >> (64 - s))};
}
__device__ __forceinline__ Key mask128(Key k, uint32_t n) {
  if (n >= 128) return k;
  if (n >= 64) return Key{k.lo, n == 64 ? 0 : (k.hi & ((1ull << (n - 64)) - 1))};
  return Key{n == 0 ? 0 : (k.lo & ((1ull << n) - 1)), 0};
}

// ---------------------------------------------------------------------------
// Wavefront procedures (one wave, no workgroup barrier).

// RANK: position = number of keys that are smaller, or equal and earlier.
template <int RW>
__device__ void wave_rank(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp) {
  const uint32_t l = lane_id();
  const uint8_t* src = in_tmp ? c.rec1 : c.rec0;
  Rec<RW> r;
  Key k{~0ull, ~0ull};
  if (l < m) { r = load_rec<RW>(src, begin + l); k = rec_key<RW>(r, c.kf); }
  uint32_t rank = 0;
  for (uint32_t j = 0; j < m; j++) {
    uint64_t lo = __shfl(k.lo, j);
    uint64_t hi = __shfl(k.hi, j);
    rank += (hi < k.hi || (hi == k.hi && (lo < k.lo || (lo == k.lo && j < l)))) ? 1u : 0u;
  }
  if (l < m) store_rec<RW>(c.rec0, begin + rank, r, false);
}

// Composite sort key of a wave element: (varying key bits) << ib | index.
struct Comp {
  uint64_t lo, hi;
};
__device__ __forceinline__ bool comp_gt(Comp a, Comp b) { return a.hi > b.hi || (a.hi == b.hi && a.lo > b.lo); }

// LSD or BITONIC on m <= 64*EMAX records by one wave.  Records are staged in
// the wave's LDS region so the sorted order can be gathered from them.
template <int RW>
__device__ void wave_sort(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp, uint32_t proc, uint32_t* reg) {
  const uint32_t l = lane_id();
  const uint8_t* src = in_tmp ? c.rec1 : c.rec0;
  const uint32_t E = (m + 63) / 64;
  uint32_t* recs = reg;                                             // ws * RW words
  uint64_t* cl = reinterpret_cast<uint64_t*>(reg + c.ws * RW);      // ws comps (lo)
  uint64_t* ch = cl + c.ws;                                         // ws comps (hi)
  uint32_t* hist = reinterpret_cast<uint32_t*>(ch + c.ws);          // 256 counters
  Key key[EMAX];
#pragma unroll
  for (uint32_t e = 0; e < EMAX; e++) {
    uint32_t i = e * 64 + l;
    key[e] = Key{0, 0};
    if (e < E && i < m) {
      Rec<RW> r = load_rec<RW>(src, begin + i);
      lds_put<RW>(recs, i, r);
      key[e] = rec_key<RW>(r, c.kf);
    }
  }
  Key ref{__shfl(key[0].lo, 0), __shfl(key[0].hi, 0)};
  uint64_t vlo = 0, vhi = 0;
#pragma unroll
  for (uint32_t e = 0; e < EMAX; e++) {
    uint32_t i = e * 64 + l;
    if (e < E && i < m) { vlo |= key[e].lo ^ ref.lo; vhi |= key[e].hi ^ ref.hi; }
  }
  Key vary{wave_or64(vlo), wave_or64(vhi)};
  wave_lds_sync();
  if (vary.lo == 0 && vary.hi == 0) {
    // all keys equal: input order is the sorted order
    if (in_tmp) {
#pragma unroll
      for (uint32_t e = 0; e < EMAX; e++) {
        uint32_t i = e * 64 + l;
        if (e < E && i < m) store_rec<RW>(c.rec0, begin + i, lds_get<RW>(recs, i), false);
      }
    }
    return;
  }
  const uint32_t lo = ctz128(vary);
  const uint32_t wv = bitlen128(vary) - lo;
  const uint32_t ib = 32 - __clz(m - 1);
  Comp cp[EMAX];
#pragma unroll
  for (uint32_t e = 0; e < EMAX; e++) {
    uint32_t i = e * 64 + l;
    if (e < E && i < m) {
      Key v = shl128(mask128(shr128(key[e], lo), wv), ib);
      cp[e] = Comp{v.lo | i, v.hi};
    } else {
      cp[e] = Comp{~0ull, ~0ull};
    }
  }
  if (proc == P_BITONIC) {
    const uint32_t P = 64 * (E == 3 ? 4 : E);
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        if (j >= 64) {
          const uint32_t ej = j >> 6;
#pragma unroll
          for (uint32_t e = 0; e < EMAX; e++) {
#pragma unroll
            for (uint32_t f = e + 1; f < EMAX; f++) {
              if (f == (e ^ ej) && f * 64 < P) {
                uint32_t i = e * 64 + l;
                bool asc = (i & k) == 0;
                Comp a = cp[e], b = cp[f];
                if (comp_gt(a, b) == asc) { cp[e] = b; cp[f] = a; }
              }
            }
          }
        } else {
#pragma unroll
          for (uint32_t e = 0; e < EMAX; e++) {
            if (e * 64 < P) {
              uint32_t i = e * 64 + l;
              Comp o{__shfl_xor(cp[e].lo, (int)j), __shfl_xor(cp[e].hi, (int)j)};
              bool asc = (i & k) == 0;
              bool lower = (l & j) == 0;
              bool take_min = lower == asc;
              bool o_less = comp_gt(cp[e], o);
              if (take_min == o_less) cp[e] = o;
            }
          }
        }
      }
    }
  } else {
    // stable counting passes over the varying bits, least significant first
    for (uint32_t s = 0; s < wv; s += 8) {
      const uint32_t d = min(8u, wv - s);
      const uint32_t R = 1u << d;
      const uint32_t sh = ib + s;
      for (uint32_t v = l; v < R; v += 64) hist[v] = 0;
      wave_lds_sync();
      uint32_t dg[EMAX], rk[EMAX];
#pragma unroll
      for (uint32_t e = 0; e < EMAX; e++) {
        if (e < E) {
          uint32_t i = e * 64 + l;
          bool valid = i < m;
          uint32_t v = (uint32_t)shr128(Key{cp[e].lo, cp[e].hi}, sh).lo & (R - 1);
          uint64_t active = __ballot(valid);
          uint64_t peers = match_digit(v, d, active);
          uint32_t before = (uint32_t)__popcll(peers & lanemask_lt());
          uint32_t base = valid ? hist[v] : 0u;
          dg[e] = v;
          rk[e] = base + before;
          if (valid && before == 0) hist[v] = base + (uint32_t)__popcll(peers);
          wave_lds_sync();
        }
      }
      // exclusive scan of the R counters: each lane sums a run of 4
      uint32_t h[4], loc = 0;
#pragma unroll
      for (int q = 0; q < 4; q++) { uint32_t v = l * 4 + q; h[q] = v < R ? hist[v] : 0u; loc += h[q]; }
      uint32_t tot;
      uint32_t ex = wave_excl_scan(loc, &tot);
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < 4; q++) { uint32_t v = l * 4 + q; if (v < R) hist[v] = ex; ex += h[q]; }
      wave_lds_sync();
#pragma unroll
      for (uint32_t e = 0; e < EMAX; e++) {
        uint32_t i = e * 64 + l;
        if (e < E && i < m) {
          uint32_t pos = hist[dg[e]] + rk[e];
          cl[pos] = cp[e].lo;
          ch[pos] = cp[e].hi;
        }
      }
      wave_lds_sync();
#pragma unroll
      for (uint32_t e = 0; e < EMAX; e++) {
        uint32_t i = e * 64 + l;
        if (e < E && i < m) cp[e] = Comp{cl[i], ch[i]};
      }
      wave_lds_sync();
    }
  }
  const uint64_t imask = (1ull << ib) - 1;
#pragma unroll
  for (uint32_t e = 0; e < EMAX; e++) {
    uint32_t i = e * 64 + l;
    if (e < E && i < m) {
      uint32_t src_i = (uint32_t)(cp[e].lo & imask);
      store_rec<RW>(c.rec0, begin + i, lds_get<RW>(recs, src_i), false);
    }
  }
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// Workgroup procedures.

// Load m records into the LDS stage and reduce the varying-bit mask.
template <int RW>
__device__ Key wg_stage(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp) {
  const uint8_t* src = in_tmp ? c.rec1 : c.rec0;
  SmallShared& S = *c.S;
  for (uint32_t q0 = 0; q0 < m; q0 += WG * 8) {
    Rec<RW> r[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      uint32_t q = q0 + u * WG + threadIdx.x;
      if (q < m) r[u] = load_rec<RW>(src, begin + q);
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      uint32_t q = q0 + u * WG + threadIdx.x;
      if (q < m) lds_put<RW>(c.dyn, q, r[u]);
    }
  }
  __syncthreads();
  Key ref = lds_key<RW>(c.dyn, 0, c.kf);
  uint64_t vlo = 0, vhi = 0;
  for (uint32_t q = threadIdx.x; q < m; q += WG) {
    Key k = lds_key<RW>(c.dyn, q, c.kf);
    vlo |= k.lo ^ ref.lo;
    vhi |= k.hi ^ ref.hi;
  }
  vlo = wave_or64(vlo);
  vhi = wave_or64(vhi);
  if (lane_id() == 0) { S.vary[2 * (threadIdx.x / 64)] = vlo; S.vary[2 * (threadIdx.x / 64) + 1] = vhi; }
  __syncthreads();
  Key v{0, 0};
#pragma unroll
  for (int q = 0; q < NWAVES; q++) { v.lo |= S.vary[2 * q]; v.hi |= S.vary[2 * q + 1]; }
  __syncthreads();
  return v;
}

// Per-digit wave offsets and tile offsets after ranking: wcnt[q][v] becomes
// the count of digit v in waves before q, tcnt[v] the tile count, toff[v]
// the first LDS slot of digit v.
__device__ void tile_offsets(SmallShared& S, uint32_t R) {
  __syncthreads();
  for (uint32_t v = threadIdx.x; v < R; v += WG) {
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < NWAVES; q++) { uint32_t x = S.wcnt[q * RB + v]; S.wcnt[q * RB + v] = s; s += x; }
    S.tcnt[v] = s;
    S.toff[v] = s;
  }
  __syncthreads();
  block_excl_scan_lds(S.toff, R, S.scan_tmp);
}

__device__ __forceinline__ uint32_t rank_digit(uint32_t* wc, uint32_t v, uint32_t d, bool valid) {
  uint64_t active = __ballot(valid);
  uint64_t peers = match_digit(v, d, active);
  uint32_t before = (uint32_t)__popcll(peers & lanemask_lt());
  uint32_t base = valid ? wc[v] : 0u;
  if (valid && before == 0) wc[v] = base + (uint32_t)__popcll(peers);
  return base + before;
}

// LSD inside LDS: a permutation of local indices is refined by stable
// counting passes over the varying key bits, least significant first.
template <int RW>
__device__ void wg_lsd(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp) {
  SmallShared& S = *c.S;
  Key vary = wg_stage<RW>(c, begin, m, in_tmp);
  uint16_t* perm0 = reinterpret_cast<uint16_t*>(c.dyn + c.p.c_fin * RW);
  uint16_t* perm1 = perm0 + c.p.c_fin;
  const uint32_t wave = threadIdx.x / 64, lane = lane_id();
  if (vary.lo == 0 && vary.hi == 0) {
    if (in_tmp)
      for (uint32_t q = threadIdx.x; q < m; q += WG) store_rec<RW>(c.rec0, begin + q, lds_get<RW>(c.dyn, q), false);
    __syncthreads();
    return;
  }
  const uint32_t lo = ctz128(vary), hi = bitlen128(vary);
  for (uint32_t q = threadIdx.x; q < m; q += WG) perm0[q] = (uint16_t)q;
  const uint32_t PW = ((m + NWAVES * 64 - 1) / (NWAVES * 64)) * 64;  // positions per wave
  const uint32_t NR = PW / 64;
  for (uint32_t s = lo; s < hi; s += 8) {
    const uint32_t d = min(8u, hi - s);
    const uint32_t R = 1u << d;
    for (uint32_t i = threadIdx.x; i < NWAVES * RB; i += WG) S.wcnt[i] = 0;
    __syncthreads();
    uint32_t dg[MAX_ROUNDS], rk[MAX_ROUNDS], ix[MAX_ROUNDS];
#pragma unroll
    for (uint32_t j = 0; j < MAX_ROUNDS; j++) {
      if (j < NR) {
        uint32_t q = wave * PW + j * 64 + lane;
        bool valid = q < m;
        uint32_t idx = valid ? perm0[q] : 0u;
        uint32_t v = valid ? key_digit(lds_key<RW>(c.dyn, idx, c.kf), s, R - 1) : 0u;
        rk[j] = rank_digit(&S.wcnt[wave * RB], v, d, valid);
        dg[j] = v;
        ix[j] = idx;
      }
    }
    tile_offsets(S, R);
#pragma unroll
    for (uint32_t j = 0; j < MAX_ROUNDS; j++) {
      if (j < NR) {
        uint32_t q = wave * PW + j * 64 + lane;
        if (q < m) perm1[S.toff[dg[j]] + S.wcnt[wave * RB + dg[j]] + rk[j]] = (uint16_t)ix[j];
      }
    }
    __syncthreads();
    uint16_t* t = perm0; perm0 = perm1; perm1 = t;
  }
  for (uint32_t q = threadIdx.x; q < m; q += WG) store_rec<RW>(c.rec0, begin + q, lds_get<RW>(c.dyn, perm0[q]), false);
  __syncthreads();
}

// Bitonic sort of (varying key bits, local index) composites in LDS.
template <int RW>
__device__ void wg_bitonic(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp) {
  Key vary = wg_stage<RW>(c, begin, m, in_tmp);
  if (vary.lo == 0 && vary.hi == 0) {
    if (in_tmp)
      for (uint32_t q = threadIdx.x; q < m; q += WG) store_rec<RW>(c.rec0, begin + q, lds_get<RW>(c.dyn, q), false);
    __syncthreads();
    return;
  }
  const uint32_t lo = ctz128(vary);
  const uint32_t wv = bitlen128(vary) - lo;
  const uint32_t ib = 32 - __clz(m - 1);
  uint32_t P = 1;
  while (P < m) P <<= 1;
  uint64_t* cl = reinterpret_cast<uint64_t*>(c.dyn + c.p.c_fin * RW);
  uint64_t* ch = cl + c.p.bitonic_max;
  for (uint32_t q = threadIdx.x; q < P; q += WG) {
    if (q < m) {
      Key v = shl128(mask128(shr128(lds_key<RW>(c.dyn, q, c.kf), lo), wv), ib);
      cl[q] = v.lo | q;
      ch[q] = v.hi;
    } else {
      cl[q] = ~0ull;
      ch[q] = ~0ull;
    }
  }
  __syncthreads();
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t t = threadIdx.x; t < P / 2; t += WG) {
        uint32_t a = 2 * j * (t / j) + (t % j);
        uint32_t b = a + j;
        bool asc = (a & k) == 0;
        Comp x{cl[a], ch[a]}, y{cl[b], ch[b]};
        if (comp_gt(x, y) == asc) { cl[a] = y.lo; ch[a] = y.hi; cl[b] = x.lo; ch[b] = x.hi; }
      }
      __syncthreads();
    }
  }
  const uint64_t imask = (1ull << ib) - 1;
  for (uint32_t q = threadIdx.x; q < m; q += WG)
    store_rec<RW>(c.rec0, begin + q, lds_get<RW>(c.dyn, (uint32_t)(cl[q] & imask)), false);
  __syncthreads();
}

// Copy a finished bucket from tmp to records.
template <int RW>
__device__ void wg_copy(Ctx& c, uint64_t begin, uint64_t m) {
  for (uint64_t q = threadIdx.x; q < m; q += WG) store_rec<RW>(c.rec0, begin + q, load_rec<RW>(c.rec1, begin + q), false);
}

// One radix pass of a bucket by the workgroup (the paper's per-bin split,
// Sec. 3.4).  Sweep 1 counts digits and finds the bits all keys share (they
// are skipped); sweep 2 moves records tile by tile to the other buffer, each
// tile ranked stably and staged in LDS, digit runs appended in tile order.
// Fills child list `slot`.  Returns false if every key is equal (the bucket
// is then already finished in records).
template <int RW>
__device__ bool block_pass(Ctx& c, const Bucket& b, uint32_t slot) {
  SmallShared& S = *c.S;
  const uint32_t wave = threadIdx.x / 64, lane = lane_id();
  const bool in_tmp = b.flags & BF_TMP;
  const uint8_t* src = in_tmp ? c.rec1 : c.rec0;
  uint8_t* dst = in_tmp ? c.rec0 : c.rec1;
  const uint32_t m = (uint32_t)b.count;
  const uint32_t KB = c.kf.kbits;
  uint32_t bit = b.bit;
  uint32_t d, R, shift;
  Key ref = load_key<RW>(src, b.begin, c.kf);
  for (;;) {
    d = min(c.p.d_block, KB - bit);
    R = 1u << d;
    shift = KB - bit - d;
    for (uint32_t v = threadIdx.x; v < R; v += WG) S.hist[v] = 0;
    __syncthreads();
    uint64_t vlo = 0, vhi = 0;
    for (uint32_t q0 = 0; q0 < m; q0 += WG * 16) {
      Key kk[16];
#pragma unroll
      for (int u = 0; u < 16; u++) {
        uint32_t q = q0 + u * WG + threadIdx.x;
        kk[u] = q < m ? load_key<RW>(src, b.begin + q, c.kf) : ref;
      }
#pragma unroll
      for (int u = 0; u < 16; u++) {
        uint32_t q = q0 + u * WG + threadIdx.x;
        bool valid = q < m;
        vlo |= kk[u].lo ^ ref.lo;
        vhi |= kk[u].hi ^ ref.hi;
        uint32_t v = key_digit(kk[u], shift, R - 1);
        uint64_t active = __ballot(valid);
        uint64_t peers = match_digit(v, d, active);
        if (valid && (uint32_t)(__ffsll((long long)peers) - 1) == lane) atomicAdd(&S.hist[v], (uint32_t)__popcll(peers));
      }
    }
    vlo = wave_or64(vlo);
    vhi = wave_or64(vhi);
    if (lane == 0) { S.vary[2 * wave] = vlo; S.vary[2 * wave + 1] = vhi; }
    __syncthreads();
    Key vary{0, 0};
#pragma unroll
    for (int q = 0; q < NWAVES; q++) { vary.lo |= S.vary[2 * q]; vary.hi |= S.vary[2 * q + 1]; }
    __syncthreads();
    if (vary.lo == 0 && vary.hi == 0) {
      if (in_tmp) wg_copy<RW>(c, b.begin, m);
      __syncthreads();
      return false;
    }
    uint32_t lead = common_prefix_bits(vary, KB);
    if (lead >= bit + d) { bit = lead; continue; }
    break;
  }
  // digit offsets
  for (uint32_t v = threadIdx.x; v < R; v += WG) { S.ccnt[slot][v] = S.hist[v]; S.toff[v] = S.hist[v]; }
  __syncthreads();
  block_excl_scan_lds(S.toff, R, S.scan_tmp);
  for (uint32_t v = threadIdx.x; v < R; v += WG) { S.cbase[slot][v] = S.toff[v]; S.run[v] = S.toff[v]; }
  if (threadIdx.x == 0) {
    S.cbit[slot] = bit + d;
    S.ctmp[slot] = in_tmp ? 0u : 1u;
    S.cbegin[slot] = b.begin;
    S.cparent[slot] = m;
  }
  __syncthreads();
  // sweep 2: stable tiles through LDS
  const uint32_t BT = c.p.block_tile;
  const uint32_t per_wave = BT / NWAVES;
  const uint32_t IPT = BT / WG;
  constexpr uint32_t IPT_MAX = RW >= 2 ? 64 / RW : 32;
  for (uint32_t t0 = 0; t0 < m; t0 += BT) {
    const uint32_t cnt = min(BT, m - t0);
    for (uint32_t i = threadIdx.x; i < NWAVES * RB; i += WG) S.wcnt[i] = 0;
    __syncthreads();
    Rec<RW> rec[IPT_MAX];
    uint32_t dg[IPT_MAX], rk[IPT_MAX];
    const uint32_t wb = t0 + wave * per_wave;
#pragma unroll
    for (uint32_t j = 0; j < IPT_MAX; j++) {
      uint32_t q = wb + j * 64 + lane;
      if (j < IPT && q < m) rec[j] = load_rec<RW>(src, b.begin + q);
    }
#pragma unroll
    for (uint32_t j = 0; j < IPT_MAX; j++) {
      if (j < IPT) {
        uint32_t q = wb + j * 64 + lane;
        bool valid = q < m;
        uint32_t v = valid ? key_digit(rec_key<RW>(rec[j], c.kf), shift, R - 1) : 0u;
        rk[j] = rank_digit(&S.wcnt[wave * RB], v, d, valid);
        dg[j] = v;
      }
    }
    tile_offsets(S, R);
#pragma unroll
    for (uint32_t j = 0; j < IPT_MAX; j++) {
      uint32_t q = wb + j * 64 + lane;
      if (j < IPT && q < m) lds_put<RW>(c.dyn, S.toff[dg[j]] + S.wcnt[wave * RB + dg[j]] + rk[j], rec[j]);
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < cnt; q += WG) {
      Rec<RW> r = lds_get<RW>(c.dyn, q);
      uint32_t v = key_digit(rec_key<RW>(r, c.kf), shift, R - 1);
      store_rec<RW>(dst, b.begin + S.run[v] + (q - S.toff[v]), r, false);
    }
    __syncthreads();
    for (uint32_t v = threadIdx.x; v < R; v += WG) S.run[v] += S.tcnt[v];
    __syncthreads();
  }
  if (threadIdx.x == 0) S.cR[slot] = R;  // number of digits, read by the caller
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------------------
// Tracing: one row per scheduled bucket.
__device__ void trace_row(Ctx& c, uint64_t m, uint64_t parent, uint32_t bit, uint32_t chosen, uint32_t observed,
                          const uint32_t* ticks, uint32_t flags) {
  if (!c.w.trace) return;
  uint64_t i = atomicAdd((unsigned long long*)c.w.trace_count, 1ull);
  if (i >= c.p.trace_cap) return;
  raduls_trace_row row;
  bucket_features(row.features, m, parent, bit, c.kf.kbits, c.p.rec_bytes, c.p.key_bytes);
  row.chosen = chosen;
  row.count = (uint32_t)m;
  row.observed = observed;
  for (int q = 0; q < 3; q++) row.time_ticks[q] = ticks[q];
  row.flags = flags;
  c.w.trace[i] = row;
}

template <int RW, bool ALLOW_RADIX>
__device__ void run_wg_proc(Ctx& c, uint32_t proc, uint64_t begin, uint32_t m, uint32_t bit, bool in_tmp,
                            uint64_t parent);

// Route the children of a radix pass held in child list `slot`.  Children of
// slot 0 may get one more radix pass (slot 1); children of slot 1 are all
// finished directly, so the nesting ends there.
template <int RW, uint32_t slot>
__device__ void handle_children(Ctx& c) {
  SmallShared& S = *c.S;
  const uint32_t R = S.cR[slot];
  const uint32_t KB = c.kf.kbits;
  const uint32_t cb = S.cbit[slot];
  const bool ctmp = S.ctmp[slot] != 0;
  const uint64_t base = S.cbegin[slot];
  const uint64_t parent = S.cparent[slot];
  if (threadIdx.x == 0) { S.wn[slot] = 0; S.gn[slot] = 0; S.wnext[slot] = 0; }
  __syncthreads();
  // classify: one child per thread (R <= WG)
  for (uint32_t v = threadIdx.x; v < R; v += WG) {
    uint32_t cnt = S.ccnt[slot][v];
    uint32_t code = C_NONE;
    if (cnt == 0) {
    } else if (cnt == 1 || cb >= KB) {
      if (ctmp) code = cnt <= 64 ? C_WRANK : C_GCOPY;
    } else if (cnt <= TINY_MAX) {
      code = C_WRANK;
    } else if (cnt > c.p.c_fin) {
      code = C_PUSH;
    } else {
      uint32_t feas = feasible_mask(c.p, cnt, cb, KB, slot == 0);
      uint32_t proc = choose_proc(c.p, c.w.model, cnt, parent, cb, KB, feas);
      bool sample = false;
      if (c.w.trace && c.p.sample_period && __popc(feas) > 1) {
        uint32_t k = atomicAdd(&S.decisions, 1u);
        sample = ((k + blockIdx.x * 7919u) % c.p.sample_period) == 0;
      }
      uint32_t ib = 32 - __clz(cnt - 1);
      bool wave_ok = cnt <= c.ws && (KB - cb) + ib <= 128;
      if (sample) code = C_CF;
      else if (proc == P_RADIX) code = C_GRADIX;
      else if (proc == P_BITONIC) code = wave_ok ? C_WBIT : C_GBIT;
      else code = wave_ok ? C_WLSD : C_GLSD;
    }
    S.ccode[slot][v] = code;
    if (code == C_WRANK || code == C_WLSD || code == C_WBIT) S.wlist[slot][atomicAdd(&S.wn[slot], 1u)] = v;
    else if (code == C_PUSH) {
      uint32_t sp = atomicAdd(&S.sp, 1u);
      if (sp < c.p.stack_cap) {
        Bucket ch{base + S.cbase[slot][v], cnt, parent, cb, ctmp ? BF_TMP : 0u};
        c.stack[sp] = ch;
      } else {
        atomicOr(&c.w.ctl->overflow, 16u);
      }
    } else if (code != C_NONE) S.glist[slot][atomicAdd(&S.gn[slot], 1u)] = v;
  }
  __syncthreads();
  // wavefront phase
  {
    const uint32_t wave = threadIdx.x / 64;
    uint32_t* reg = c.dyn + wave * (c.ws * RW + 4 * c.ws + RB);
    const uint32_t wn = S.wn[slot];
    for (;;) {
      uint32_t j = 0;
      if (lane_id() == 0) j = atomicAdd(&S.wnext[slot], 1u);
      j = __shfl(j, 0);
      if (j >= wn) break;
      uint32_t v = S.wlist[slot][j];
      uint32_t cnt = S.ccnt[slot][v];
      uint32_t code = S.ccode[slot][v];
      uint64_t cbeg = base + S.cbase[slot][v];
      uint64_t t0 = c.w.trace ? now_ticks() : 0;
      if (code == C_WRANK) wave_rank<RW>(c, cbeg, cnt, ctmp);
      else wave_sort<RW>(c, cbeg, cnt, ctmp, code == C_WBIT ? P_BITONIC : P_LSD, reg);
      if (c.w.trace && code != C_WRANK && lane_id() == 0) {
        uint32_t proc = code == C_WBIT ? P_BITONIC : P_LSD;
        uint32_t ticks[3] = {0, 0, 0};
        ticks[proc] = (uint32_t)((now_ticks() - t0 + 2) / 4);  // one wave of four
        trace_row(c, cnt, parent, cb, proc, 1u << proc, ticks, 0u);
      }
    }
  }
  __syncthreads();
  // workgroup phase
  const uint32_t gn = S.gn[slot];
  for (uint32_t j = 0; j < gn; j++) {
    uint32_t v = S.glist[slot][j];
    uint32_t cnt = S.ccnt[slot][v];
    uint32_t code = S.ccode[slot][v];
    uint64_t cbeg = base + S.cbase[slot][v];
    if (code == C_GCOPY) {
      wg_copy<RW>(c, cbeg, cnt);
      __syncthreads();
      continue;
    }
    uint32_t proc = code == C_GRADIX ? P_RADIX : (code == C_GBIT ? P_BITONIC : (code == C_GLSD ? P_LSD : 0xFFu));
    if (code == C_CF) {
      // counterfactual sample: run every feasible procedure on the same
      // input (kept in tmp), timing each; the last run leaves the output
      uint32_t feas = feasible_mask(c.p, cnt, cb, KB, slot == 0);
      uint32_t chosen = choose_proc(c.p, c.w.model, cnt, parent, cb, KB, feas);
      bool in_tmp = ctmp;
      if (!in_tmp) {
        for (uint64_t q = threadIdx.x; q < cnt; q += WG)
          store_rec<RW>(c.rec1, cbeg + q, load_rec<RW>(c.rec0, cbeg + q), false);
        __syncthreads();
        in_tmp = true;
      }
      uint32_t ticks[3] = {0, 0, 0};
      for (uint32_t k = 0; k < 3; k++) {
        uint32_t q = (chosen + 1 + k) % 3;  // chosen procedure runs last
        if (!((feas >> q) & 1u)) continue;
        __syncthreads();
        uint64_t t0 = now_ticks();
        run_wg_proc<RW, slot == 0>(c, q, cbeg, cnt, cb, in_tmp, parent);
        __syncthreads();
        ticks[q] = (uint32_t)(now_ticks() - t0);
      }
      if (threadIdx.x == 0) trace_row(c, cnt, parent, cb, chosen, feas, ticks, 1u);
      __syncthreads();
      continue;
    }
    uint64_t t0 = c.w.trace ? now_ticks() : 0;
    run_wg_proc<RW, slot == 0>(c, proc, cbeg, cnt, cb, ctmp, parent);
    if (c.w.trace && threadIdx.x == 0) {
      uint32_t ticks[3] = {0, 0, 0};
      ticks[proc] = (uint32_t)(now_ticks() - t0);
      trace_row(c, cnt, parent, cb, proc, 1u << proc, ticks, 0u);
    }
    __syncthreads();
  }
}

// A procedure run by the whole workgroup on a bucket of m <= c_fin records.
// RADIX here is one pass whose children are all finished right away.
template <int RW, bool ALLOW_RADIX>
__device__ void run_wg_proc(Ctx& c, uint32_t proc, uint64_t begin, uint32_t m, uint32_t bit, bool in_tmp,
                            uint64_t parent) {
  if constexpr (ALLOW_RADIX) {
    if (proc == P_RADIX) {
      Bucket b{begin, m, parent, bit, in_tmp ? BF_TMP : 0u};
      if (block_pass<RW>(c, b, 1)) handle_children<RW, 1>(c);
      return;
    }
  }
  const bool wave_ok = m <= c.ws && (c.kf.kbits - bit) + (32 - __clz(m - 1)) <= 128;
  if (wave_ok) {
    if (threadIdx.x < 64) wave_sort<RW>(c, begin, m, in_tmp, proc == P_BITONIC ? P_BITONIC : P_LSD, c.dyn);
    __syncthreads();
  } else if (proc == P_BITONIC) {
    wg_bitonic<RW>(c, begin, m, in_tmp);
  } else {
    wg_lsd<RW>(c, begin, m, in_tmp);
  }
}

// A bucket taken from the queue or from the workgroup's stack.
template <int RW>
__device__ void process_root(Ctx& c, const Bucket& b) {
  const uint32_t KB = c.kf.kbits;
  const uint32_t m = (uint32_t)b.count;
  const bool in_tmp = b.flags & BF_TMP;
  if (m <= TINY_MAX) {
    if (threadIdx.x < 64) wave_rank<RW>(c, b.begin, m, in_tmp);
    __syncthreads();
    return;
  }
  if (m > c.p.c_fin) {
    if (block_pass<RW>(c, b, 0)) handle_children<RW, 0>(c);
    return;
  }
  uint32_t feas = feasible_mask(c.p, m, b.bit, KB, true);
  uint32_t proc = choose_proc(c.p, c.w.model, m, b.parent, b.bit, KB, feas);
  uint64_t t0 = c.w.trace ? now_ticks() : 0;
  run_wg_proc<RW, true>(c, proc, b.begin, m, b.bit, in_tmp, b.parent);
  if (c.w.trace && threadIdx.x == 0 && __popc(feas) > 1) {
    uint32_t ticks[3] = {0, 0, 0};
    ticks[proc] = (uint32_t)(now_ticks() - t0);
    trace_row(c, m, b.parent, b.bit, proc, 1u << proc, ticks, 0u);
  }
  __syncthreads();
}

template <int RW>
__global__ __launch_bounds__(WG) void k_small(Plan p, Work w, uint8_t* rec0, uint8_t* rec1) {
  extern __shared__ __align__(16) uint32_t dyn[];
  __shared__ SmallShared S;
  Ctx c;
  c.p = p;
  c.w = w;
  c.rec0 = rec0;
  c.rec1 = rec1;
  c.kf = make_keyfmt(p.key_bytes);
  c.S = &S;
  c.dyn = dyn;
  c.stack = w.stacks + (uint64_t)blockIdx.x * p.stack_cap;
  c.ws = p.wave_cap;
  if (threadIdx.x == 0) { S.sp = 0; S.decisions = 0; }
  __syncthreads();
  const uint32_t ns = (uint32_t)min((uint64_t)w.ctl->nsmall, p.cap_small);
  for (;;) {
    if (threadIdx.x == 0) S.bcast = atomicAdd(&w.ctl->small_head, 1u);
    __syncthreads();
    const uint32_t idx = S.bcast;
    __syncthreads();
    if (idx >= ns) break;
    Bucket b = w.small_ord[idx];
    process_root<RW>(c, b);
    for (;;) {
      __syncthreads();
      if (S.sp == 0) break;
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t sp = min(S.sp, p.stack_cap) - 1;
        S.sp = sp;
        S.item = c.stack[sp];
      }
      __syncthreads();
      Bucket b2 = S.item;
      process_root<RW>(c, b2);
    }
  }
  // tiny buckets, one wavefront each
  const uint32_t nt = (uint32_t)min((uint64_t)w.ctl->ntiny, p.cap_tiny);
  for (;;) {
    uint32_t j = 0;
    if (lane_id() == 0) j = atomicAdd(&w.ctl->tiny_head, 1u);
    j = __shfl(j, 0);
    if (j >= nt) break;
    uint64_t x = w.tiny[j];
    uint64_t begin = x & ((1ull << 40) - 1);
    uint32_t cnt = (uint32_t)(x >> 40) & 63u;
    bool tmp = (x >> 46) & 1u;
    wave_rank<RW>(c, begin, cnt, tmp);
  }
}

uint32_t small_dynamic_lds(const Plan& p) {
  uint32_t r = p.rec_bytes;
  uint32_t block = p.block_tile * r;
  uint32_t fin = p.c_fin * r + max(4u * p.c_fin, 16u * p.bitonic_max);
  uint32_t waves = NWAVES * (p.wave_cap * r + 16u * p.wave_cap + 4u * RB);
  return max(block, max(fin, waves));
}

void launch_small(const Plan& p, const Work& w, void* records, void* tmp, hipStream_t s) {
  uint32_t lds = small_dynamic_lds(p);
  switch (p.rw) {
#define RD_CASE(n) case n: k_small<n><<<p.grid_small, WG, lds, s>>>(p, w, (uint8_t*)records, (uint8_t*)tmp); break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

}  // namespace rd
