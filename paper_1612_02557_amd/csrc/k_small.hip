// k_small.hip -- single-workgroup work: the bucket queue (paper, Sec. 3.4:
// small bins are handed out from a shared queue, largest first, and each is
// processed by one thread) and the finishing sorts of Sec. 3.5.
//
// A persistent grid takes buckets from the queue, largest size class first.
// A bucket larger than the LDS finishing capacity C gets a one-workgroup
// radix pass (RADIX).  Its children lie consecutively in digit order, so runs
// of whole children holding at most C records are finished together: one
// coalesced load into LDS, a stable sort there (LSD counting passes or a
// bitonic network, as the scheduler picks), one coalesced store.  Children
// above C go to the workgroup's own depth-first stack.  A queued bucket of at
// most C records is finished directly (or, if the scheduler says so, split
// once more first); one of at most 32 records is ranked by one wavefront
// (RANK, the insertion-sort slot of Sec. 3.5).  Every procedure is stable, so
// the output does not depend on which one runs.
#include "raduls_dev.hpp"
#include "raduls_kernels.hpp"
#include "sched_dev.hpp"

namespace rd {

constexpr uint32_t RB = 256;          // radix of one-workgroup passes (d_block <= 8)
constexpr uint32_t MAX_ROUNDS = 16;   // LDS finishing capacity <= 16 * WG records
constexpr uint32_t IPT_BLOCK = 8;     // records per thread in a radix-pass tile
constexpr uint32_t EMAX = 4;          // records per lane of a wavefront job (at most 256)
// The in-LDS radix procedure computes each record's slot within its
// sub-bucket by counting the smaller composites there, a cost that grows
// with the sub-bucket; above this size the job is finished by the bitonic
// network instead.
constexpr uint32_t RANK_SUB_MAX = 256;

struct SmallShared {
  uint32_t hist[RB];
  uint32_t run[RB];
  uint32_t wcnt[NWAVES * RB];
  uint32_t toff[RB + 1];
  uint32_t tcnt[RB];
  uint32_t scan_tmp[NWAVES + 1];
  uint64_t vary[2 * NWAVES];
  // children of the current radix pass, grouped into finishing jobs
  uint32_t cbase[RB + 1];  // child starts; then job starts and the end of the last job
  uint32_t ccnt[RB];
  uint32_t jb[RB];        // job start (offset in the parent bucket)
  uint32_t jn[RB];        // job length
  uint32_t jinfo[RB];     // shared key bits | procedure << 16 | sampled << 24 | feasible << 28
  uint32_t nw, wnext;
  uint32_t cbit, pbit, cR, ctmp;
  uint64_t cbegin, cparent;
  uint32_t sp;
  uint32_t bcast;
  // the scheduler network, copied from global memory when it is in use,
  // with the layer-2 matrix transposed (lane j then reads its column of a
  // row of the matrix without bank conflicts)
  float model[MLP_MODEL_FLOATS];
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
  const float* model;  // the network in LDS, or null
  Bucket* stack;
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
__device__ __forceinline__ void wave_rank(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp) {
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

// LSD or BITONIC on m <= 64*EMAX records by one wave, no workgroup barrier.
// The records are staged in the wave's own LDS region; the composites
// (varying key bits << ib | local index) are sorted in registers -- bitonic
// steps across lanes by shuffles and within a lane by register exchange --
// or by stable counting passes through the wave's LDS, and the sorted
// composites name the records to gather.
template <int RW>
__device__ __forceinline__ void wave_sort(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp, uint32_t proc,
                                          uint32_t* reg) {
  const uint32_t ws = c.p.wave_cap;
  const uint32_t l = lane_id();
  const uint8_t* src = in_tmp ? c.rec1 : c.rec0;
  const uint32_t E = (m + 63) / 64;
  uint32_t* recs = reg;                                             // ws * RW words
  uint64_t* cl = reinterpret_cast<uint64_t*>(reg + ws * RW);      // ws comps (lo)
  uint64_t* ch = cl + ws;                                         // ws comps (hi)
  uint32_t* hist = reinterpret_cast<uint32_t*>(ch + ws);          // 256 counters
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
  Key vary = Key{wave_or64(vlo), wave_or64(vhi)};
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
      RankPart rp[EMAX];
#pragma unroll
      for (uint32_t e = 0; e < EMAX; e++) {
        if (e < E) {
          uint32_t i = e * 64 + l;
          bool valid = i < m;
          uint32_t v = (uint32_t)shr128(Key{cp[e].lo, cp[e].hi}, sh).lo & (R - 1);
          rp[e] = rank_issue(hist, v, d, valid);
          dg[e] = v;
        }
      }
#pragma unroll
      for (uint32_t e = 0; e < EMAX; e++)
        if (e < E) rk[e] = rank_finish(rp[e]);
      wave_lds_sync();
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


// wave_sort for jobs whose composite fits 64 bits ((key bits left) + index
// bits <= 64): the same two procedures on single 64-bit values.
template <int RW>
__device__ __forceinline__ void wave_sort64(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp, uint32_t proc,
                                            uint32_t* reg) {
  const uint32_t ws = c.p.wave_cap;
  const uint32_t l = lane_id();
  const uint8_t* src = in_tmp ? c.rec1 : c.rec0;
  const uint32_t E = (m + 63) / 64;
  uint32_t* recs = reg;                                        // ws * RW words
  uint64_t* cl = reinterpret_cast<uint64_t*>(reg + ws * RW);   // ws composites
  uint32_t* hist = reinterpret_cast<uint32_t*>(cl + 2 * ws);   // 256 counters
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
  const uint64_t vmask = wv >= 64 ? ~0ull : ((1ull << wv) - 1);
  uint64_t cp[EMAX];
#pragma unroll
  for (uint32_t e = 0; e < EMAX; e++) {
    uint32_t i = e * 64 + l;
    cp[e] = (e < E && i < m) ? (((shr128(key[e], lo).lo & vmask) << ib) | i) : ~0ull;
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
                bool asc = ((e * 64 + l) & k) == 0;
                uint64_t a = cp[e], b = cp[f];
                if ((a > b) == asc) { cp[e] = b; cp[f] = a; }
              }
            }
          }
        } else {
          const bool lower = (l & j) == 0;
#pragma unroll
          for (uint32_t e = 0; e < EMAX; e++) {
            if (e * 64 < P) {
              uint64_t o = __shfl_xor(cp[e], (int)j);
              bool asc = ((e * 64 + l) & k) == 0;
              // keep the smaller value when (lower == asc), else the larger
              if ((lower == asc) == (cp[e] > o)) cp[e] = o;
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
      RankPart rp[EMAX];
#pragma unroll
      for (uint32_t e = 0; e < EMAX; e++) {
        if (e < E) {
          uint32_t i = e * 64 + l;
          bool valid = i < m;
          uint32_t v = (uint32_t)(cp[e] >> sh) & (R - 1);
          rp[e] = rank_issue(hist, v, d, valid);
          dg[e] = v;
        }
      }
#pragma unroll
      for (uint32_t e = 0; e < EMAX; e++)
        if (e < E) rk[e] = rank_finish(rp[e]);
      wave_lds_sync();
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
        if (e < E && i < m) cl[hist[dg[e]] + rk[e]] = cp[e];
      }
      wave_lds_sync();
#pragma unroll
      for (uint32_t e = 0; e < EMAX; e++) {
        uint32_t i = e * 64 + l;
        if (e < E && i < m) cp[e] = cl[i];
      }
      wave_lds_sync();
    }
  }
  const uint64_t imask = (1ull << ib) - 1;
#pragma unroll
  for (uint32_t e = 0; e < EMAX; e++) {
    uint32_t i = e * 64 + l;
    if (e < E && i < m) store_rec<RW>(c.rec0, begin + i, lds_get<RW>(recs, (uint32_t)(cp[e] & imask)), false);
  }
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// Workgroup procedures.

// OR over the staged records of (key XOR the first key): the bits that vary.
template <int RW>
__device__ __forceinline__ Key stage_vary(Ctx& c, uint32_t m) {
  SmallShared& S = *c.S;
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
  // no barrier here: S.vary is written again only by the next job's stage,
  // several barriers later
  return v;
}

// A job's records held in registers (record q = u * WG + thread in slot u),
// so the next job's loads can be in flight while this one is sorted.
template <int RW>
struct JobRegs {
  static constexpr uint32_t CMAX0 = (60u * 1024u / (4u * RW + 16u)) / 64u * 64u;
  static constexpr uint32_t CMAX = CMAX0 < 4096u ? CMAX0 : 4096u;  // the largest LDS job
  static constexpr uint32_t N = (CMAX + WG - 1) / WG;
  Rec<RW> r[N];
};

template <int RW>
__device__ __forceinline__ void regs_load(Ctx& c, JobRegs<RW>& jr, uint64_t begin, uint32_t m, bool in_tmp) {
  const uint8_t* src = in_tmp ? c.rec1 : c.rec0;
#pragma unroll
  for (uint32_t u = 0; u < JobRegs<RW>::N; u++) {
    uint32_t q = u * WG + threadIdx.x;
    if (q < m) jr.r[u] = load_rec<RW>(src, begin + q);
  }
}

template <int RW>
__device__ __forceinline__ void regs_stage(Ctx& c, const JobRegs<RW>& jr, uint32_t m) {
#pragma unroll
  for (uint32_t u = 0; u < JobRegs<RW>::N; u++) {
    uint32_t q = u * WG + threadIdx.x;
    if (q < m) lds_put<RW>(c.dyn, q, jr.r[u]);
  }
}

// Load m records into the LDS stage and reduce the varying-bit mask.
template <int RW>
__device__ __forceinline__ Key wg_stage(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp) {
  const uint8_t* src = in_tmp ? c.rec1 : c.rec0;
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
  return stage_vary<RW>(c, m);
}

// Per-digit wave offsets and tile offsets after ranking: wcnt[q][v] becomes
// the count of digit v in waves before q, tcnt[v] the tile count, toff[v]
// the first slot of digit v.
__device__ __forceinline__ void tile_offsets(SmallShared& S, uint32_t R) {
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

// One stable counting pass over 64-bit values in LDS (digit = bits
// [shift, shift + d) of the value): src -> dst.  Wave q owns positions
// [q*PW, (q+1)*PW), taken 64 at a time, so ranks follow position order.
__device__ __forceinline__ void lds_pass64(SmallShared& S, const uint64_t* src, uint64_t* dst, uint32_t m, uint32_t shift,
                           uint32_t d) {
  const uint32_t wave = threadIdx.x / 64, lane = lane_id();
  const uint32_t R = 1u << d;
  const uint32_t PW = ((m + NWAVES * 64 - 1) / (NWAVES * 64)) * 64;
  const uint32_t NR = PW / 64;
  for (uint32_t i = threadIdx.x; i < NWAVES * RB; i += WG) S.wcnt[i] = 0;
  __syncthreads();
  uint64_t xv[MAX_ROUNDS];
  uint32_t dg[MAX_ROUNDS], rk[MAX_ROUNDS];
  RankPart rp[MAX_ROUNDS];
#pragma unroll
  for (uint32_t j = 0; j < MAX_ROUNDS; j++) {
    if (j < NR) {
      uint32_t q = wave * PW + j * 64 + lane;
      bool valid = q < m;
      uint64_t x = valid ? src[q] : 0ull;
      uint32_t v = (uint32_t)(x >> shift) & (R - 1);
      rp[j] = rank_issue(&S.wcnt[wave * RB], v, d, valid);
      dg[j] = v;
      xv[j] = x;
    }
  }
#pragma unroll
  for (uint32_t j = 0; j < MAX_ROUNDS; j++)
    if (j < NR) rk[j] = rank_finish(rp[j]);
  tile_offsets(S, R);
#pragma unroll
  for (uint32_t j = 0; j < MAX_ROUNDS; j++) {
    if (j < NR) {
      uint32_t q = wave * PW + j * 64 + lane;
      if (q < m) dst[S.toff[dg[j]] + S.wcnt[wave * RB + dg[j]] + rk[j]] = xv[j];
    }
  }
  __syncthreads();
}

// Finish m <= C records at [begin, begin+m) of one buffer into records,
// stably by key.  The records are staged in LDS; what is sorted is the
// composite (key bits that vary in this range) << ib | local index, so the
// sort needs no tie rule and its result names the record to gather.
//   LSD     stable counting passes over the varying bits, 8 at a time,
//           least significant first (paper, Sec. 1)
//   BITONIC a bitonic network on the (unique) composites
// When the varying bits and the index do not fit in 64 bits, LSD refines a
// permutation reading the keys from the stage, and BITONIC sorts 128-bit
// composites (or, above 128 bits, takes the LSD refinement too).
template <int RW>
__device__ __forceinline__ void wg_sort_staged(Ctx& c, uint64_t begin, uint32_t m, uint32_t proc, Key vary) {
  SmallShared& S = *c.S;
  const uint32_t C = c.p.c_fin;
  const uint32_t* stage = c.dyn;
  const uint32_t lo = ctz128(vary);
  const uint32_t W = bitlen128(vary) - lo;
  const uint32_t ib = 32 - __clz(m - 1);
  uint64_t* c0 = reinterpret_cast<uint64_t*>(c.dyn + C * RW);
  uint64_t* c1 = c0 + C;
  uint32_t P = 1;
  while (P < m) P <<= 1;
  const uint64_t imask = (1ull << ib) - 1;
  if (W + ib <= 64) {
    const uint32_t n_fill = proc == P_BITONIC ? P : m;
    for (uint32_t q = threadIdx.x; q < n_fill; q += WG) {
      if (q < m) {
        Key k = lds_key<RW>(stage, q, c.kf);
        uint64_t v = shr128(k, lo).lo & (W >= 64 ? ~0ull : ((1ull << W) - 1));
        c0[q] = (v << ib) | q;
      } else {
        c0[q] = ~0ull;
      }
    }
    __syncthreads();
    const uint64_t* out = c0;
    if (proc == P_BITONIC) {
      for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
          for (uint32_t t = threadIdx.x; t < P / 2; t += WG) {
            uint32_t a = 2 * j * (t / j) + (t % j);
            uint32_t b = a + j;
            bool asc = (a & k) == 0;
            uint64_t x = c0[a], y = c0[b];
            if ((x > y) == asc) { c0[a] = y; c0[b] = x; }
          }
          __syncthreads();
        }
      }
    } else {
      uint64_t* a = c0;
      uint64_t* b = c1;
      for (uint32_t s = 0; s < W; s += 8) {
        lds_pass64(S, a, b, m, ib + s, min(8u, W - s));
        uint64_t* t = a; a = b; b = t;
      }
      out = a;
    }
    for (uint32_t q = threadIdx.x; q < m; q += WG)
      store_rec<RW>(c.rec0, begin + q, lds_get<RW>(stage, (uint32_t)(out[q] & imask)), false);
    __syncthreads();
    return;
  }
  if (proc == P_BITONIC && P <= C && W + ib <= 128) {
    uint64_t* cl = c0;
    uint64_t* ch = c0 + P;
    for (uint32_t q = threadIdx.x; q < P; q += WG) {
      if (q < m) {
        Key v = shl128(mask128(shr128(lds_key<RW>(stage, q, c.kf), lo), W), ib);
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
          uint64_t xl = cl[a], xh = ch[a], yl = cl[b], yh = ch[b];
          bool gt = xh > yh || (xh == yh && xl > yl);
          if (gt == asc) { cl[a] = yl; ch[a] = yh; cl[b] = xl; ch[b] = xh; }
        }
        __syncthreads();
      }
    }
    for (uint32_t q = threadIdx.x; q < m; q += WG)
      store_rec<RW>(c.rec0, begin + q, lds_get<RW>(stage, (uint32_t)(cl[q] & imask)), false);
    __syncthreads();
    return;
  }
  // wide keys: refine a permutation of local indices
  uint16_t* perm0 = reinterpret_cast<uint16_t*>(c0);
  uint16_t* perm1 = perm0 + C;
  const uint32_t wave = threadIdx.x / 64, lane = lane_id();
  for (uint32_t q = threadIdx.x; q < m; q += WG) perm0[q] = (uint16_t)q;
  const uint32_t PW = ((m + NWAVES * 64 - 1) / (NWAVES * 64)) * 64;
  const uint32_t NR = PW / 64;
  const uint32_t hi = lo + W;
  for (uint32_t s = lo; s < hi; s += 8) {
    const uint32_t d = min(8u, hi - s);
    const uint32_t R = 1u << d;
    for (uint32_t i = threadIdx.x; i < NWAVES * RB; i += WG) S.wcnt[i] = 0;
    __syncthreads();
    uint32_t dg[MAX_ROUNDS], rk[MAX_ROUNDS], ix[MAX_ROUNDS];
    RankPart rp[MAX_ROUNDS];
#pragma unroll
    for (uint32_t j = 0; j < MAX_ROUNDS; j++) {
      if (j < NR) {
        uint32_t q = wave * PW + j * 64 + lane;
        bool valid = q < m;
        uint32_t idx = valid ? perm0[q] : 0u;
        uint32_t v = valid ? key_digit(lds_key<RW>(stage, idx, c.kf), s, R - 1, c.kf) : 0u;
        rp[j] = rank_issue(&S.wcnt[wave * RB], v, d, valid);
        dg[j] = v;
        ix[j] = idx;
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < MAX_ROUNDS; j++)
      if (j < NR) rk[j] = rank_finish(rp[j]);
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
  for (uint32_t q = threadIdx.x; q < m; q += WG) store_rec<RW>(c.rec0, begin + q, lds_get<RW>(stage, perm0[q]), false);
  __syncthreads();
}

// Stage a job (unless `staged`: its records are in the LDS stage already);
// returns false when it is finished already (at most one record, or every
// key equal), after putting it in records if it lay in tmp.
template <int RW>
__device__ __forceinline__ bool wg_begin(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp, Key& vary, bool staged) {
  if (m <= 1) {
    if (m == 1 && in_tmp && threadIdx.x == 0) store_rec<RW>(c.rec0, begin, load_rec<RW>(c.rec1, begin), false);
    __syncthreads();
    return false;
  }
  vary = staged ? stage_vary<RW>(c, m) : wg_stage<RW>(c, begin, m, in_tmp);
  if (vary.lo == 0 && vary.hi == 0) {
    if (in_tmp)
      for (uint32_t q = threadIdx.x; q < m; q += WG) store_rec<RW>(c.rec0, begin + q, lds_get<RW>(c.dyn, q), false);
    __syncthreads();
    return false;
  }
  return true;
}

template <int RW>
__device__ __forceinline__ void wg_finish(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp, uint32_t proc,
                                          bool staged = false) {
  Key vary;
  if (wg_begin<RW>(c, begin, m, in_tmp, vary, staged)) wg_sort_staged<RW>(c, begin, m, proc, vary);
}

// RADIX on a job that fits LDS: the next radix pass of the bin is made in
// fast memory and the bins it yields are sorted directly (paper, Sec.
// 3.4-3.5, which uses insertion sort on bins of at most 32 keys there).  The
// composites (varying key bits << ib | local index) are counted by their top
// D <= 10 bits and placed in digit order (any order within a digit); then
// each composite's final slot is its sub-bucket's start plus the number of
// smaller composites in the sub-bucket -- the insertion sort's result,
// computed by independent LDS reads instead of a chain of shifts.  The
// composites are unique, so the result is the stable order.  A sub-bucket
// above RANK_SUB_MAX composites (a skewed job: runs of equal keys) makes the workgroup
// finish the job from the same stage by the bitonic network instead (by LSD
// if the job exceeds the bitonic capacity), which costs the same whatever
// the duplicates.  With wide keys (varying bits plus index
// bits above 64) the composite keeps only the top varying bits, and
// composites that tie there are ordered by the staged full keys, then by
// index, so the slots stay exact.
template <int RW>
__device__ __forceinline__ void wg_radix_lds(Ctx& c, uint64_t begin, uint32_t m, bool in_tmp, bool staged) {
  SmallShared& S = *c.S;
  uint32_t* cnt = S.wcnt;  // NWAVES * RB >= 1024 counters
  // cleared before the stage's first barrier (the previous job ended with one)
  for (uint32_t v = threadIdx.x; v < 1024; v += WG) cnt[v] = 0;
  Key vary;
  if (!wg_begin<RW>(c, begin, m, in_tmp, vary, staged)) return;
  const uint32_t lo = ctz128(vary);
  const uint32_t W = bitlen128(vary) - lo;
  const uint32_t ib = 32 - __clz(m - 1);
  // the composite holds the top Wt varying bits; when that drops some
  // (wide keys), equal composite keys are ordered by the full key from the
  // stage, then by index
  const uint32_t Wt = min(W, 64 - ib);
  const bool trunc = Wt < W;
  const uint32_t C = c.p.c_fin;
  const uint32_t* stage = c.dyn;
  uint64_t* c0 = reinterpret_cast<uint64_t*>(c.dyn + C * RW);
  uint64_t* c1 = c0 + C;
  const uint32_t D = min(10u, Wt);
  const uint32_t R = 1u << D;
  const uint32_t dsh = ib + Wt - D;
  const uint32_t ksh = lo + W - Wt;
  const uint64_t wmask = Wt >= 64 ? ~0ull : ((1ull << Wt) - 1);
  const uint64_t imask = (1ull << ib) - 1;
  for (uint32_t q = threadIdx.x; q < m; q += WG) {
    uint64_t x = ((shr128(lds_key<RW>(stage, q, c.kf), ksh).lo & wmask) << ib) | q;
    c0[q] = x;
    atomicAdd(&cnt[(uint32_t)(x >> dsh)], 1u);
  }
  __syncthreads();
  // counts -> sub-bucket starts (exclusive scan), and the largest count
  {
    const uint32_t t = threadIdx.x;
    const uint32_t per = (R + WG - 1) / WG;
    const uint32_t a = min(R, t * per), e = min(R, a + per);
    uint32_t sum = 0, mx = 0;
    for (uint32_t i = a; i < e; i++) { const uint32_t x = cnt[i]; sum += x; mx = max(mx, x); }
    uint32_t wtot;
    uint32_t ex = wave_excl_scan(sum, &wtot);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o));
    if (lane_id() == 0) { S.scan_tmp[t / 64] = wtot; S.tcnt[t / 64] = mx; }
    __syncthreads();
    uint32_t base = 0, big = 0;
#pragma unroll
    for (uint32_t q = 0; q < NWAVES; q++) {
      if (q < t / 64) base += S.scan_tmp[q];
      big = max(big, S.tcnt[q]);
    }
    uint32_t run = base + ex;
    for (uint32_t i = a; i < e; i++) { const uint32_t x = cnt[i]; cnt[i] = run; run += x; }
    S.bcast = big;  // the same value from every thread
  }
  __syncthreads();
  if (S.bcast > RANK_SUB_MAX) {
    wg_sort_staged<RW>(c, begin, m, m <= c.p.bitonic_max ? P_BITONIC : P_LSD, vary);
    return;
  }
  for (uint32_t q = threadIdx.x; q < m; q += WG) {
    uint64_t x = c0[q];
    c1[atomicAdd(&cnt[(uint32_t)(x >> dsh)], 1u)] = x;
  }
  __syncthreads();
  // cnt[v] is now the end of sub-bucket v
  for (uint32_t q = threadIdx.x; q < m; q += WG) {
    const uint64_t x = c1[q];
    const uint32_t v = (uint32_t)(x >> dsh);
    const uint32_t s0 = v ? cnt[v - 1] : 0u, e = cnt[v];
    uint32_t below = 0;
    if (!trunc) {
      for (uint32_t i = s0; i < e; i++) below += c1[i] < x ? 1u : 0u;
    } else {
      const uint64_t xk = x >> ib;
      const uint32_t xi = (uint32_t)(x & imask);
      for (uint32_t i = s0; i < e; i++) {
        const uint64_t y = c1[i];
        const uint64_t yk = y >> ib;
        bool lt = yk < xk;
        if (yk == xk && y != x) {
          const Key ky = lds_key<RW>(stage, (uint32_t)(y & imask), c.kf);
          const Key kx = lds_key<RW>(stage, xi, c.kf);
          lt = key_less(ky, kx) || (!key_less(kx, ky) && (uint32_t)(y & imask) < xi);
        }
        below += lt ? 1u : 0u;
      }
    }
    c0[s0 + below] = x;
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < m; q += WG)
    store_rec<RW>(c.rec0, begin + q, lds_get<RW>(stage, (uint32_t)(c0[q] & imask)), false);
  __syncthreads();
}

// Copy a finished bucket from tmp to records.
template <int RW>
__device__ __forceinline__ void wg_copy(Ctx& c, uint64_t begin, uint64_t m) {
  for (uint64_t q = threadIdx.x; q < m; q += WG) store_rec<RW>(c.rec0, begin + q, load_rec<RW>(c.rec1, begin + q), false);
}

// One radix pass of a bucket by the workgroup (the paper's per-bin split,
// Sec. 3.4).  Sweep 1 counts digits and finds the bits all keys share (they
// are skipped); sweep 2 moves records tile by tile to the other buffer, each
// tile ranked stably and staged in LDS, digit runs appended in tile order.
// Fills the child list.  Returns false if every key is equal (the bucket is
// then already finished in records).
template <int RW>
__device__ __forceinline__ bool block_pass(Ctx& c, const Bucket& b) {
  SmallShared& S = *c.S;
  const uint32_t wave = threadIdx.x / 64, lane = lane_id();
  const bool in_tmp = b.flags & BF_TMP;
  const uint8_t* src = in_tmp ? c.rec1 : c.rec0;
  uint8_t* dst = in_tmp ? c.rec0 : c.rec1;
  const uint32_t m = (uint32_t)b.count;
  const uint32_t KB = c.kf.kbits;
  uint32_t bit = b.bit;
  uint32_t d, R, shift;
  if (threadIdx.x == 0) atomicAdd(&c.w.ctl->stage_records[0], (unsigned long long)m);
  Key ref = load_key<RW>(src, b.begin, c.kf);
  for (;;) {
    d = min(c.p.d_block, KB - bit);
    R = 1u << d;
    shift = KB - bit - d;
    for (uint32_t v = threadIdx.x; v < NWAVES * RB; v += WG) S.wcnt[v] = 0;
    __syncthreads();
    uint32_t* wh = &S.wcnt[wave * RB];  // this wave's counters
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
        uint32_t v = key_digit(kk[u], shift, R - 1, c.kf);
        // one LDS add per key, or one per wave when all 64 keys share the digit
        const uint64_t active = __ballot(valid);
        const uint32_t v0 = __shfl(v, 0);
        if (active == ~0ull && __ballot(v == v0) == ~0ull) {
          if (lane == 0) atomicAdd(&wh[v0], 64u);
        } else if (valid) {
          atomicAdd(&wh[v], 1u);
        }
      }
    }
    vlo = wave_or64(vlo);
    vhi = wave_or64(vhi);
    if (lane == 0) { S.vary[2 * wave] = vlo; S.vary[2 * wave + 1] = vhi; }
    __syncthreads();
    for (uint32_t v = threadIdx.x; v < R; v += WG) {
      uint32_t h = 0;
#pragma unroll
      for (int q = 0; q < NWAVES; q++) h += S.wcnt[q * RB + v];
      S.hist[v] = h;
    }
    Key vary{0, 0};
#pragma unroll
    for (int q = 0; q < NWAVES; q++) { vary.lo |= S.vary[2 * q]; vary.hi |= S.vary[2 * q + 1]; }
    vary = vary;
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
  for (uint32_t v = threadIdx.x; v < R; v += WG) { S.ccnt[v] = S.hist[v]; S.toff[v] = S.hist[v]; }
  __syncthreads();
  block_excl_scan_lds(S.toff, R, S.scan_tmp);
  for (uint32_t v = threadIdx.x; v < R; v += WG) { S.cbase[v] = S.toff[v]; S.run[v] = S.toff[v]; }
  if (threadIdx.x == 0) {
    S.cbit = bit + d;
    S.pbit = bit;
    S.cR = R;
    S.ctmp = in_tmp ? 0u : 1u;
    S.cbegin = b.begin;
    S.cparent = m;
  }
  __syncthreads();
  // sweep 2: stable tiles through LDS
  const uint32_t BT = c.p.block_tile;
  const uint32_t per_wave = BT / NWAVES;
  const uint32_t IPT = BT / WG;
  constexpr uint32_t IPT_MAX = (RW >= 2 ? 64 / RW : 32) < IPT_BLOCK ? (RW >= 2 ? 64 / RW : 32) : IPT_BLOCK;
  // each tile's records are loaded while the tile before it is written out
  Rec<RW> rec[IPT_MAX];
  auto load_tile = [&](uint32_t t) {
#pragma unroll
    for (uint32_t j = 0; j < IPT_MAX; j++) {
      uint32_t q = t + wave * per_wave + j * 64 + lane;
      if (j < IPT && q < m) rec[j] = load_rec<RW>(src, b.begin + q);
    }
  };
  for (uint32_t i = threadIdx.x; i < NWAVES * RB; i += WG) S.wcnt[i] = 0;
  load_tile(0);
  __syncthreads();
  for (uint32_t t0 = 0; t0 < m; t0 += BT) {
    const uint32_t cnt = min(BT, m - t0);
    uint32_t dg[IPT_MAX], rk[IPT_MAX];
    const uint32_t wb = t0 + wave * per_wave;
    RankPart rp[IPT_MAX];
#pragma unroll
    for (uint32_t j = 0; j < IPT_MAX; j++) {
      if (j < IPT) {
        uint32_t q = wb + j * 64 + lane;
        bool valid = q < m;
        uint32_t v = valid ? key_digit(rec_key<RW>(rec[j], c.kf), shift, R - 1, c.kf) : 0u;
        rp[j] = rank_issue(&S.wcnt[wave * RB], v, d, valid);
        dg[j] = v;
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < IPT_MAX; j++)
      if (j < IPT) rk[j] = rank_finish(rp[j]);
    tile_offsets(S, R);
#pragma unroll
    for (uint32_t j = 0; j < IPT_MAX; j++) {
      uint32_t q = wb + j * 64 + lane;
      if (j < IPT && q < m) lds_put<RW>(c.dyn, S.toff[dg[j]] + S.wcnt[wave * RB + dg[j]] + rk[j], rec[j]);
    }
    if (t0 + BT < m) load_tile(t0 + BT);
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < cnt; q += WG) {
      Rec<RW> r = lds_get<RW>(c.dyn, q);
      uint32_t v = key_digit(rec_key<RW>(r, c.kf), shift, R - 1, c.kf);
      store_rec<RW>(dst, b.begin + S.run[v] + (q - S.toff[v]), r, false);
    }
    __syncthreads();
    for (uint32_t v = threadIdx.x; v < R; v += WG) S.run[v] += S.tcnt[v];
    for (uint32_t i = threadIdx.x; i < NWAVES * RB; i += WG) S.wcnt[i] = 0;
    __syncthreads();
  }
  return true;
}

// ---------------------------------------------------------------------------
// Tracing: one row per scheduled job.
__device__ __forceinline__ void trace_row(Ctx& c, uint64_t m, uint64_t parent, uint32_t bit, uint32_t chosen, uint32_t observed,
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

template <int RW>
__device__ __forceinline__ void run_job(Ctx& c, uint32_t proc, uint64_t begin, uint32_t m, bool in_tmp, bool staged);

// Is this job sampled for counterfactual timing?  (Workgroup-uniform.)
__device__ __forceinline__ bool sample_job(Ctx& c, uint32_t feas) {
  if (!c.w.trace || !c.p.sample_period || __popc(feas) < 2) return false;
  SmallShared& S = *c.S;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t k = S.decisions++;
    S.bcast = ((k + blockIdx.x * 7919u) % c.p.sample_period) == 0 ? 1u : 0u;
  }
  __syncthreads();
  bool s = S.bcast != 0;
  __syncthreads();
  return s;
}

// Schedule and run one workgroup job of m <= C records (a queued bucket or a
// child), tracing it if asked.  In a counterfactual sample every feasible
// procedure runs in turn on the same input (each is a complete stable sort,
// so later runs see input that is already in order and rewrite the same
// bytes) and the chosen one runs last.
template <int RW>
__device__ __forceinline__ void schedule_job(Ctx& c, uint64_t begin, uint32_t m, uint32_t bit, bool in_tmp,
                                             uint64_t parent, JobRegs<RW>& jr, uint64_t nbegin, uint32_t nm,
                                             bool ntmp) {
  const uint32_t KB = c.kf.kbits;
  const uint32_t feas = feasible_mask(c.p, m, bit, KB, true);
  uint32_t proc;
  if (c.p.sched_mode == RADULS_SCHED_LEARNED && c.model && __popc(feas) > 1) {
    // every wavefront evaluates the network on the same inputs by the same
    // instructions, so all reach the same choice without a barrier
    proc = choose_proc_wave<true>(c.p, c.model, m, parent, bit, KB, feas);
  } else {
    proc = choose_proc<true>(c.p, c.model, m, parent, bit, KB, feas);
  }
  const bool cf = sample_job(c, feas);
  const uint32_t runs = cf ? 3u : 1u;
  uint32_t ticks[3] = {0, 0, 0};
  // A sample keeps its input: a job that lies in records is first copied to
  // the same place in tmp, and every run then reads tmp and writes records,
  // so each procedure sees the same unsorted input.  It also first runs the
  // chosen procedure untimed, so every timed run finds the records in cache
  // alike.
  bool src_tmp = in_tmp;
  if (cf && !in_tmp) {
    for (uint32_t q = threadIdx.x; q < m; q += WG) store_rec<RW>(c.rec1, begin + q, load_rec<RW>(c.rec0, begin + q), false);
    src_tmp = true;
  }
  // This job's records arrived in registers while the previous job ran:
  // stage them (a sample re-reads its input for every run instead), then
  // start loading the next job's records into the same registers.
  const bool staged = !cf && m > 1;
  if (staged) regs_stage<RW>(c, jr, m);
  regs_load<RW>(c, jr, nbegin, nm, ntmp);
#pragma unroll 1
  for (uint32_t k = cf ? 0u : 1u; k <= runs; k++) {
    const uint32_t q = cf ? (proc + k) % 3 : proc;
    if (!((feas >> q) & 1u) && cf) continue;
    if (cf) __syncthreads();
    uint64_t t0 = now_ticks();
    run_job<RW>(c, q, begin, m, src_tmp, staged);  // every procedure ends with a barrier
    if (k > 0) ticks[q] = (uint32_t)(now_ticks() - t0);
  }
  if (c.w.trace && __popc(feas) > 1 && threadIdx.x == 0)
    trace_row(c, m, parent, bit, proc, cf ? feas : (1u << proc), ticks, cf ? 1u : 0u);
}

// Group the children of the last radix pass into finishing jobs.  Children
// lie consecutively in key order, so a run of whole children is a valid job:
// sorting the run by key sorts each child and leaves the children in place.
// With T = the job window (at most C/2), a child above T is a job of its own
// and smaller children are grouped by the T-window their first record falls
// in, so a group holds at most 2T <= C records.  Jobs of at most the
// wavefront capacity go to the wavefront list, larger ones are deferred to
// the global workgroup-job list, and a child above C goes to the
// workgroup's stack.  All threads take part.
template <int RW>
__device__ __forceinline__ void build_jobs(Ctx& c) {
  SmallShared& S = *c.S;
  const uint32_t C = c.p.c_fin;
  const uint32_t WSC = c.p.wave_cap;
  const uint32_t KB = c.kf.kbits;
  // with register finishing, groups keep the parent's resolved bits and are
  // bounded by what a job with those bits may hold
  const uint32_t T = c.p.fin_max ? (uint32_t)min<uint64_t>(c.p.job_window, max<uint64_t>(job_cap(c.p, S.pbit, KB) / 2, 32))
                                 : c.p.job_window;
  const uint32_t R = S.cR;
  const uint32_t t = threadIdx.x;
  // 1. compact the non-empty children (stable)
  const uint32_t cnt = t < R ? S.ccnt[t] : 0u;
  const uint32_t st = t < R ? S.cbase[t] : 0u;
  S.toff[t] = cnt > 0 ? 1u : 0u;
  if (t == 0) { S.nw = 0; S.wnext = 0; }
  __syncthreads();
  const uint32_t nn = block_excl_scan_lds(S.toff, WG, S.scan_tmp);
  if (cnt > 0) { S.jb[S.toff[t]] = st; S.jn[S.toff[t]] = cnt; }
  __syncthreads();
  // 2. job boundaries among the compacted children
  uint32_t kst = 0, kcnt = 0, kbnd = 0;
  if (t < nn) {
    kst = S.jb[t];
    kcnt = S.jn[t];
    kbnd = 1;
    if (t > 0) {
      uint32_t pst = S.jb[t - 1], pcnt = S.jn[t - 1];
      kbnd = (kcnt > T || pcnt > T || kst / T != pst / T) ? 1u : 0u;
    }
  }
  __syncthreads();
  S.toff[t] = kbnd;
  __syncthreads();
  const uint32_t nj = block_excl_scan_lds(S.toff, WG, S.scan_tmp);
  // job j: start (cbase[j]) and size of its first child (ccnt[j]); cbase[nj]
  // is the end of the last child
  if (kbnd) { S.cbase[S.toff[t]] = kst; S.ccnt[S.toff[t]] = kcnt; }
  if (t < nn && t + 1 == nn) S.cbase[nj] = kst + kcnt;
  __syncthreads();
  // 3. classify the jobs (one per thread) and choose their procedures
  const uint32_t cb = S.cbit, pb = S.pbit;
  const bool ctmp = S.ctmp != 0;
  const uint64_t parent = S.cparent;
  for (uint32_t j = t; j < nj; j += WG) {
    const uint32_t js = S.cbase[j];
    const uint32_t m = S.cbase[j + 1] - js;
    const uint32_t bit = m == S.ccnt[j] ? cb : pb;
    const uint32_t ib = 32 - __clz(m > 1 ? m - 1 : 1);
    if (m > C && c.p.fin_max && job_ok(c.p, m, bit, KB)) {
      uint32_t i = atomicAdd(&c.w.ctl->nwg, 1u);
      if (i < c.p.cap_wg) c.w.wgjobs[i] = Bucket{S.cbegin + js, m, parent, bit, (ctmp ? BF_TMP : 0u) | (bit == pb ? BF_GROUP : 0u)};
      else atomicOr(&c.w.ctl->overflow, 32u);
      continue;
    }
    if (m > C) {
      uint32_t sp = atomicAdd(&S.sp, 1u);
      if (sp < c.p.stack_cap) c.stack[sp] = Bucket{S.cbegin + js, m, parent, cb, ctmp ? BF_TMP : 0u};
      else atomicOr(&c.w.ctl->overflow, 16u);
      continue;
    }
    if (m <= TINY_MAX || (m <= WSC && (KB - bit) + ib <= 128)) {
      uint32_t feas = m > TINY_MAX ? feasible_mask(c.p, m, bit, KB, false) : 0u;
      uint32_t proc = __popc(feas) > 1 ? choose_proc<true>(c.p, c.model, m, parent, bit, KB, feas)
                                       : (feas ? (uint32_t)(__ffs(feas) - 1) : P_LSD);
      uint32_t sampled = 0;
      if (c.w.trace && c.p.sample_period && __popc(feas) > 1) {
        uint32_t k = atomicAdd(&S.decisions, 1u);
        sampled = ((k + blockIdx.x * 7919u) % c.p.sample_period) == 0 ? 1u : 0u;
      }
      uint32_t slot = atomicAdd(&S.nw, 1u);
      S.jb[slot] = js;
      S.jn[slot] = m;
      S.jinfo[slot] = bit | (proc << 16) | (sampled << 24) | ((feas & 7u) << 28);
      continue;
    }
    uint32_t i = atomicAdd(&c.w.ctl->nwg, 1u);
    if (i < c.p.cap_wg) c.w.wgjobs[i] = Bucket{S.cbegin + js, m, parent, bit, (ctmp ? BF_TMP : 0u) | (bit == pb ? BF_GROUP : 0u)};
    else atomicOr(&c.w.ctl->overflow, 32u);
  }
  __syncthreads();
}

// Wavefront jobs: each wave takes the next job (no workgroup barrier); a job
// of at most 32 records is ranked (the insertion-sort slot of the paper),
// others get the chosen procedure -- or, if sampled, every feasible one in
// turn with the chosen one last, each timed.
template <int RW>
__device__ __forceinline__ void run_wave_jobs(Ctx& c) {
  SmallShared& S = *c.S;
  const uint32_t WSC = c.p.wave_cap;
  const uint32_t wave = threadIdx.x / 64;
  uint32_t* reg = c.dyn + wave * (WSC * RW + 4 * WSC + RB);
  // The claim loops below keep their bounds and claims in scalar registers
  // (readfirstlane of values every lane holds alike), so the loop exit is
  // uniform and the compiler cannot split a wave across iterations: with a
  // per-lane bound it may send lane 0 (the one that claims) out of the loop
  // while the other lanes keep reading a stale claim.
  const uint32_t nw = __builtin_amdgcn_readfirstlane(S.nw);
  const bool ctmp = S.ctmp != 0;
  const uint64_t base = S.cbegin;
  const uint64_t parent = S.cparent;
  for (;;) {
    uint32_t i = 0;
    if (lane_id() == 0) i = atomicAdd(&S.wnext, 1u);
    i = __builtin_amdgcn_readfirstlane(__shfl(i, 0));
    if (i >= nw) break;
    const uint32_t m = S.jn[i];
    const uint32_t info = S.jinfo[i];
    const uint64_t jb = base + S.jb[i];
    if (lane_id() == 0) atomicAdd(&c.w.ctl->stage_records[1], (unsigned long long)m);
    if (m <= TINY_MAX) {
      wave_rank<RW>(c, jb, m, ctmp);
      continue;
    }
    const uint32_t bit = info & 0xFFu, proc = (info >> 16) & 0xFu, feas = (info >> 28) & 7u;
    const bool cf = (info >> 24) & 1u;
    uint32_t ticks[3] = {0, 0, 0};
    const uint32_t runs = cf ? 3u : 1u;
    const bool narrow = (c.kf.kbits - bit) + (32 - __clz(m - 1)) <= 64;
    // a sample keeps its input in tmp (see schedule_job)
    bool src_tmp = ctmp;
    if (cf && !ctmp) {
      for (uint32_t q = lane_id(); q < m; q += 64) store_rec<RW>(c.rec1, jb + q, load_rec<RW>(c.rec0, jb + q), false);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      src_tmp = true;
    }
#pragma unroll 1
    for (uint32_t k = cf ? 0u : 1u; k <= runs; k++) {  // k = 0: untimed warm-up of a sample
      const uint32_t q = cf ? (proc + k) % 3 : proc;
      if (cf && !((feas >> q) & 1u)) continue;
      uint64_t t0 = now_ticks();
      if (narrow) wave_sort64<RW>(c, jb, m, src_tmp, q, reg);
      else wave_sort<RW>(c, jb, m, src_tmp, q, reg);
      if (k > 0) ticks[q] = (uint32_t)((now_ticks() - t0 + 2) / 4);  // one wave of four
    }
    if (c.w.trace && __popc(feas) > 1 && lane_id() == 0)
      trace_row(c, m, parent, bit, proc, cf ? feas : (1u << proc), ticks, (cf ? 1u : 0u) | 2u);
  }
  __syncthreads();
}

// Finish the children of the last radix pass: wavefront jobs now, workgroup
// jobs deferred to the jobs kernel.
template <int RW>
__device__ __forceinline__ void finish_children(Ctx& c) {
  build_jobs<RW>(c);
  run_wave_jobs<RW>(c);
}

// A job of m <= C records by the chosen procedure.
template <int RW>
__device__ __forceinline__ void run_job(Ctx& c, uint32_t proc, uint64_t begin, uint32_t m, bool in_tmp, bool staged) {
  if (proc == P_RADIX) wg_radix_lds<RW>(c, begin, m, in_tmp, staged);
  else wg_finish<RW>(c, begin, m, in_tmp, proc == P_BITONIC ? P_BITONIC : P_LSD, staged);
}

__device__ __forceinline__ void init_ctx(Ctx& c, const Plan& p, const Work& w, uint8_t* rec0, uint8_t* rec1,
                                         SmallShared* S, uint32_t* dyn) {
  c.p = p;
  c.w = w;
  c.rec0 = rec0;
  c.rec1 = rec1;
  c.kf = make_keyfmt(p.key_bytes);
  c.S = S;
  c.dyn = dyn;
  c.stack = w.stacks + (uint64_t)blockIdx.x * p.stack_cap;
  c.model = nullptr;
  if (p.sched_mode == RADULS_SCHED_LEARNED && w.model) {
    constexpr uint32_t W2 = MLP_H * MLP_F + MLP_H, W2E = W2 + MLP_H * MLP_H;
    for (uint32_t i = threadIdx.x; i < MLP_MODEL_FLOATS; i += WG) {
      uint32_t d = i;
      if (i >= W2 && i < W2E) d = W2 + ((i - W2) % MLP_H) * MLP_H + (i - W2) / MLP_H;
      S->model[d] = w.model[i];
    }
    c.model = S->model;
  }
  if (threadIdx.x == 0) { S->sp = 0; S->decisions = 0; }
  __syncthreads();
}

// Pass A: buckets above C records (radix pass, then their children) from the
// queue and the stack; tiny buckets; everything else is deferred to pass B.
template <int RW>
__global__ __launch_bounds__(WG) void k_small(Plan p, Work w, uint8_t* rec0, uint8_t* rec1) {
  extern __shared__ __align__(16) uint32_t dyn[];
  __shared__ SmallShared S;
  Ctx c;
  init_ctx(c, p, w, rec0, rec1, &S, dyn);
  const uint32_t ns = (uint32_t)min((uint64_t)w.ctl->nsmall, p.cap_small);
  for (;;) {
    if (threadIdx.x == 0) S.bcast = atomicAdd(&w.ctl->small_head, 1u);
    __syncthreads();
    const uint32_t idx = S.bcast;
    __syncthreads();
    if (idx >= ns) break;
    Bucket b = w.small_ord[idx];
    if (b.count <= p.c_fin) {
      if (b.count <= TINY_MAX) {
        if (threadIdx.x < 64) wave_rank<RW>(c, b.begin, (uint32_t)b.count, (b.flags & BF_TMP) != 0);
      } else if (threadIdx.x == 0) {
        uint32_t i = atomicAdd(&w.ctl->nwg, 1u);
        b.flags |= BF_ROOT;
        if (i < p.cap_wg) w.wgjobs[i] = b;
        else atomicOr(&w.ctl->overflow, 32u);
      }
      __syncthreads();
      continue;
    }
    if (block_pass<RW>(c, b)) finish_children<RW>(c);
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
      if (block_pass<RW>(c, b2)) finish_children<RW>(c);
    }
  }
  // tiny buckets, one wavefront each
  // scalar bound and claim, as in run_wave_jobs
  const uint32_t nt = __builtin_amdgcn_readfirstlane((uint32_t)min((uint64_t)w.ctl->ntiny, p.cap_tiny));
  for (;;) {
    uint32_t j = 0;
    if (lane_id() == 0) j = atomicAdd(&w.ctl->tiny_head, 1u);
    j = __builtin_amdgcn_readfirstlane(__shfl(j, 0));
    if (j >= nt) break;
    uint64_t x = w.tiny[j];
    uint64_t begin = x & ((1ull << 40) - 1);
    uint32_t cnt = (uint32_t)(x >> 40) & 63u;
    bool tmp = (x >> 46) & 1u;
    if (lane_id() == 0) atomicAdd(&w.ctl->stage_records[3], (unsigned long long)cnt);
    wave_rank<RW>(c, begin, cnt, tmp);
  }
}

// Pass B: jobs of at most C records -- queued buckets and groups of
// children deferred by pass A -- each by its scheduled procedure.
template <int RW>
__global__ __launch_bounds__(WG) void k_small_jobs(Plan p, Work w, uint8_t* rec0, uint8_t* rec1) {
  extern __shared__ __align__(16) uint32_t dyn[];
  __shared__ SmallShared S;
  Ctx c;
  init_ctx(c, p, w, rec0, rec1, &S, dyn);
  const uint32_t nj = (uint32_t)min((uint64_t)w.ctl->nwg, p.cap_wg);
  // Each job is claimed one job ahead, and its records are loaded into
  // registers while the workgroup sorts the job before it.
  JobRegs<RW> jr;
  if (threadIdx.x == 0) S.bcast = atomicAdd(&w.ctl->wg_head, 1u);
  __syncthreads();
  uint32_t idx = S.bcast;
  __syncthreads();
  if (idx < nj) {
    const Bucket b = w.wgjobs[idx];
    regs_load<RW>(c, jr, b.begin, (uint32_t)b.count, (b.flags & BF_TMP) != 0);
  }
  while (idx < nj) {
    const Bucket b = w.wgjobs[idx];
    if (threadIdx.x == 0) S.bcast = atomicAdd(&w.ctl->wg_head, 1u);
    __syncthreads();
    const uint32_t nidx = S.bcast;
    __syncthreads();
    Bucket nb{0, 0, 0, 0, 0};
    if (nidx < nj) nb = w.wgjobs[nidx];
    if (threadIdx.x == 0) atomicAdd(&w.ctl->stage_records[2], (unsigned long long)b.count);
    schedule_job<RW>(c, b.begin, (uint32_t)b.count, b.bit, (b.flags & BF_TMP) != 0, b.parent, jr, nb.begin,
                     (uint32_t)nb.count, (nb.flags & BF_TMP) != 0);
    idx = nidx;
  }
}

uint32_t small_dynamic_lds(const Plan& p) {
  uint32_t r = p.rec_bytes;
  uint32_t block = p.block_tile * r;
  uint32_t fin = p.c_fin * r + 16u * p.c_fin;
  uint32_t waves = NWAVES * (p.wave_cap * r + 16u * p.wave_cap + 4u * RB);
  return max(block, max(fin, waves));
}

void launch_small(const Plan& p, const Work& w, void* records, void* tmp, hipStream_t s) {
  uint32_t lds = small_dynamic_lds(p);
  uint8_t* r0 = (uint8_t*)records;
  uint8_t* r1 = (uint8_t*)tmp;
  switch (p.rw) {
#define RD_CASE(n)                                                   \
  case n:                                                            \
    k_small<n><<<p.grid_small, WG, lds, s>>>(p, w, r0, r1);          \
    break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

void launch_small_jobs(const Plan& p, const Work& w, void* records, void* tmp, hipStream_t s) {
  uint32_t lds = small_dynamic_lds(p);
  uint8_t* r0 = (uint8_t*)records;
  uint8_t* r1 = (uint8_t*)tmp;
  switch (p.rw) {
#define RD_CASE(n)                                                   \
  case n:                                                            \
    k_small_jobs<n><<<p.grid_small, WG, lds, s>>>(p, w, r0, r1);     \
    break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

}  // namespace rd
