// k_finish.hip -- finishing jobs held in registers.
//
// The paper finishes a bin once it is small enough to be sorted where it
// sits in fast memory (Sec. 3.4-3.5).  On this GPU the largest fast memory a
// single workgroup owns is its register file: a 1024-thread workgroup holds
// E records per thread (16K records of 16 bytes is 256 KiB of a CU's
// 512 KiB), so one workgroup finishes a whole bucket of up to 1024*E records
// with one read and one write of every record:
//
//   1. every thread loads E records of the job into registers (coalesced);
//   2. the bits that vary over the job are found (OR of key XOR first key);
//   3. the top D <= 11 of them form a digit; one counting pass in LDS
//      (counts, exclusive scan, atomic slots) places every record's
//      composite (key bits below the digit) << ib | index in its digit's
//      sub-bin, in any order;
//   4. a record's final slot is its sub-bin's start plus the number of
//      smaller composites in the sub-bin (the slot insertion sort would give
//      it, Sec. 3.5); sub-bins above FSUB composites (runs of equal or close
//      keys) are first sorted by a bitonic network run by one wavefront,
//      and a record then finds its slot by binary search;
//   5. the records go out through LDS in slot order, a slice of the job per
//      round, with coalesced stores to `records`.
//
// Composites are unique (they hold the index), so every step's result is
// the stable order whatever order the atomics gave.  A job qualifies when
// its key bits below the digit plus the index bits fit the composite (the
// levels route only such jobs here): 64 bits for keys of at most 8 bytes,
// 128 bits for longer keys, whose jobs hold half as many records (the
// composites of a job fill the same LDS).  Jobs whose keys are all equal are
// written unchanged.
#include <type_traits>

#include "raduls_dev.hpp"
#include "raduls_kernels.hpp"

namespace rd {

// 128-bit keys and composites of jobs with keys above 8 bytes.
struct FU128 {
  uint64_t lo, hi;
};
__device__ __forceinline__ FU128 operator^(FU128 a, FU128 b) { return FU128{a.lo ^ b.lo, a.hi ^ b.hi}; }
__device__ __forceinline__ FU128 operator|(FU128 a, FU128 b) { return FU128{a.lo | b.lo, a.hi | b.hi}; }
__device__ __forceinline__ FU128 operator&(FU128 a, FU128 b) { return FU128{a.lo & b.lo, a.hi & b.hi}; }
__device__ __forceinline__ FU128 operator|(FU128 a, uint32_t q) { return FU128{a.lo | q, a.hi}; }
__device__ __forceinline__ FU128 operator>>(FU128 a, uint32_t s) {
  if (s == 0) return a;
  if (s >= 64) return FU128{s >= 128 ? 0ull : a.hi >> (s - 64), 0ull};
  return FU128{(a.lo >> s) | (a.hi << (64 - s)), a.hi >> s};
}
__device__ __forceinline__ FU128 operator<<(FU128 a, uint32_t s) {
  if (s == 0) return a;
  if (s >= 64) return FU128{0ull, s >= 128 ? 0ull : a.lo << (s - 64)};
  return FU128{a.lo << s, (a.hi << s) | (a.lo >> (64 - s))};
}
__device__ __forceinline__ bool operator<(FU128 a, FU128 b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
__device__ __forceinline__ bool operator>(FU128 a, FU128 b) { return b < a; }
__device__ __forceinline__ bool operator==(FU128 a, FU128 b) { return a.lo == b.lo && a.hi == b.hi; }
__device__ __forceinline__ bool operator!=(FU128 a, FU128 b) { return !(a == b); }

// the same operations on both key types
__device__ __forceinline__ uint32_t low32(uint64_t x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t low32(FU128 x) { return (uint32_t)x.lo; }
__device__ __forceinline__ bool is_zero(uint64_t x) { return x == 0; }
__device__ __forceinline__ bool is_zero(FU128 x) { return (x.lo | x.hi) == 0; }
__device__ __forceinline__ uint32_t lowest_bit(uint64_t x) { return (uint32_t)__builtin_ctzll(x); }
__device__ __forceinline__ uint32_t lowest_bit(FU128 x) {
  return x.lo ? (uint32_t)__builtin_ctzll(x.lo) : 64u + (uint32_t)__builtin_ctzll(x.hi);
}
__device__ __forceinline__ uint32_t bit_length(uint64_t x) { return 64u - (uint32_t)__clzll(x); }
__device__ __forceinline__ uint32_t bit_length(FU128 x) {
  return x.hi ? 128u - (uint32_t)__clzll(x.hi) : 64u - (uint32_t)__clzll(x.lo);
}
template <typename K>
__device__ __forceinline__ K zero_key() {
  if constexpr (std::is_same<K, FU128>::value) return FU128{0ull, 0ull};
  else return 0ull;
}
// bits [0, rb) set
template <typename K>
__device__ __forceinline__ K low_mask(uint32_t rb) {
  if constexpr (std::is_same<K, FU128>::value) {
    if (rb == 0) return FU128{0ull, 0ull};
    if (rb < 64) return FU128{(1ull << rb) - 1, 0ull};
    return FU128{~0ull, rb >= 128 ? ~0ull : (rb == 64 ? 0ull : ((1ull << (rb - 64)) - 1))};
  } else {
    return rb == 0 ? 0ull : (rb >= 64 ? ~0ull : ((1ull << rb) - 1));
  }
}
__device__ __forceinline__ uint64_t uniform_key(uint64_t x) { return uniform64(x); }
__device__ __forceinline__ FU128 uniform_key(FU128 x) { return FU128{uniform64(x.lo), uniform64(x.hi)}; }

constexpr int FWG = 1024;              // threads of a finishing workgroup
constexpr int FWAVES = FWG / 64;
constexpr uint32_t FSUB = 32;          // larger sub-bins are split or sorted by a wavefront network
constexpr uint32_t FIN_SPLIT_MAX = 64; // large sub-bins that may be split
constexpr uint32_t FIN_MINORS = 24;    // records of a split sub-bin outside its run of equal keys
constexpr uint32_t FIN_POOL_WAVE = 32; // pool of those records' composites, per wave

template <int RW, bool WIDE>
struct FinShape {
  static constexpr uint32_t E = WIDE ? fin_records_per_thread_wide(RW) : fin_records_per_thread(RW);
  static constexpr uint32_t M = E * FWG;
};

// K: the key and composite type (64-bit, or 128-bit for keys above 8 bytes,
// which keep half the pool so that the static LDS stays the same)
template <typename K>
struct FinShared {
  static constexpr uint32_t POOL_WAVE = sizeof(K) == 8 ? FIN_POOL_WAVE : FIN_POOL_WAVE / 2;
  K wv[FWAVES];                        // per-wave OR of key XOR reference
  uint32_t wsum[FWAVES];               // per-wave sums of the counter scan
  uint32_t wmax[FWAVES];
  uint32_t job[2];                     // claimed job index (by iteration parity)
  uint32_t nbig;                       // large sub-bins
  uint32_t ntop;                       // distinct top-8-bit values of a grouped job
  uint16_t big[FIN_LDS_BIG];           // digits of the large sub-bins
  uint8_t rank8[256];                  // grouped job: rank of a top-8-bit value among those present
  uint8_t btag[1u << FIN_DIGIT_BITS];  // sub-bin -> 1 + its index among the split ones, or 0
  // split large sub-bins (the first FIN_SPLIT_MAX of them in digit order)
  K bH[FIN_SPLIT_MAX];                 // the shared key part
  uint32_t binfo[FIN_SPLIT_MAX];       // pool offset | minors << 16
  uint32_t bless[FIN_SPLIT_MAX];       // minors with a smaller key part
  union {
    uint32_t h8[256];                  // grouped job: counts of the top 8 varying bits
    uint32_t cw[FWAVES * FIN_SPLIT_MAX];  // H records per wave, then those of earlier waves
  };
  K pool[POOL_WAVE * FWAVES];          // the minors' composites
};

static_assert(sizeof(FinShared<uint64_t>) <= FIN_STATIC_LDS, "static LDS of the finishing kernel");
static_assert(sizeof(FinShared<FU128>) <= FIN_STATIC_LDS, "static LDS of the finishing kernel");

// Keeps the scheduler from interleaving the unrolled per-record iterations
// (that would hold every iteration's temporaries at once and spill).
__device__ __forceinline__ void fin_sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// Wave reductions and scans by ds_bpermute on an explicit lane number (the
// lane is recomputed each job from a laundered thread index, so that none of
// the shuffle addresses is held in registers across the persistent loop).
__device__ __forceinline__ uint32_t fshfl(uint32_t x, uint32_t src_lane) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src_lane << 2), (int)x);
}
__device__ __forceinline__ uint64_t fwave_or64(uint64_t x, uint32_t lane) {
#pragma unroll
  for (uint32_t o = 32; o >= 1; o >>= 1) {
    const uint32_t lo = fshfl((uint32_t)x, lane ^ o), hi = fshfl((uint32_t)(x >> 32), lane ^ o);
    x |= (uint64_t)lo | ((uint64_t)hi << 32);
  }
  return x;
}
__device__ __forceinline__ FU128 fwave_or64(FU128 x, uint32_t lane) {
  return FU128{fwave_or64(x.lo, lane), fwave_or64(x.hi, lane)};
}
__device__ __forceinline__ uint32_t fwave_max(uint32_t x, uint32_t lane) {
#pragma unroll
  for (uint32_t o = 32; o >= 1; o >>= 1) x = max(x, fshfl(x, lane ^ o));
  return x;
}
// exclusive prefix sum over the wave; *total gets the wave's sum
__device__ __forceinline__ uint32_t fwave_excl_scan(uint32_t x, uint32_t lane, uint32_t* total) {
  uint32_t inc = x;
#pragma unroll
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const uint32_t y = fshfl(inc, lane >= o ? lane - o : lane);
    if (lane >= o) inc += y;
  }
  *total = fshfl(inc, 63);
  return inc - x;
}

// The key of a record held in registers, masked to the key bytes.  Each
// phase takes the mask through an empty asm statement, so that the masked
// keys are recomputed per phase (two instructions) rather than held for all
// E records across the phases.
template <int RW>
__device__ __forceinline__ uint64_t fkey(const Rec<RW>& r, uint64_t km) {
  uint64_t k = r.w[0];
  if constexpr (RW > 1) k |= (uint64_t)r.w[1] << 32;
  return k & km;
}
// the key as K: 64 bits (masks lo) or 128 bits (masks lo, hi)
template <typename K, int RW>
__device__ __forceinline__ K fkey_k(const Rec<RW>& r, uint64_t km, uint64_t kmh) {
  if constexpr (std::is_same<K, FU128>::value) {
    uint64_t h = 0;
    if constexpr (RW > 2) h = r.w[2];
    if constexpr (RW > 3) h |= (uint64_t)r.w[3] << 32;
    return FU128{fkey<RW>(r, km), h & kmh};
  } else {
    (void)kmh;
    return fkey<RW>(r, km);
  }
}
__device__ __forceinline__ uint64_t phase_mask(uint64_t km) {
  asm volatile("" : "+s"(km));
  return km;
}

__device__ __forceinline__ void fin_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Ascending bitonic network over c[0, s), run by one wavefront.  Positions
// at or above s act as +infinity: every comparator puts the smaller value
// at the lower index, so they never move and are never touched.  Each
// merge phase of block size k starts by comparing an element with its
// mirror in the block, then halves the distance down to 1.
template <typename T>
__device__ __forceinline__ void wave_bitonic(T* c, uint32_t s, uint32_t lane) {
  uint32_t P = 1;
  while (P < s) P <<= 1;
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = lane; i < P / 2; i += 64) {
        uint32_t a, b;
        if (j == (k >> 1)) {
          const uint32_t h = k >> 1;
          a = (i / h) * k + (i % h);
          b = (a / k) * k + (k - 1 - (a % k));
        } else {
          a = 2 * j * (i / j) + (i % j);
          b = a + j;
        }
        if (b < s) {
          const T x = c[a], y = c[b];
          if (x > y) { c[a] = y; c[b] = x; }
        }
      }
      fin_wave_sync();
    }
  }
}

template <int RW, bool WIDE>
__global__ __launch_bounds__(FWG) void k_fin_jobs(Plan p, Work w, uint8_t* rec0, uint8_t* rec1) {
  using K = typename std::conditional<WIDE, FU128, uint64_t>::type;  // keys and composites
  constexpr uint32_t E = FinShape<RW, WIDE>::E;
  constexpr uint32_t M = FinShape<RW, WIDE>::M;
  constexpr uint32_t CB = 8 * sizeof(K);   // composite bits
  constexpr uint32_t POOL_WAVE = FinShared<K>::POOL_WAVE;
  constexpr uint32_t RMAX = 1u << FIN_DIGIT_BITS;
  constexpr uint32_t NCW = RMAX / 2 + 1;  // counter words: two 16-bit counters each
  constexpr uint32_t RB = 4 * RW;  // record bytes
  extern __shared__ __align__(16) uint32_t dyn[];
  __shared__ FinShared<K> S;
  K* comp = reinterpret_cast<K*>(dyn);                        // M composites
  uint32_t* cnt = dyn + (sizeof(K) / 4) * M;                  // NCW words of packed counters
  uint32_t* stage = dyn;                                      // records, while delivering
  const uint32_t stage_cap = FIN_LDS_BYTES / RB;
  const KeyFmt kf = make_keyfmt(p.key_bytes);
  const uint32_t nj = uniform32((uint32_t)min((uint64_t)w.ctl->nwg, p.cap_wg));

  // Record q of a job sits in wave q / (64E), slot (q / 64) mod E, lane
  // q mod 64: each wave holds a contiguous block, loaded 64 records at a
  // time, so counting in slot order within a wave and then over the waves
  // follows the input order.
  Rec<RW> r[E];
  // The last slice of a job stays in LDS until the next iteration has issued
  // the loads of its job's records: those loads are then in flight while the
  // slice is written out.
  __amdgpu_buffer_rsrc_t pend_dr = job_rsrc(rec0, 0);
  uint32_t pend_base = 0, pend_cnt = 0;
  // job claims alternate between two slots: a wave still reading one claim
  // is never overtaken by the next
  if (threadIdx.x == 0) S.job[0] = atomicAdd(&w.ctl->wg_head, 1u);
  __syncthreads();

  for (uint32_t it = 0;; it++) {
    uint32_t t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const uint32_t wave = t / 64, lane = t & 63;
    const uint32_t q0 = wave * (E * 64) + lane;     // record of slot 0
    const uint32_t idx = uniform32(S.job[it & 1]);
    uint64_t jbegin = 0;
    uint32_t m = 0, jflags = 0;
    if (idx < nj) {
      // every lane reads the same descriptor: keep it in scalar registers
      jbegin = uniform64(w.wgjobs[idx].begin);
      m = uniform32((uint32_t)w.wgjobs[idx].count);
      jflags = uniform32(w.wgjobs[idx].flags);
      if (m <= M) {
        const uint8_t* src = (jflags & BF_TMP) ? rec1 : rec0;
        const __amdgpu_buffer_rsrc_t sr = job_rsrc(src + jbegin * RB, m * RB);
        // offsets past the job read 0
#pragma unroll
        for (uint32_t u = 0; u < E; u++) r[u] = buf_load_rec<RW>(sr, q0 * RB, u * 64 * RB);
      }
    }
    for (uint32_t i = t; i < pend_cnt; i += FWG) buf_store_rec<RW>(pend_dr, i * RB, pend_base * RB, lds_get<RW>(stage, i));
    pend_cnt = 0;
    __syncthreads();
    if (idx >= nj) break;
    // slots u < nv hold records of the job.  The count is re-read through an
    // empty asm statement at each phase, so that the compiler recomputes the
    // per-slot conditions there instead of holding E lane masks throughout.
    uint32_t nv = m > q0 ? min(E, (m - q0 + 63) / 64) : 0u;
    uint64_t km = kf.mlo, kmh = kf.mhi;
    for (uint32_t v = t; v < NCW; v += FWG) cnt[v] = 0;
    for (uint32_t v = t; v < 256; v += FWG) S.h8[v] = 0;
    if (t == 0) S.nbig = 0;
    if (t == 0) atomicAdd(&w.ctl->stage_records[2], (unsigned long long)m);
    const __amdgpu_buffer_rsrc_t dr = job_rsrc(rec0 + jbegin * RB, m * RB);
    // the next job is claimed early: every path below passes a barrier
    // before the next iteration reads the claim
    if (t == 0) S.job[(it + 1) & 1] = atomicAdd(&w.ctl->wg_head, 1u);
    if (m > M) {  // the routing never queues such a job; refuse it loudly
      if (t == 0) atomicOr(&w.ctl->error, 4u);
      __syncthreads();
      continue;
    }

    // the bits that vary over the job
    const K ref = uniform_key(fkey_k<K, RW>(buf_load_rec<RW>(job_rsrc(((jflags & BF_TMP) ? rec1 : rec0) + jbegin * RB, RB), 0, 0), kf.mlo, kf.mhi));
    K vo = zero_key<K>();
    asm volatile("" : "+v"(nv));
    km = phase_mask(kf.mlo);
    kmh = phase_mask(kf.mhi);
#pragma unroll
    for (uint32_t u = 0; u < E; u++)
      if (u < nv) vo = vo | (fkey_k<K, RW>(r[u], km, kmh) ^ ref);
    vo = fwave_or64(vo, lane);
    if (lane == 0) S.wv[wave] = vo;
    __syncthreads();
    K vary = zero_key<K>();
#pragma unroll
    for (int q = 0; q < FWAVES; q++) vary = vary | S.wv[q];
    if (is_zero(vary)) {
      // every key equal: the job is in order already
      if (jflags & BF_TMP) {
        asm volatile("" : "+v"(nv));
        km = phase_mask(kf.mlo);
        kmh = phase_mask(kf.mhi);
#pragma unroll
        for (uint32_t u = 0; u < E; u++)
          if (u < nv) buf_store_rec<RW>(dr, q0 * RB, u * 64 * RB, r[u]);
      }
      __syncthreads();
      continue;
    }
    const uint32_t lo = lowest_bit(vary);
    const uint32_t hi = bit_length(vary);
    const uint32_t W = hi - lo;
    // The digit is the top D <= 12 varying bits.  A job grouped from
    // consecutive children holds only a few values of their parent's digit
    // in its top bits, so there the digit is the rank of the top 8 varying
    // bits among the values present, followed by as many lower bits as fit.
    const bool grouped = (jflags & BF_GROUP) && W > FIN_DIGIT_BITS;
    const uint32_t sh8 = hi >= 8 ? hi - 8 : 0;
    uint32_t xb = 0;  // lower bits after the rank (grouped jobs)
    if (grouped) {
      asm volatile("" : "+v"(nv));
      km = phase_mask(kf.mlo);
      kmh = phase_mask(kf.mhi);
#pragma unroll
      for (uint32_t u = 0; u < E; u++)
        if (u < nv) atomicAdd(&S.h8[low32(fkey_k<K, RW>(r[u], km, kmh) >> sh8) & 255u], 1u);
      __syncthreads();
      if (wave == 0) {
        uint32_t pres = 0;
#pragma unroll
        for (uint32_t k = 0; k < 4; k++) pres |= (S.h8[4 * lane + k] ? 1u : 0u) << k;
        uint32_t tot;
        uint32_t ex = fwave_excl_scan((uint32_t)__popc(pres), lane, &tot);
#pragma unroll
        for (uint32_t k = 0; k < 4; k++) {
          S.rank8[4 * lane + k] = (uint8_t)ex;
          ex += (pres >> k) & 1u;
        }
        if (lane == 0) S.ntop = tot;
      }
      __syncthreads();
      const uint32_t c = S.ntop;  // at least 2: the top varying bit takes both values
      const uint32_t cb = 32u - __clz(c - 1);
      xb = min(FIN_DIGIT_BITS - cb, W - 8);
    }
    const uint32_t D = grouped ? (32u - __clz(S.ntop - 1)) + xb : min(FIN_DIGIT_BITS, W);
    const uint32_t dsh = grouped ? sh8 - xb : hi - D;  // lowest bit of the digit's key bits
    const uint32_t rb = dsh - lo;                    // key bits below the digit
    const uint32_t ib = 32u - __clz(m - 1);          // index bits
    if (rb + ib > CB) {  // the routing never queues such a job
      if (t == 0) atomicOr(&w.ctl->error, 4u);
      __syncthreads();
      continue;
    }
    const K rmask = low_mask<K>(rb);
    const uint32_t R = 1u << D;
    const uint32_t xmask = (1u << xb) - 1u;
    auto digit_of = [&](K key) -> uint32_t {
      if (grouped) return ((uint32_t)S.rank8[low32(key >> sh8) & 255u] << xb) | (low32(key >> dsh) & xmask);
      return low32(key >> dsh) & (R - 1);
    };
    auto comp_of = [&](K key, uint32_t q) -> K { return (((key >> lo) & rmask) << ib) | q; };
    // sub-bin v occupies [end(v - 1), end(v)) once the placement is done
    auto cnt_end = [&](uint32_t v) -> uint32_t { return (cnt[v >> 1] >> (16 * (v & 1))) & 0xFFFFu; };
    auto cnt_start = [&](uint32_t v) -> uint32_t { return v ? cnt_end(v - 1) : 0u; };

    // counting pass: counts, exclusive scan, placement (16-bit counters,
    // two per word: no count exceeds M < 2^16)
    asm volatile("" : "+v"(nv));
    km = phase_mask(kf.mlo);
    kmh = phase_mask(kf.mhi);
#pragma unroll
    for (uint32_t u = 0; u < E; u++)
      if (u < nv) {
        const uint32_t v = digit_of(fkey_k<K, RW>(r[u], km, kmh));
        atomicAdd(&cnt[v >> 1], 1u << (16 * (v & 1)));
      }
    __syncthreads();
    {
      // four digits (two words) per thread (R <= 4096): scan in registers,
      // then over the waves through LDS; the largest count on the way
      const uint32_t nw = R / 2;  // R >= 2
      const uint32_t w0 = 2 * t < nw ? cnt[2 * t] : 0u;
      const uint32_t w1 = 2 * t + 1 < nw ? cnt[2 * t + 1] : 0u;
      const uint32_t a0 = w0 & 0xFFFFu, a1 = w0 >> 16, a2 = w1 & 0xFFFFu, a3 = w1 >> 16;
      uint32_t wt;
      const uint32_t ex = fwave_excl_scan(a0 + a1 + a2 + a3, lane, &wt);
      const uint32_t mx = fwave_max(max(max(a0, a1), max(a2, a3)), lane);
      if (lane == 0) { S.wsum[wave] = wt; S.wmax[wave] = mx; }
      __syncthreads();
      uint32_t base = 0;
#pragma unroll
      for (uint32_t q = 0; q < FWAVES; q++) base += q < wave ? S.wsum[q] : 0u;
      const uint32_t s0 = base + ex, s1 = s0 + a0, s2 = s1 + a1, s3 = s2 + a2;
      if (2 * t < nw) cnt[2 * t] = s0 | (s1 << 16);
      if (2 * t + 1 < nw) cnt[2 * t + 1] = s2 | (s3 << 16);
    }
    __syncthreads();
    uint32_t bigmax = 0;
#pragma unroll
    for (uint32_t q = 0; q < FWAVES; q++) bigmax = max(bigmax, S.wmax[q]);
    asm volatile("" : "+v"(nv));
    km = phase_mask(kf.mlo);
    kmh = phase_mask(kf.mhi);
#pragma unroll
    for (uint32_t u = 0; u < E; u++) {
      if (u < nv) {
        const K key = fkey_k<K, RW>(r[u], km, kmh);
        const uint32_t v = digit_of(key);
        const uint32_t sh = 16 * (v & 1);
        const uint32_t pos = (atomicAdd(&cnt[v >> 1], 1u << sh) >> sh) & 0xFFFFu;
        comp[pos] = comp_of(key, q0 + 64 * u);
      }
      fin_sched_fence();
    }
    __syncthreads();

    // Sub-bins above FSUB composites.  The usual cause is a run of equal
    // keys: if all but at most FIN_MINORS of a sub-bin's composites share one
    // key part H, those "minors" are copied to a pool and the H records are
    // ranked among themselves in input order (stable counting by sub-bin
    // below); otherwise one wavefront sorts the sub-bin in place.  Split
    // sub-bins are tagged in btag.
    // slots fit 16 bits (M <= 2^16): two per register.  An H record of a
    // split sub-bin first keeps its rank among the H records of its wave.
    uint32_t slot2[(E + 1) / 2];
#pragma unroll
    for (uint32_t h = 0; h < (E + 1) / 2; h++) slot2[h] = 0;
    if (bigmax > FSUB) {
      for (uint32_t v = t; v < R; v += FWG) {
        if (cnt_end(v) - cnt_start(v) > FSUB) {
          const uint32_t i = atomicAdd(&S.nbig, 1u);
          if (i < FIN_LDS_BIG) S.big[i] = (uint16_t)v;
        }
      }
      for (uint32_t i = t; i < (1u << FIN_DIGIT_BITS) / 4; i += FWG) reinterpret_cast<uint32_t*>(S.btag)[i] = 0;
      for (uint32_t i = t; i < FIN_SPLIT_MAX * FWAVES; i += FWG) S.cw[i] = 0;
      __syncthreads();
      // Large sub-bin i goes to wave i mod FWAVES.  The bounds are scalar
      // (the same LDS word in every lane), so the loop cannot split a wave:
      // a claim made by one lane and broadcast with readfirstlane, against a
      // bound held per lane, let the compiler send lane 0 out of the loop
      // while the other lanes read a stale claim and looped forever.
      const uint32_t nbig = uniform32(min(S.nbig, FIN_LDS_BIG));
      const uint32_t wv = uniform32(wave);
      uint32_t pool_used = 0;  // this wave's part of the pool: [wv * FIN_POOL_WAVE, +FIN_POOL_WAVE)
      for (uint32_t i = wv; i < nbig; i += FWAVES) {
        const uint32_t v = uniform32(S.big[i]);
        const uint32_t s0 = uniform32(cnt_start(v)), e = uniform32(cnt_end(v));
        uint32_t kind = 0;  // 0: sorted by the network, 1: split
        if (i < FIN_SPLIT_MAX) {
          // H: the key part shared by two of three samples, if any
          const K k0 = comp[s0] >> ib, k1 = comp[(s0 + e) / 2] >> ib, k2 = comp[e - 1] >> ib;
          const K H = (k0 == k1 || k0 == k2) ? k0 : k1;
          uint32_t nm = 0, nless = 0;
          for (uint32_t j0 = s0; j0 < e && nm <= FIN_MINORS; j0 += 64) {
            const uint32_t j = j0 + lane;
            const K x = j < e ? comp[j] : zero_key<K>();
            const bool minor = j < e && (x >> ib) != H;
            nm += (uint32_t)__popcll(__ballot(minor));
            nless += (uint32_t)__popcll(__ballot(minor && (x >> ib) < H));
          }
          if (nm <= FIN_MINORS && pool_used + nm <= POOL_WAVE) {
            const uint32_t at = wv * POOL_WAVE + pool_used;
            pool_used += nm;
            {
              uint32_t put = at;
              for (uint32_t j0 = s0; j0 < e; j0 += 64) {
                const uint32_t j = j0 + lane;
                const K x = j < e ? comp[j] : zero_key<K>();
                const bool minor = j < e && (x >> ib) != H;
                const uint64_t bal = __ballot(minor);
                if (minor) S.pool[put + (uint32_t)__popcll(bal & lanemask_lt())] = x;
                put += (uint32_t)__popcll(bal);
              }
              if (lane == 0) {
                S.bH[i] = H;
                S.binfo[i] = at | (nm << 16);
                S.bless[i] = nless;
                S.btag[v] = (uint8_t)(i + 1);
              }
              kind = 1;
            }
          }
        }
        if (!kind) wave_bitonic(comp + s0, e - s0, lane);
      }
      __syncthreads();
      // H records of split sub-bins: count them per wave in slot order
      // (peers of a round found by ballots on the sub-bin index)
      asm volatile("" : "+v"(nv));
      km = phase_mask(kf.mlo);
      kmh = phase_mask(kf.mhi);
#pragma unroll
      for (uint32_t u = 0; u < E; u++) {
        uint32_t bi = FIN_SPLIT_MAX;
        if (u < nv) {
          const K key = fkey_k<K, RW>(r[u], km, kmh);
          const uint32_t tag = S.btag[digit_of(key)];
          if (tag && ((key >> lo) & rmask) == S.bH[tag - 1]) bi = tag - 1;
        }
        const bool act = bi < FIN_SPLIT_MAX;
        const uint64_t peers = match_digit_n<7>(bi, __ballot(act));
        if (act) {
          const uint32_t leader = (uint32_t)(__ffsll((long long)peers) - 1);
          uint32_t old = 0;
          if (leader == lane) old = atomicAdd(&S.cw[wave * FIN_SPLIT_MAX + bi], (uint32_t)__popcll(peers));
          old = fshfl(old, leader);
          slot2[u / 2] |= (old + (uint32_t)__popcll(peers & lanemask_lt())) << (16 * (u & 1));
        }
        fin_sched_fence();
      }
      __syncthreads();
      // per sub-bin: H records of the earlier waves
      if (t < FIN_SPLIT_MAX) {
        uint32_t run = 0;
#pragma unroll
        for (uint32_t q = 0; q < FWAVES; q++) {
          const uint32_t x = S.cw[q * FIN_SPLIT_MAX + t];
          S.cw[q * FIN_SPLIT_MAX + t] = run;
          run += x;
        }
      }
      __syncthreads();
    }
    // every record's slot
    asm volatile("" : "+v"(nv));
    km = phase_mask(kf.mlo);
    kmh = phase_mask(kf.mhi);
#pragma unroll
    for (uint32_t u = 0; u < E; u++) {
      const uint32_t q = q0 + 64 * u;
      if (u < nv) {
        const K key = fkey_k<K, RW>(r[u], km, kmh);
        const K x = comp_of(key, q);
        const uint32_t v = digit_of(key);
        const uint32_t s0 = cnt_start(v), e = cnt_end(v);
        uint32_t pos;
        if (e - s0 <= FSUB) {
          // count the smaller composites, two at a time (16-byte reads; the
          // few words read past the sub-bin are ignored)
          uint32_t below = 0;
          for (uint32_t j = s0 & ~1u; j < e; j += 4) {
            const K y0 = comp[j], y1 = comp[j + 1], y2 = comp[j + 2], y3 = comp[j + 3];
            below += (j >= s0 && y0 < x) ? 1u : 0u;
            below += (j + 1 < e && y1 < x) ? 1u : 0u;
            below += (j + 2 < e && y2 < x) ? 1u : 0u;
            below += (j + 3 < e && y3 < x) ? 1u : 0u;
          }
          pos = s0 + below;
        } else {
          const uint32_t tag = S.btag[v];
          if (tag) {
            const uint32_t bi = tag - 1;
            const K H = S.bH[bi];
            const uint32_t info = S.binfo[bi];
            const uint32_t nm = info >> 16, at = info & 0xFFFFu;
            const K xk = (key >> lo) & rmask;
            if (xk == H) {
              pos = s0 + S.bless[bi] + S.cw[wave * FIN_SPLIT_MAX + bi] + ((slot2[u / 2] >> (16 * (u & 1))) & 0xFFFFu);
            } else {
              uint32_t below = 0;
              for (uint32_t j = 0; j < nm; j++) below += S.pool[at + j] < x ? 1u : 0u;
              pos = s0 + below + (H < xk ? (e - s0 - nm) : 0u);
            }
          } else {
            // sorted sub-bin: x is in it; lower bound
            uint32_t a = s0, z = e;
            while (a < z) {
              const uint32_t mid = (a + z) >> 1;
              if (comp[mid] < x) a = mid + 1; else z = mid;
            }
            pos = a;
          }
        }
        slot2[u / 2] = (slot2[u / 2] & (0xFFFF0000u >> (16 * (u & 1)))) | (pos << (16 * (u & 1)));
      }
      fin_sched_fence();
    }
    // out in slot order, stage_cap records per round (the stage overlays
    // the composites: every wave must be done with them); the last slice is
    // written out by the next iteration
    __syncthreads();
    const uint32_t nround = (m + stage_cap - 1) / stage_cap;
    for (uint32_t k = 0; k < nround; k++) {
      const uint32_t base = k * stage_cap;
      asm volatile("" : "+v"(nv));
      km = phase_mask(kf.mlo);
      kmh = phase_mask(kf.mhi);
#pragma unroll
      for (uint32_t u = 0; u < E; u++) {
        const uint32_t o = ((slot2[u / 2] >> (16 * (u & 1))) & 0xFFFFu) - base;
        if (u < nv && o < stage_cap) lds_put<RW>(stage, o, r[u]);
      }
      __syncthreads();
      const uint32_t cntr = min(stage_cap, m - base);
      if (k + 1 == nround) {
        pend_dr = dr;
        pend_base = base;
        pend_cnt = cntr;
      } else {
        for (uint32_t i = t; i < cntr; i += FWG) buf_store_rec<RW>(dr, i * RB, base * RB, lds_get<RW>(stage, i));
        __syncthreads();
      }
    }
  }
}

void launch_fin_jobs(const Plan& p, const Work& w, void* records, void* tmp, hipStream_t s) {
  uint8_t* r0 = (uint8_t*)records;
  uint8_t* r1 = (uint8_t*)tmp;
  const uint32_t lds = FIN_LDS_BYTES;
  const bool wide = p.key_bytes > 8;  // keys above 8 bytes need records of 12 bytes or more
  switch (p.rw) {
#define RD_CASE(n)                                                      \
  case n:                                                               \
    k_fin_jobs<n, false><<<p.grid_fin, FWG, lds, s>>>(p, w, r0, r1);    \
    break;
#define RD_CASE_W(n)                                                    \
  case n:                                                               \
    if (wide) k_fin_jobs<n, true><<<p.grid_fin, FWG, lds, s>>>(p, w, r0, r1); \
    else k_fin_jobs<n, false><<<p.grid_fin, FWG, lds, s>>>(p, w, r0, r1); \
    break;
    RD_CASE(1) RD_CASE(2) RD_CASE_W(3) RD_CASE_W(4) RD_CASE_W(5) RD_CASE_W(6) RD_CASE_W(7) RD_CASE_W(8)
    RD_CASE_W(9) RD_CASE_W(10) RD_CASE_W(11) RD_CASE_W(12) RD_CASE_W(13) RD_CASE_W(14) RD_CASE_W(15) RD_CASE_W(16)
#undef RD_CASE
#undef RD_CASE_W
    default: break;
  }
}

}  // namespace rd
