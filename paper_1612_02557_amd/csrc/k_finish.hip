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
// its key bits below the digit plus the index bits fit 64 bits (the levels
// route only such jobs here).  Jobs whose keys are all equal are written
// unchanged.
#include "raduls_dev.hpp"
#include "raduls_kernels.hpp"

namespace rd {

constexpr int FWG = 1024;              // threads of a finishing workgroup
constexpr int FWAVES = FWG / 64;
constexpr uint32_t FSUB = 32;          // larger sub-bins are sorted by a wavefront network

template <int RW>
struct FinShape {
  static constexpr uint32_t E = fin_records_per_thread(RW);
  static constexpr uint32_t M = E * FWG;
};

struct FinShared {
  uint64_t wv[FWAVES];                 // per-wave OR of key XOR reference
  uint32_t wsum[FWAVES];               // per-wave sums of the counter scan
  uint32_t wmax[FWAVES];
  uint32_t job[2];                     // claimed job index (by iteration parity)
  uint32_t nbig, bignext;              // sub-bins above FSUB and the next one to sort
  uint32_t big[FIN_LDS_BIG];           // their digits
};

// Keeps the scheduler from interleaving the unrolled per-record iterations
// (that would hold every iteration's temporaries at once and spill).
__device__ __forceinline__ void fin_sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// Buffer access to one job: a resource over the job's bytes (wave-uniform
// base), one VGPR offset per thread and the record slot u in the scalar
// offset, so that holding E records costs no address registers.
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

__device__ __forceinline__ uint32_t uniform32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  return (uint64_t)uniform32((uint32_t)x) | ((uint64_t)uniform32((uint32_t)(x >> 32)) << 32);
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
__device__ __forceinline__ void wave_bitonic(uint64_t* c, uint32_t s, uint32_t lane) {
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
          const uint64_t x = c[a], y = c[b];
          if (x > y) { c[a] = y; c[b] = x; }
        }
      }
      fin_wave_sync();
    }
  }
}

template <int RW>
__global__ __launch_bounds__(FWG) void k_fin_jobs(Plan p, Work w, uint8_t* rec0, uint8_t* rec1) {
  constexpr uint32_t E = FinShape<RW>::E;
  constexpr uint32_t M = FinShape<RW>::M;
  constexpr uint32_t RMAX = 1u << FIN_DIGIT_BITS;
  extern __shared__ __align__(16) uint32_t dyn[];
  __shared__ FinShared S;
  uint64_t* comp = reinterpret_cast<uint64_t*>(dyn);          // M composites
  uint32_t* cnt = dyn + 2 * M;                                // RMAX + 1 counters
  uint32_t* stage = dyn;                                      // records, while delivering
  const uint32_t stage_cap = FIN_LDS_BYTES / (4 * RW);
  const KeyFmt kf = make_keyfmt(p.key_bytes);
  const uint32_t nj = (uint32_t)min((uint64_t)w.ctl->nwg, p.cap_wg);

  for (uint32_t it = 0;; it++) {
    uint32_t t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const uint32_t wave = t / 64, lane = t & 63;
    // the claimed index alternates between two slots: a slow wave still
    // reading this job's slot is never overtaken by the next claim
    if (t == 0) S.job[it & 1] = atomicAdd(&w.ctl->wg_head, 1u);
    for (uint32_t v = t; v <= RMAX; v += FWG) cnt[v] = 0;
    if (t == 0) { S.nbig = 0; S.bignext = 0; }
    __syncthreads();
    const uint32_t idx = uniform32(S.job[it & 1]);
    if (idx >= nj) break;
    // every lane reads the same descriptor: keep it in scalar registers
    const uint64_t jbegin = uniform64(w.wgjobs[idx].begin);
    const uint32_t m = uniform32((uint32_t)w.wgjobs[idx].count);
    const uint32_t jflags = uniform32(w.wgjobs[idx].flags);
    const uint8_t* src = (jflags & BF_TMP) ? rec1 : rec0;
    uint8_t* dst = rec0;
    if (t == 0) atomicAdd(&w.ctl->stage_records[2], (unsigned long long)m);
    if (m > M) {  // the routing never queues such a job; refuse it loudly
      if (t == 0) atomicOr(&w.ctl->error, 4u);
      continue;
    }
    constexpr uint32_t RB = 4 * RW;  // record bytes
    const __amdgpu_buffer_rsrc_t sr = job_rsrc(src + jbegin * RB, m * RB);
    const __amdgpu_buffer_rsrc_t dr = job_rsrc(dst + jbegin * RB, m * RB);

    // records of this thread: slots u < nv.  The count is re-read through an
    // empty asm statement at each phase, so that the compiler recomputes the
    // per-slot conditions there instead of holding E lane masks throughout.
    uint32_t nv = m > t ? min(E, (m - t + FWG - 1) / FWG) : 0u;
    // 1. the job's records into registers (offsets past the job read 0)
    Rec<RW> r[E];
#pragma unroll
    for (uint32_t u = 0; u < E; u++) r[u] = buf_load_rec<RW>(sr, t * RB, u * FWG * RB);
    // 2. the bits that vary over the job
    const uint64_t ref = rec_key<RW>(buf_load_rec<RW>(sr, 0, 0), kf).lo;
    uint64_t vo = 0;
    asm volatile("" : "+v"(nv));
#pragma unroll
    for (uint32_t u = 0; u < E; u++)
      if (u < nv) vo |= rec_key<RW>(r[u], kf).lo ^ ref;
    vo = fwave_or64(vo, lane);
    if (lane == 0) S.wv[wave] = vo;
    __syncthreads();
    uint64_t vary = 0;
#pragma unroll
    for (int q = 0; q < FWAVES; q++) vary |= S.wv[q];
    if (vary == 0) {
      // every key equal: the job is in order already
      if (src != dst) {
#pragma unroll
        for (uint32_t u = 0; u < E; u++)
          if (u < nv) buf_store_rec<RW>(dr, t * RB, u * FWG * RB, r[u]);
      }
      continue;
    }
    const uint32_t lo = (uint32_t)__builtin_ctzll(vary);
    const uint32_t hi = 64u - (uint32_t)__clzll(vary);
    const uint32_t D = min(FIN_DIGIT_BITS, hi - lo);
    const uint32_t dsh = hi - D;
    const uint32_t rb = dsh - lo;                    // key bits below the digit
    const uint32_t ib = 32u - __clz(m - 1);          // index bits
    if (rb + ib > 64) {  // the routing never queues such a job
      if (t == 0) atomicOr(&w.ctl->error, 4u);
      continue;
    }
    const uint64_t rmask = rb == 0 ? 0ull : (rb >= 64 ? ~0ull : ((1ull << rb) - 1));
    const uint32_t R = 1u << D;
    auto digit_of = [&](uint64_t key) -> uint32_t { return (uint32_t)(key >> dsh) & (R - 1); };
    auto comp_of = [&](uint64_t key, uint32_t q) -> uint64_t { return (((key >> lo) & rmask) << ib) | q; };

    // 3. counting pass: counts, exclusive scan, placement
    asm volatile("" : "+v"(nv));
#pragma unroll
    for (uint32_t u = 0; u < E; u++)
      if (u < nv) atomicAdd(&cnt[digit_of(rec_key<RW>(r[u], kf).lo)], 1u);
    __syncthreads();
    {
      // two digits per thread (R <= 2048): scan in registers, then over the
      // waves through LDS; the largest count is found on the way
      const uint32_t v0 = 2 * t;
      const uint32_t a = v0 < R ? cnt[v0] : 0u, c = v0 + 1 < R ? cnt[v0 + 1] : 0u;
      uint32_t wt;
      const uint32_t ex = fwave_excl_scan(a + c, lane, &wt);
      const uint32_t mx = fwave_max(max(a, c), lane);
      if (lane == 0) { S.wsum[wave] = wt; S.wmax[wave] = mx; }
      __syncthreads();
      uint32_t base = 0;
#pragma unroll
      for (uint32_t q = 0; q < FWAVES; q++) base += q < wave ? S.wsum[q] : 0u;
      if (v0 < R) cnt[v0] = base + ex;
      if (v0 + 1 < R) cnt[v0 + 1] = base + ex + a;
    }
    __syncthreads();
    uint32_t bigmax = 0;
#pragma unroll
    for (uint32_t q = 0; q < FWAVES; q++) bigmax = max(bigmax, S.wmax[q]);
    asm volatile("" : "+v"(nv));
#pragma unroll
    for (uint32_t u = 0; u < E; u++) {
      const uint32_t q = u * FWG + t;
      if (u < nv) {
        const uint64_t key = rec_key<RW>(r[u], kf).lo;
        comp[atomicAdd(&cnt[digit_of(key)], 1u)] = comp_of(key, q);
      }
      fin_sched_fence();
    }
    __syncthreads();
    // cnt[v] is now the end of sub-bin v (and the start of v + 1)

    // 4a. sub-bins above FSUB: sorted in place, one wavefront each
    if (bigmax > FSUB) {
      for (uint32_t v = t; v < R; v += FWG) {
        const uint32_t s0 = v ? cnt[v - 1] : 0u;
        if (cnt[v] - s0 > FSUB) {
          const uint32_t i = atomicAdd(&S.nbig, 1u);
          if (i < FIN_LDS_BIG) S.big[i] = v;
        }
      }
      __syncthreads();
      const uint32_t nbig = min(S.nbig, FIN_LDS_BIG);
      for (;;) {
        uint32_t i = 0;
        if (lane == 0) i = atomicAdd(&S.bignext, 1u);
        i = uniform32(i);
        if (i >= nbig) break;
        const uint32_t v = S.big[i];
        const uint32_t s0 = v ? cnt[v - 1] : 0u;
        wave_bitonic(comp + s0, cnt[v] - s0, lane);
      }
      __syncthreads();
    }
    // 4b. every record's slot
    // slots fit 16 bits (M <= 2^16): two per register
    uint32_t slot2[(E + 1) / 2];
#pragma unroll
    for (uint32_t h = 0; h < (E + 1) / 2; h++) slot2[h] = 0;
    asm volatile("" : "+v"(nv));
#pragma unroll
    for (uint32_t u = 0; u < E; u++) {
      const uint32_t q = u * FWG + t;
      if (u < nv) {
        const uint64_t key = rec_key<RW>(r[u], kf).lo;
        const uint64_t x = comp_of(key, q);
        const uint32_t v = digit_of(key);
        const uint32_t s0 = v ? cnt[v - 1] : 0u, e = cnt[v];
        uint32_t pos;
        if (e - s0 > FSUB) {
          // sorted sub-bin: x is in it; lower bound
          uint32_t a = s0, z = e;
          while (a < z) {
            const uint32_t mid = (a + z) >> 1;
            if (comp[mid] < x) a = mid + 1; else z = mid;
          }
          pos = a;
        } else {
          uint32_t below = 0;
          for (uint32_t i = s0; i < e; i++) below += comp[i] < x ? 1u : 0u;
          pos = s0 + below;
        }
        slot2[u / 2] |= pos << (16 * (u & 1));
      }
      fin_sched_fence();
    }
    __syncthreads();
    // 5. out in slot order, stage_cap records per round
    for (uint32_t base = 0; base < m; base += stage_cap) {
      asm volatile("" : "+v"(nv));
#pragma unroll
      for (uint32_t u = 0; u < E; u++) {
        const uint32_t o = ((slot2[u / 2] >> (16 * (u & 1))) & 0xFFFFu) - base;
        if (u < nv && o < stage_cap) lds_put<RW>(stage, o, r[u]);
      }
      __syncthreads();
      const uint32_t cntr = min(stage_cap, m - base);
      for (uint32_t i = t; i < cntr; i += FWG) buf_store_rec<RW>(dr, i * RB, base * RB, lds_get<RW>(stage, i));
      __syncthreads();
    }
  }
}

void launch_fin_jobs(const Plan& p, const Work& w, void* records, void* tmp, hipStream_t s) {
  uint8_t* r0 = (uint8_t*)records;
  uint8_t* r1 = (uint8_t*)tmp;
  const uint32_t lds = FIN_LDS_BYTES;
  switch (p.rw) {
#define RD_CASE(n)                                                      \
  case n:                                                               \
    k_fin_jobs<n><<<p.grid_fin, FWG, lds, s>>>(p, w, r0, r1);           \
    break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

}  // namespace rd
