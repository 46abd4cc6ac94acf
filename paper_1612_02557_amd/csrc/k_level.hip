// k_level.hip -- multi-workgroup levels of the MSD radix sort.
//
// One level splits every bucket of a list by its next digit (paper, Sec. 1:
// a counting pass is a histogram traversal, the offsets of smaller digits,
// and a distribution traversal; Sec. 3.2-3.3: the first pass and the passes
// on big bins use all threads).  On the GPU a level is:
//   k_prefix   tile ranges of the list's buckets
//   k_hist     per-bucket digit histogram (per-wave LDS counters) and the OR of
//              key XOR a reference key (which bits vary in the bucket)
//   k_scan     per bucket: digit offsets, child buckets classified into the
//              next list, the single-workgroup queue, the tiny queue or done
//   k_scatter  stable tile ranking, decoupled look-back over tiles of the
//              bucket, LDS staging by digit, coalesced writes
#include "raduls_dev.hpp"
#include "raduls_kernels.hpp"

namespace rd {


__device__ __forceinline__ Bucket* level_list(const Plan& p, const Work& w, uint32_t level) {
  return w.big + (uint64_t)level * p.cap_big;
}
__device__ __forceinline__ uint64_t* level_start(const Plan& p, const Work& w, uint32_t level) {
  return w.tile_start + (uint64_t)level * (p.cap_big + 1);
}

// ---------------------------------------------------------------------------
// Control-block reset and the look-back epoch of this sort.
__global__ void k_init(Work w) {
  uint32_t* epoch_counter = w.epoch_counter;
  uint32_t* c = reinterpret_cast<uint32_t*>(w.ctl);
  for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) c[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t e = *epoch_counter + (LMAX + 1);
    *epoch_counter = e;
    w.ctl->epoch = e;
  }
}

// ---------------------------------------------------------------------------
// Appending buckets to the queues.  Classification of a bucket that still
// needs work (Sec. 3.2: big bins above 2N/3T; Sec. 3.5: the smallest bins).
__device__ __forceinline__ void push_big(const Plan& p, const Work& w, uint32_t level, const Bucket& b) {
  uint32_t i = atomicAdd(&w.ctl->nbig[level], 1u);
  if (i < p.cap_big) level_list(p, w, level)[i] = b;
  else atomicOr(&w.ctl->overflow, 1u);
}
__device__ __forceinline__ void push_small(const Plan& p, const Work& w, const Bucket& b) {
  uint32_t i = atomicAdd(&w.ctl->nsmall, 1u);
  if (i < p.cap_small) w.small[i] = b;
  else atomicOr(&w.ctl->overflow, 2u);
}
__device__ __forceinline__ void push_tiny(const Plan& p, const Work& w, uint64_t packed) {
  uint32_t i = atomicAdd(&w.ctl->ntiny, 1u);
  if (i < p.cap_tiny) w.tiny[i] = packed;
  else atomicOr(&w.ctl->overflow, 4u);
}
__device__ __forceinline__ void push_job(const Plan& p, const Work& w, const Bucket& b) {
  uint32_t i = atomicAdd(&w.ctl->nwg, 1u);
  if (i < p.cap_wg) w.wgjobs[i] = b;
  else atomicOr(&w.ctl->overflow, 32u);
}
__device__ __forceinline__ void push_copy(const Plan& p, const Work& w, const Bucket& b) {
  uint32_t i = atomicAdd(&w.ctl->ncopy, 1u);
  if (i < p.cap_copy) w.copy[i] = b;
  else atomicOr(&w.ctl->overflow, 8u);
}

// Route a bucket (records [begin, begin+count) at resolved bit `bit`, in tmp
// if `in_tmp`) to where it is finished.  `level` is the next list.
__device__ void route_bucket(const Plan& p, const Work& w, uint32_t next_level, Bucket b, uint32_t kbits) {
  bool in_tmp = b.flags & BF_TMP;
  bool done = b.count <= 1 || b.bit >= kbits;
  if (done) {
    if (!in_tmp || b.count == 0) return;
    if (b.count <= 63) push_tiny(p, w, pack_tiny(b.begin, (uint32_t)b.count, 1u, kbits));
    else push_copy(p, w, b);
    return;
  }
  if (p.fin_max) {
    // register finishing: every bucket that qualifies as a job is one;
    // the others take another level while levels are left
    if (b.count <= TINY_MAX) {
      push_tiny(p, w, pack_tiny(b.begin, (uint32_t)b.count, in_tmp ? 1u : 0u, b.bit));
    } else if (job_ok(p, b.count, b.bit, kbits)) {
      b.flags |= BF_ROOT;
      push_job(p, w, b);
    } else if (next_level < p.lmax) {
      push_big(p, w, next_level, b);
    } else {
      push_small(p, w, b);
    }
    return;
  }
  if (b.count > p.t_big && next_level < p.lmax) {
    push_big(p, w, next_level, b);
  } else if (b.count <= TINY_MAX) {
    push_tiny(p, w, pack_tiny(b.begin, (uint32_t)b.count, in_tmp ? 1u : 0u, b.bit));
  } else {
    push_small(p, w, b);
  }
}

// The whole array as one bucket.
__global__ void k_seed_single(Plan p, Work w) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (p.partition) {
    Bucket b{0, p.n, p.n, p.partition_bit, 0u};
    push_big(p, w, 0, b);
    return;
  }
  Bucket b{0, p.n, p.n, 0u, 0u};
  route_bucket(p, w, 0, b, 8 * p.key_bytes);
}

// Segment offsets must start at 0, never decrease and end at the total.
__global__ void k_check_segments(Plan p, Work w, const uint64_t* off, uint32_t S) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i == 0 && (off[0] != 0 || off[S] != p.n)) atomicOr(&w.ctl->error, 1u);
  if (i < S && off[i + 1] < off[i]) atomicOr(&w.ctl->error, 1u);
}

// Every segment is a bucket of its own (a batch of independent arrays).
__global__ void k_seed_segments(Plan p, Work w, const uint64_t* off, uint32_t S) {
  if (w.ctl->error) return;
  uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (s >= S) return;
  uint64_t a = off[s], c = off[s + 1] - a;
  Bucket b{a, c, c, 0u, 0u};
  route_bucket(p, w, 0, b, 8 * p.key_bytes);
}

// ---------------------------------------------------------------------------
// Tile ranges of a list: start[i] = sum of ceil(count/tile) over entries < i.
// One workgroup; also resets the list's tile ticket.
__global__ void k_prefix(const Bucket* list, const uint32_t* nlist, uint64_t cap, uint64_t* start,
                         uint64_t* total, uint32_t* ticket, uint32_t tile) {
  __shared__ uint64_t part[WG];
  uint32_t nb = min((uint64_t)*nlist, cap);
  uint32_t t = threadIdx.x;
  uint32_t per = (nb + WG - 1) / WG;
  uint32_t lo = min(nb, t * per), hi = min(nb, lo + per);
  uint64_t s = 0;
  for (uint32_t i = lo; i < hi; i++) s += (list[i].count + tile - 1) / tile;
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    uint64_t run = 0;
    for (int i = 0; i < WG; i++) { uint64_t c = part[i]; part[i] = run; run += c; }
    *total = run;
    start[nb] = run;
    if (ticket) *ticket = 0;
  }
  __syncthreads();
  uint64_t run = part[t];
  for (uint32_t i = lo; i < hi; i++) { start[i] = run; run += (list[i].count + tile - 1) / tile; }
}

// Zero the histogram and varying-bit words of a level's buckets.
__global__ void k_clear_hist(Plan p, Work w, uint32_t level) {
  uint32_t nb = min((uint64_t)w.ctl->nbig[level], p.cap_big);
  uint64_t R = 1ull << p.d_big;
  uint64_t total = (uint64_t)nb * R;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x)
    w.hist[i] = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < 2ull * nb;
       i += (uint64_t)gridDim.x * blockDim.x)
    w.vary[i] = 0;
}

// Zero `words` 64-bit words (a fill kernel, so that the clearing can sit in
// a captured stream without a memset node).
__global__ void k_zero_words(uint64_t* p, uint64_t words) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

template <int RW, int DB>
__global__ __launch_bounds__(WG) void k_hist(Plan p, Work w, uint32_t level, const uint8_t* rec0,
                                             const uint8_t* rec1) {
  constexpr uint32_t RMAX = 1u << DB;
  constexpr uint32_t HB = 16;  // keys loaded per thread before they are counted
  constexpr uint32_t HW = RMAX <= 256 ? NWAVES : 1;  // per-wave counters when they are small
  // two sets of counters: a tile counts into one while the other, holding
  // the previous tile's counts, is read out and cleared
  __shared__ uint32_t sh[2 * HW * RMAX];
  __shared__ uint64_t sv[2 * NWAVES];
  const Bucket* list = level_list(p, w, level);
  const uint64_t* start = level_start(p, w, level);
  uint32_t nb = min((uint64_t)w.ctl->nbig[level], p.cap_big);
  uint64_t T = w.ctl->ntiles[level];
  if (nb == 0 || T == 0) return;
  uint64_t per = (T + gridDim.x - 1) / gridDim.x;
  uint64_t t = blockIdx.x * per;
  uint64_t t1 = min(T, t + per);
  const KeyFmt kf = make_keyfmt(p.key_bytes);
  const uint32_t lane = lane_id();
  const uint32_t RS = 1u << p.d_big;
  const uint32_t IPT = p.tile / WG;
  while (t < t1) {
    uint32_t b = find_entry(start, nb, t);
    Bucket B = list[b];
    uint64_t bt0 = start[b];
    uint64_t tend = min(t1, start[b + 1]);
    uint32_t d = min(p.d_big, kf.kbits - B.bit);
    uint32_t shift = kf.kbits - B.bit - d;
    uint32_t mask = (1u << d) - 1u;
    const uint8_t* src = (B.flags & BF_TMP) ? rec1 : rec0;
    Key ref = load_key<RW>(src, B.begin, kf);
    for (uint32_t i = threadIdx.x; i < 2 * HW * RMAX; i += WG) sh[i] = 0;
    __syncthreads();
    uint32_t par = 0;
    uint64_t vlo = 0, vhi = 0;
    uint64_t bend = B.begin + B.count;
    constexpr uint32_t KV = (RMAX + WG - 1) / WG;  // digits per thread
    uint32_t acc[KV];
#pragma unroll
    for (uint32_t k = 0; k < KV; k++) acc[k] = 0;
    for (; t < tend; t++, par ^= 1u) {
      uint32_t* cur = sh + par * HW * RMAX;
      uint32_t* shw = cur + (HW > 1 ? (threadIdx.x / 64) * RMAX : 0);
      uint64_t r0 = B.begin + (t - bt0) * p.tile;
      for (uint32_t j0 = 0; j0 < IPT; j0 += HB) {
        Key kk[HB];
#pragma unroll
        for (uint32_t u = 0; u < HB; u++) {
          uint64_t i = r0 + (uint64_t)(j0 + u) * WG + threadIdx.x;
          kk[u] = (j0 + u < IPT && i < bend) ? load_key<RW>(src, i, kf) : ref;
        }
#pragma unroll
        for (uint32_t u = 0; u < HB; u++) {
          uint64_t i = r0 + (uint64_t)(j0 + u) * WG + threadIdx.x;
          bool valid = j0 + u < IPT && i < bend;
          vlo |= kk[u].lo ^ ref.lo;
          vhi |= kk[u].hi ^ ref.hi;
          uint32_t v = key_digit(kk[u], shift, mask, kf);
          // one LDS add per key, or one per wave when all 64 keys share the
          // digit (runs of equal keys)
          const uint64_t active = __ballot(valid);
          const uint32_t v0 = __shfl(v, 0);
          if (active == ~0ull && __ballot(v == v0) == ~0ull) {
            if (lane == 0) atomicAdd(&shw[v0], 64u);
          } else if (valid) {
            atomicAdd(&shw[v], 1u);
          }
        }
      }
      // the tile's counts go to the tile-count array (read by the offset
      // scan) and into this run's totals, and its counters are cleared
      // while the next tile counts into the other set
      __syncthreads();
      uint32_t* tc = w.tcnt + t * RS;
#pragma unroll
      for (uint32_t k = 0; k < KV; k++) {
        const uint32_t i = threadIdx.x + k * WG;
        if (i < (1u << d)) {
          uint32_t c = 0;
#pragma unroll
          for (uint32_t q = 0; q < HW; q++) { c += cur[q * RMAX + i]; cur[q * RMAX + i] = 0; }
          tc[i] = c;
          acc[k] += c;
        }
      }
    }
    vlo = wave_or64(vlo);
    vhi = wave_or64(vhi);
    if (lane == 0) { sv[2 * (threadIdx.x / 64)] = vlo; sv[2 * (threadIdx.x / 64) + 1] = vhi; }
    __syncthreads();
    uint64_t* gh = w.hist + (uint64_t)b * RS;
#pragma unroll
    for (uint32_t k = 0; k < KV; k++) {
      const uint32_t i = threadIdx.x + k * WG;
      if (i < (1u << d) && acc[k]) atomicAdd((unsigned long long*)&gh[i], (unsigned long long)acc[k]);
    }
    if (threadIdx.x == 0) {
      uint64_t a = 0, c = 0;
      for (int q = 0; q < NWAVES; q++) { a |= sv[2 * q]; c |= sv[2 * q + 1]; }
      if (a) atomicOr((unsigned long long*)&w.vary[2 * b], (unsigned long long)a);
      if (c) atomicOr((unsigned long long*)&w.vary[2 * b + 1], (unsigned long long)c);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Per-bucket scan and classification.  One workgroup per list entry.
// Per-level histogram for digits of at most 8 bits, one wavefront per
// tile: wave q of a workgroup takes tiles ta + q, ta + q + NWAVES, ... of the
// workgroup's range, counts a tile's digits in its own LDS counters, writes
// them out as the tile's counts and adds them to per-lane totals, which go to
// the bucket's histogram (and the key-bit OR to its varying mask) when the
// wave moves on to another bucket.  No workgroup barrier, so a wave's loads
// keep streaming from one tile into the next: each wave has two sets of
// counters, and a tile's counts are read out only once the first keys of
// the wave's next tile have been requested (into the other set), so the
// read-out overlaps those loads.
template <int RW, bool WIDE>
__global__ __launch_bounds__(WG) void k_hist_wave(Plan p, Work w, uint32_t level, const uint8_t* rec0,
                                                  const uint8_t* rec1) {
  constexpr uint32_t RMAX = 256;
  constexpr uint32_t HB = 8;           // keys loaded per lane before they are counted
  constexpr uint32_t DL = RMAX / 64;   // digits per lane
  constexpr uint32_t RB = RW * 4;      // record bytes
  __shared__ uint32_t sh[2 * NWAVES * RMAX];
  const Bucket* list = level_list(p, w, level);
  const uint64_t* start = level_start(p, w, level);
  const uint32_t nb = min((uint64_t)w.ctl->nbig[level], p.cap_big);
  const uint64_t T = w.ctl->ntiles[level];
  if (nb == 0 || T == 0) return;
  const uint64_t per = (T + gridDim.x - 1) / gridDim.x;
  const uint64_t ta = blockIdx.x * per, tz = min(T, ta + per);
  const KeyFmt kf = make_keyfmt(p.key_bytes);
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / 64;
  const uint32_t RS = 1u << p.d_big;
  const uint32_t IPW = p.tile / 64;    // records per lane of a tile
  uint32_t* const cset0 = sh + wave * 2 * RMAX;
  for (uint32_t v = threadIdx.x; v < 2 * NWAVES * RMAX; v += WG) sh[v] = 0;
  __syncthreads();
  constexpr uint32_t NONE = 0xFFFFFFFFu;
  uint32_t b = NONE, d = 0, shift = 0, mask = 0;
  uint64_t bt0 = 0, bnext = 0, bbegin = 0, bend = 0;
  const uint8_t* src = rec0;
  Key ref{0, 0};
  uint64_t vlo = 0, vhi = 0;
  uint32_t acc[DL];
#pragma unroll
  for (uint32_t k = 0; k < DL; k++) acc[k] = 0;
  auto flush = [&]() {
    uint64_t* gh = w.hist + (uint64_t)b * RS;
#pragma unroll
    for (uint32_t k = 0; k < DL; k++) {
      const uint32_t v = lane + 64 * k;
      if (v < (1u << d) && acc[k]) atomicAdd((unsigned long long*)&gh[v], (unsigned long long)acc[k]);
    }
    const uint64_t a = wave_or64(vlo), c = wave_or64(vhi);
    if (lane == 0) {
      if (a) atomicOr((unsigned long long*)&w.vary[2 * b], (unsigned long long)a);
      if (c) atomicOr((unsigned long long*)&w.vary[2 * b + 1], (unsigned long long)c);
    }
  };
  // read out (and clear) the counters of tile tt, digit width dd
  auto readout = [&](uint32_t* cw, uint64_t tt, uint32_t dd) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint32_t* tc = w.tcnt + tt * RS;
#pragma unroll
    for (uint32_t k = 0; k < DL; k++) {
      const uint32_t v = lane + 64 * k;
      if (v < (1u << dd)) {
        const uint32_t c = cw[v];
        cw[v] = 0;
        tc[v] = c;
        acc[k] += c;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };
  uint32_t cur = 0;            // counter set of the current tile
  bool pending = false;        // the previous tile's counts are still in the other set
  uint64_t tprev = 0;
  uint32_t dprev = 0;
  for (uint64_t t = ta + wave; t < tz; t += NWAVES) {
    // the tile's bucket (the wave's tiles are increasing, so it only moves on)
    const bool nextb = b == NONE || t >= bnext;
    uint32_t nbk = b;
    if (nextb) {
      if (b == NONE) nbk = find_entry(start, nb, t);
      else while (start[nbk + 1] <= t) nbk++;
    }
    const Bucket B = list[nbk];
    const uint64_t nbt0 = start[nbk];
    const uint64_t nbegin = B.begin, nend = B.begin + B.count;
    const uint32_t nd = min(p.d_big, kf.kbits - B.bit);
    const uint32_t nshift = kf.kbits - B.bit - nd;
    const uint8_t* nsrc = (B.flags & BF_TMP) ? rec1 : rec0;
    const uint64_t r0 = nbegin + (t - nbt0) * p.tile;
    // the tile's records through a buffer resource: one offset register per
    // lane, and records past the tile's end read as 0 (they are not counted)
    const uint32_t cnt = (uint32_t)min((uint64_t)p.tile, nend - r0);
    const __amdgpu_buffer_rsrc_t rs = job_rsrc(nsrc + r0 * RB, cnt * RB);
    const uint32_t voff = lane * RB;
    // the first keys of this tile are requested before the previous tile's
    // counts are read out
    Key kk[HB];
    Key nref = ref;
    if (nextb) nref = load_key<RW>(nsrc, nbegin, kf);
#pragma unroll
    for (uint32_t u = 0; u < HB; u++) kk[u] = buf_load_key<RW, WIDE>(rs, voff, u * 64 * RB, kf);
    if (pending) readout(cset0 + (cur ^ 1u) * RMAX, tprev, dprev);
    if (nextb) {
      if (b != NONE) flush();
      b = nbk;
      bt0 = nbt0;
      bnext = start[b + 1];
      bbegin = nbegin;
      bend = nend;
      d = nd;
      shift = nshift;
      mask = (1u << d) - 1u;
      src = nsrc;
      ref = nref;
      vlo = vhi = 0;
#pragma unroll
      for (uint32_t k = 0; k < DL; k++) acc[k] = 0;
    }
    uint32_t* cw = cset0 + cur * RMAX;
    for (uint32_t j0 = 0; j0 < IPW; j0 += HB) {
      if (j0 > 0) {
#pragma unroll
        for (uint32_t u = 0; u < HB; u++) kk[u] = buf_load_key<RW, WIDE>(rs, voff, (j0 + u) * 64 * RB, kf);
      }
#pragma unroll
      for (uint32_t u = 0; u < HB; u++) {
        const bool valid = j0 + u < IPW && (j0 + u) * 64 + lane < cnt;
        if (!valid) kk[u] = ref;
        vlo |= kk[u].lo ^ ref.lo;
        vhi |= kk[u].hi ^ ref.hi;
        const uint32_t v = key_digit(kk[u], shift, mask, kf);
        const uint64_t active = __ballot(valid);
        const uint32_t v0 = __shfl(v, 0);
        if (active == ~0ull && __ballot(v == v0) == ~0ull) {
          if (lane == 0) atomicAdd(&cw[v0], 64u);
        } else if (valid) {
          atomicAdd(&cw[v], 1u);
        }
      }
    }
    pending = true;
    tprev = t;
    dprev = d;
    cur ^= 1u;
  }
  if (pending) readout(cset0 + (cur ^ 1u) * RMAX, tprev, dprev);
  if (b != NONE) flush();
}

template <int DB>
__global__ __launch_bounds__(WG) void k_scan(Plan p, Work w, uint32_t level) {
  constexpr uint32_t RMAX = 1u << DB;
  __shared__ uint64_t off[RMAX];
  __shared__ uint64_t part[WG];
  // grouping of small children into finishing jobs (digits <= WG)
  __shared__ uint32_t flag[WG];
  __shared__ uint32_t stmp[NWAVES], smax[NWAVES];
  __shared__ uint64_t cst[WG], ccn[WG], gst[WG], gfc[WG];
  __shared__ uint64_t gend;
  Bucket* list = level_list(p, w, level);
  uint32_t nb = min((uint64_t)w.ctl->nbig[level], p.cap_big);
  const KeyFmt kf = make_keyfmt(p.key_bytes);
  const uint32_t RS = 1u << p.d_big;
  for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
    Bucket B = list[b];
    Key vary = Key{w.vary[2 * b], w.vary[2 * b + 1]};
    uint32_t d = min(p.d_big, kf.kbits - B.bit);
    if (p.partition) {
      // one stable pass for the caller: always move, report the counts
      uint64_t* gh = w.hist + (uint64_t)b * RS;
      uint32_t R = 1u << d;
      if (w.counts_out)
        for (uint32_t i = threadIdx.x; i < R; i += WG) w.counts_out[i] = gh[i];
      __syncthreads();
      if (threadIdx.x == 0) {
        uint64_t run = 0;
        for (uint32_t i = 0; i < R; i++) { uint64_t c = gh[i]; gh[i] = run; run += c; }
      }
      __syncthreads();
      continue;
    }
    if (vary.lo == 0 && vary.hi == 0) {
      // every key equal: the bucket is finished where it lies
      if (threadIdx.x == 0) {
        list[b].flags = B.flags | BF_SKIP;
        Bucket c = B;
        c.bit = kf.kbits;
        route_bucket(p, w, level + 1, c, kf.kbits);
      }
      __syncthreads();
      continue;
    }
    uint32_t lead = common_prefix_bits(vary, kf.kbits);
    if (lead >= B.bit + d) {
      // the digit is the same for all keys: skip the move, resolve the
      // shared bits and split on the first differing digit next level
      if (threadIdx.x == 0) {
        list[b].flags = B.flags | BF_SKIP;
        Bucket c = B;
        c.bit = lead;
        route_bucket(p, w, level + 1, c, kf.kbits);
      }
      __syncthreads();
      continue;
    }
    uint64_t* gh = w.hist + (uint64_t)b * RS;
    uint32_t R = 1u << d;
    uint32_t per = (R + WG - 1) / WG;
    uint32_t lo = min(R, threadIdx.x * per), hi = min(R, lo + per);
    uint64_t s = 0;
    for (uint32_t i = lo; i < hi; i++) { off[i] = gh[i]; s += off[i]; }
    // exclusive scan of the threads' sums: within each wavefront by
    // shuffles, then across the wavefronts through LDS
    uint64_t run = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t y = __shfl_up((unsigned long long)run, o);
      if ((int)lane_id() >= o) run += y;
    }
    if (lane_id() == 63) part[threadIdx.x / 64] = run;
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < NWAVES; q++) run += q < threadIdx.x / 64 ? part[q] : 0ull;
    run -= s;
    if (R <= WG) {
      // Thread t owns digit t.  Children lie consecutively in key order, so
      // a run of whole children is a valid finishing job.  A child above T
      // (half the job size J) is routed on its own; smaller ones are grouped
      // by the window of V = J - (largest of them) records their first
      // record falls in, so a group holds under V + largest <= J records.
      const uint32_t t = threadIdx.x;
      // a group keeps the parent's resolved bits: its size is bounded by
      // what a job with those bits may hold
      const uint64_t T = min((uint64_t)p.job_window, max<uint64_t>(job_cap(p, B.bit, kf.kbits) / 2, 32));
      const uint64_t cnt = t < R ? off[t] : 0ull;
      if (t < R) gh[t] = run;  // digit base, read by the scatter
      flag[t] = cnt > 0 ? 1u : 0u;
      const uint32_t nn = block_excl_scan_lds(flag, WG, stmp);
      if (cnt > 0) { cst[flag[t]] = run; ccn[flag[t]] = cnt; }
      uint32_t mx = cnt <= T ? (uint32_t)cnt : 0u;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o));
      if (lane_id() == 0) smax[t / 64] = mx;
      __syncthreads();
#pragma unroll
      for (uint32_t q = 0; q < NWAVES; q++) mx = max(mx, smax[q]);
      const uint64_t V = 2 * T - max<uint64_t>(mx, 1);
      uint32_t kb = 0;
      uint64_t kst = 0, kcnt = 0;
      if (t < nn) {
        kst = cst[t];
        kcnt = ccn[t];
        kb = 1;
        if (t > 0) {
          const uint64_t pst = cst[t - 1], pcnt = ccn[t - 1];
          kb = (kcnt > T || pcnt > T || kst / V != pst / V) ? 1u : 0u;
        }
      }
      flag[t] = kb;
      const uint32_t nj = block_excl_scan_lds(flag, WG, stmp);
      if (kb) { gst[flag[t]] = kst; gfc[flag[t]] = kcnt; }
      if (t < nn && t + 1 == nn) gend = kst + kcnt;
      __syncthreads();
      // a job that a workgroup finishes in LDS goes straight to the job
      // list (one ticket per bucket); the others are routed one by one
      Bucket ch{0, 0, 0, 0, 0};
      bool direct = false;
      if (t < nj) {
        const uint64_t js = gst[t], m = (t + 1 < nj ? gst[t + 1] : gend) - js;
        ch.begin = B.begin + js;
        ch.count = m;
        ch.parent = B.count;
        ch.bit = m == gfc[t] ? B.bit + d : B.bit;
        ch.flags = (p.inplace ? 0u : ((B.flags & BF_TMP) ^ BF_TMP)) | (m == gfc[t] ? 0u : BF_GROUP);
        direct = job_ok(p, m, ch.bit, kf.kbits);
        if (!direct) route_bucket(p, w, level + 1, ch, kf.kbits);
      }
      flag[t] = direct ? 1u : 0u;
      const uint32_t nd = block_excl_scan_lds(flag, WG, stmp);
      if (nd) {
        if (t == 0) gend = atomicAdd(&w.ctl->nwg, nd);
        __syncthreads();
        if (direct) {
          const uint64_t i = gend + flag[t];
          ch.flags |= BF_ROOT;
          if (i < p.cap_wg) w.wgjobs[i] = ch;
          else atomicOr(&w.ctl->overflow, 32u);
        }
      }
      __syncthreads();
      continue;
    }
    for (uint32_t i = lo; i < hi; i++) {
      uint64_t c = off[i];
      gh[i] = run;  // digit base, read by the scatter
      if (c) {
        Bucket ch;
        ch.begin = B.begin + run;
        ch.count = c;
        ch.parent = B.count;
        ch.bit = B.bit + d;
        ch.flags = p.inplace ? 0u : ((B.flags & BF_TMP) ^ BF_TMP);
        route_bucket(p, w, level + 1, ch, kf.kbits);
      }
      run += c;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Tile digit offsets of one level: for tile t of bucket b and digit v,
//   off[t][v] = base[b][v] + (records of digit v in the earlier tiles of b),
// where base is the digit's start within the bucket (from the scan kernel).
// The level's tiles are cut into chunks of TSCAN_CH consecutive tiles, which
// may hold the end of one bucket and the start of others.  A chunk sums, per
// digit, its tiles of its last bucket and publishes that sum: inclusive when
// that bucket starts inside the chunk, an aggregate otherwise; a chunk whose
// first bucket started earlier adds up the words of the chunks before it
// (decoupled look-back over chunks, tickets taken in order).  Then the
// scatter reads its tile's offsets instead of waiting on other tiles.
template <int DB>
__global__ __launch_bounds__(WG) void k_tile_scan(Plan p, Work w, uint32_t level) {
  constexpr uint32_t RMAX = 1u << DB;
  constexpr uint32_t KV = (RMAX + WG - 1) / WG;  // digits per thread
  constexpr uint32_t CH = TSCAN_CH;
  static_assert(CH <= WG, "one thread per tile of a chunk");
  __shared__ uint64_t sticket;
  __shared__ uint32_t sb;
  __shared__ uint64_t sst[CH];   // starts of the buckets after the first one (chunk order)
  const Bucket* list = level_list(p, w, level);
  const uint64_t* start = level_start(p, w, level);
  const uint32_t nb = min((uint64_t)w.ctl->nbig[level], p.cap_big);
  const uint64_t T = w.ctl->ntiles[level];
  if (nb == 0 || T == 0) return;
  const uint64_t NC = (T + CH - 1) / CH;
  const uint32_t RS = 1u << p.d_big;
  const KeyFmt kf = make_keyfmt(p.key_bytes);
  const uint64_t epoch = (uint64_t)((w.ctl->epoch + level) & 0x3FFFFFu) << LB_EPOCH_SHIFT;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint64_t c = atomicAdd(&w.ctl->cticket[level], 1u);
      sticket = c;
      sb = c < NC ? find_entry(start, nb, c * CH) : 0u;
    }
    __syncthreads();
    const uint64_t c = sticket;
    const uint32_t b0 = sb;
    if (c >= NC) break;
    const uint64_t t0 = c * CH, t1 = min(T, t0 + CH);
    if (threadIdx.x < CH) {
      const uint32_t bj = b0 + 1 + threadIdx.x;
      sst[threadIdx.x] = bj < nb ? start[bj] : ~0ull;
    }
    __syncthreads();
    // buckets b0 .. bl hold the chunk's tiles; bucket b0 + 1 + j starts at sst[j]
    uint32_t nin = 0;
#pragma unroll
    for (uint32_t j = 0; j < CH; j++) nin += sst[j] < t1 ? 1u : 0u;
    const uint32_t bl = b0 + nin;
    const bool cont = start[b0] < t0;          // the first bucket started before this chunk
    const bool lin = nin > 0 || !cont;         // the last bucket starts inside it (else bl == b0)
    const uint64_t ts = nin > 0 ? sst[nin - 1] : t0;   // first tile of the last bucket here
    // digits of the first and the last bucket (a bucket's tile counts hold
    // only its own digits)
    const uint32_t rf = 1u << min(p.d_big, kf.kbits - list[b0].bit);
    const uint32_t rl = 1u << min(p.d_big, kf.kbits - list[bl].bit);
#pragma unroll 1
    for (uint32_t k = 0; k < KV; k++) {
      const uint32_t v = threadIdx.x + k * WG;
      if (v >= RS) break;
      uint32_t cnt[CH];
#pragma unroll
      for (uint32_t u = 0; u < CH; u++) cnt[u] = t0 + u < t1 ? w.tcnt[(t0 + u) * RS + v] : 0u;
      // 1. the last bucket's sum over this chunk, published at once
      uint64_t agg = 0;
#pragma unroll
      for (uint32_t u = 0; u < CH; u++) agg += t0 + u >= ts ? cnt[u] : 0u;
      uint64_t* cs = w.cstatus + c * RS;
      if (v < rl) atomic_store_agent(&cs[v], epoch | (lin ? LB_INC : LB_AGG) | agg);
      // 2. the carry into the first bucket: the sums of the earlier chunks
      //    back to one that holds that bucket's start
      uint64_t run = 0;
      if (cont && v < rf) {
        // the words of LW chunks are read at once, then used in order up to
        // the first inclusive one (or the first that is not ready yet)
        constexpr uint32_t LW = 16;
        uint64_t jc = c;  // the window is chunks jc-1, jc-2, ...
        uint32_t spins = 0;
        bool gave_up = false;
        for (;;) {
          // the wait is bounded: past the plan's poll limit the chunk gives
          // up, flags the error and publishes nothing more, so every wave
          // exits and the scatter of this level is skipped
          if (spins >= p.spin_limit) { atomicOr(&w.ctl->error, 2u); gave_up = true; break; }
          uint64_t sw[LW];
#pragma unroll
          for (uint32_t i = 0; i < LW; i++)
            sw[i] = jc > i ? atomic_load_agent(&w.cstatus[(jc - 1 - i) * RS + v]) : (epoch | LB_INC);
          bool done = false, stall = false;
          uint32_t used = 0;
#pragma unroll
          for (uint32_t i = 0; i < LW; i++) {
            if (done || stall) continue;
            const uint64_t s = sw[i];
            if ((s >> LB_EPOCH_SHIFT) != (epoch >> LB_EPOCH_SHIFT) || (s & LB_FLAGS) == 0) { stall = true; continue; }
            run += s & LB_VAL;
            used = i + 1;
            done = (s & LB_FLAGS) == LB_INC;
          }
          jc -= used;
          if (done) break;
          if (stall) {
            ++spins;
            __builtin_amdgcn_s_sleep(1);
          }
        }
        // a chunk inside one bucket can now publish its inclusive sum too
        // (not after a give-up: its carry is incomplete)
        if (!lin && !gave_up) atomic_store_agent(&cs[v], epoch | LB_INC | (run + agg));
      }
      // 3. the tiles' offsets
      uint32_t b = b0, nxt = 0;
      uint32_t r = rf;
      uint64_t base = v < r ? w.hist[(uint64_t)b * RS + v] : 0ull;
#pragma unroll
      for (uint32_t u = 0; u < CH; u++) {
        const uint64_t t = t0 + u;
        if (t < t1) {
          if (nxt < nin && sst[nxt] == t) {
            b++;
            nxt++;
            run = 0;
            r = 1u << min(p.d_big, kf.kbits - list[b].bit);
            base = v < r ? w.hist[(uint64_t)b * RS + v] : 0ull;
          }
          if (v < r) w.status[t * RS + v] = base + run;
          if (k == 0 && threadIdx.x == 0) w.tbucket[t] = b;
          run += cnt[u];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Stable scatter of one level.
//
// A tile is `tile` consecutive records of one bucket (the same tiles the
// histogram kernel counted); workgroups take tiles through an atomic ticket.
// Within a tile, wave q owns records [q*tile/4, (q+1)*tile/4) and takes them
// 64 at a time; a record's rank among equal digits is (count in earlier
// waves) + (count in earlier rounds of its wave) + (lanes of its round with
// the same digit below it), so the tile keeps input order within each digit.
// The tile stages its records in LDS ordered by digit and writes each
// digit's run contiguously at the offset the tile-offset scan computed for
// it, so no tile waits for another.
// SMALL: tiles of at most 32 words of records per thread (half the
// registers and staging), so that more workgroups share a CU.
template <int RW, int DB, bool SMALL>
__global__ __launch_bounds__(WG) void k_scatter(Plan p, Work w, uint32_t level, const uint8_t* rec0,
                                                uint8_t* rec0w, const uint8_t* rec1, uint8_t* rec1w) {
  constexpr uint32_t RMAX = 1u << DB;
  // at most 64 (SMALL: 32) words of records per thread, and 32 records (the
  // plan's tiles never hold more per thread)
  constexpr uint32_t IPT_MAX = RW >= 2 ? (SMALL ? 32 : 64) / RW : 32;
  extern __shared__ __align__(16) uint32_t stage[];
  // per-wave digit counters; with digits of at most 8 bits two sets, used by
  // alternate tiles, so a tile's set is cleared during the next tile and no
  // barrier closes the write-out
  constexpr bool DBUF = DB <= 8;
  constexpr uint32_t WCN = NWAVES * RMAX;
  __shared__ uint32_t wcnt[(DBUF ? 2 : 1) * WCN];
  __shared__ uint32_t toff[RMAX + 1];
  __shared__ uint64_t gbase[RMAX];
  __shared__ uint32_t sscan[NWAVES + 1];
  __shared__ uint64_t sticket;
  __shared__ uint32_t sb;

  const Bucket* list = level_list(p, w, level);
  const uint64_t* start = level_start(p, w, level);
  uint32_t nb = min((uint64_t)w.ctl->nbig[level], p.cap_big);
  uint64_t T = w.ctl->ntiles[level];
  if (nb == 0 || T == 0) return;
  // a tile-offset scan that gave up leaves offsets that are not to be used
  if (w.ctl->error & 2u) return;
  const KeyFmt kf = make_keyfmt(p.key_bytes);
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / 64;
  const uint32_t RS = 1u << p.d_big;
  const uint32_t IPT = p.tile / WG;
  const uint32_t per_wave = p.tile / NWAVES;
  const bool nt = p.nontemporal != 0;

  constexpr uint32_t RB = 4 * RW;  // record bytes
  // Tiles are claimed through an atomic ticket.  A tile's records are held in
  // registers only until they are staged in LDS; the next tile is claimed
  // before that staging barrier, and its records are loaded into the same
  // registers while the staged tile is written out.
  auto claim = [&]() {
    uint64_t tk = atomicAdd(&w.ctl->ticket[level], 1u);
    sticket = tk;
    sb = tk < T ? w.tbucket[tk] : 0;
  };
  Rec<RW> rec[IPT_MAX];
  // load tile `ticket` of list entry `b` (nothing for a finished claim or a
  // bucket whose move is skipped); offsets past the bucket read 0
  auto load_tile = [&](uint64_t ticket, uint32_t b) {
    if (ticket >= T) return;
    const Bucket B = list[b];
    if (B.flags & BF_SKIP) return;
    const uint64_t r0 = B.begin + (ticket - start[b]) * p.tile;
    const uint64_t bend = B.begin + B.count;
    const uint32_t cnt = (uint32_t)min((uint64_t)p.tile, bend - r0);
    const uint8_t* src = (B.flags & BF_TMP) ? rec1 : rec0;
    const __amdgpu_buffer_rsrc_t sr = job_rsrc(src + r0 * RB, cnt * RB);
    const uint32_t voff = (wave * per_wave + lane) * RB;
#pragma unroll
    for (uint32_t j = 0; j < IPT_MAX; j++)
      if (j < IPT) rec[j] = buf_load_rec<RW>(sr, voff, j * 64 * RB);
  };
  for (uint32_t i = threadIdx.x; i < (DBUF ? 2 : 1) * WCN; i += WG) wcnt[i] = 0;
  if (threadIdx.x == 0) claim();
  __syncthreads();
  uint32_t par = 0;  // counter set of the current tile
  uint64_t ticket = uniform64(sticket);
  uint32_t b = uniform32(sb);
  load_tile(ticket, b);
  for (;;) {
    if (ticket >= T) break;
    Bucket B = list[b];
    if (B.flags & BF_SKIP) {
      __syncthreads();  // everyone has read the ticket
      if (threadIdx.x == 0) claim();
      __syncthreads();
      ticket = uniform64(sticket);
      b = uniform32(sb);
      load_tile(ticket, b);
      continue;
    }
    uint64_t ti = ticket - start[b];
    uint64_t r0 = B.begin + ti * p.tile;
    // this tile's digit offsets, loaded early (used after the staging)
    const uint64_t tofs = threadIdx.x < (1u << min(p.d_big, kf.kbits - B.bit)) && threadIdx.x < RS
                              ? w.status[ticket * RS + threadIdx.x] : 0ull;
    uint64_t bend = B.begin + B.count;
    uint32_t cnt = (uint32_t)min((uint64_t)p.tile, bend - r0);
    uint32_t d = min(p.d_big, kf.kbits - B.bit);
    uint32_t R = 1u << d;
    uint32_t shift = kf.kbits - B.bit - d;
    uint32_t mask = R - 1u;
    uint8_t* dst = (B.flags & BF_TMP) ? rec0w : rec1w;

    // one register of rank state per record (the digit is recomputed from
    // the record where it is needed): more waves fit the register file
    uint32_t* const wc = wcnt + par * WCN;
    uint32_t rk[IPT_MAX];
    uint64_t wbase = r0 + (uint64_t)wave * per_wave;
#pragma unroll
    for (uint32_t j = 0; j < IPT_MAX; j++) {
      if (j < IPT) {
        uint64_t i = wbase + (uint64_t)j * 64 + lane;
        bool valid = i < bend;
        uint32_t v = valid ? key_digit(rec_key<RW>(rec[j], kf), shift, mask, kf) : 0u;
        rk[j] = rank_issue32(&wc[wave * RMAX], v, d, valid);
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < IPT_MAX; j++)
      if (j < IPT) rk[j] = rank_finish32(rk[j]);
    __syncthreads();
    // the tile's digit counts: per-wave bases, and the tile's own digit
    // starts (an exclusive scan) for staging
    if constexpr (DBUF) {
      // the other set (the previous tile's) is free: clear it for the next tile
      for (uint32_t i = threadIdx.x; i < WCN; i += WG) wcnt[(par ^ 1u) * WCN + i] = 0;
      // thread v takes digit v (R <= 256 = WG): bases over the waves, then
      // the tile's exclusive scan over the digits
      const uint32_t v = threadIdx.x;
      uint32_t tot = 0;
      if (v < R) {
#pragma unroll
        for (int q = 0; q < NWAVES; q++) { const uint32_t c = wc[q * RMAX + v]; wc[q * RMAX + v] = tot; tot += c; }
      }
      uint32_t wt;
      const uint32_t ex = wave_excl_scan(tot, &wt);
      if (lane == 0) sscan[wave] = wt;
      __syncthreads();
      uint32_t base = 0;
#pragma unroll
      for (uint32_t q = 0; q < NWAVES; q++) base += q < wave ? sscan[q] : 0u;
      if (v < R) toff[v] = base + ex;
      __syncthreads();
    } else {
      for (uint32_t v = threadIdx.x; v < R; v += WG) {
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < NWAVES; q++) { uint32_t c = wc[q * RMAX + v]; wc[q * RMAX + v] = s; s += c; }
        toff[v] = s;
      }
      __syncthreads();
      block_excl_scan_lds(toff, R, sscan);
    }
    // stage the records in LDS ordered by digit
#pragma unroll
    for (uint32_t j = 0; j < IPT_MAX; j++) {
      if (j < IPT) {
        uint64_t i = wbase + (uint64_t)j * 64 + lane;
        if (i < bend) {
          const uint32_t v = key_digit(rec_key<RW>(rec[j], kf), shift, mask, kf);
          uint32_t pos = toff[v] + wc[wave * RMAX + v] + rk[j];
          lds_put<RW>(stage, pos, rec[j]);
        }
      }
    }
    // where each digit's run of this tile goes (from the offset scan)
    if (R <= WG) {
      if (threadIdx.x < R) gbase[threadIdx.x] = B.begin + tofs - toff[threadIdx.x];
    } else {
      const uint64_t* to = w.status + ticket * RS;
      for (uint32_t v = threadIdx.x; v < R; v += WG) gbase[v] = B.begin + to[v] - toff[v];
    }
    if (threadIdx.x == 0) claim();
    __syncthreads();
    // the registers are free: the next tile's loads go out now
    ticket = uniform64(sticket);
    b = uniform32(sb);
    load_tile(ticket, b);
    for (uint32_t q = threadIdx.x; q < cnt; q += WG) {
      Rec<RW> r = lds_get<RW>(stage, q);
      uint32_t v = key_digit(rec_key<RW>(r, kf), shift, mask, kf);
      store_rec<RW>(dst, gbase[v] + q, r, nt);
    }
    if constexpr (DBUF) {
      // the next tile's first barrier comes after every thread's write-out
      // here, before its staging reuses the stage
      par ^= 1u;
    } else {
      for (uint32_t i = threadIdx.x; i < WCN; i += WG) wcnt[i] = 0;
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Copy finished buckets that lie in tmp back to records (tile-parallel).
template <int RW>
__global__ __launch_bounds__(WG) void k_copy(Plan p, Work w, const uint8_t* tmp, uint8_t* records) {
  __shared__ uint64_t sticket;
  __shared__ uint32_t sb;
  uint32_t nb = min((uint64_t)w.ctl->ncopy, p.cap_copy);
  uint64_t T = w.ctl->copy_tiles;
  if (nb == 0 || T == 0) return;
  for (;;) {
    if (threadIdx.x == 0) {
      uint64_t tk = atomicAdd(&w.ctl->copy_ticket, 1u);
      sticket = tk;
      sb = tk < T ? find_entry(w.copy_start, nb, tk) : 0;
    }
    __syncthreads();
    uint64_t ticket = sticket;
    uint32_t b = sb;
    __syncthreads();
    if (ticket >= T) break;
    Bucket B = w.copy[b];
    uint64_t r0 = B.begin + (ticket - w.copy_start[b]) * p.tile;
    uint64_t r1 = min(B.begin + B.count, r0 + p.tile);
    for (uint64_t i = r0 + threadIdx.x; i < r1; i += WG) store_rec<RW>(records, i, load_rec<RW>(tmp, i), false);
  }
}

// ---------------------------------------------------------------------------
// Order the single-workgroup queue by size class, largest first (Sec. 3.2:
// the queue hands out the largest bins first).
__global__ void k_class_count(Plan p, Work w) {
  __shared__ uint32_t c[NCLASS];
  for (uint32_t i = threadIdx.x; i < NCLASS; i += blockDim.x) c[i] = 0;
  __syncthreads();
  uint32_t ns = min((uint64_t)w.ctl->nsmall, p.cap_small);
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < ns; i += (uint64_t)gridDim.x * blockDim.x)
    atomicAdd(&c[63 - __clzll(w.small[i].count)], 1u);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < NCLASS; i += blockDim.x)
    if (c[i]) atomicAdd(&w.ctl->class_count[i], c[i]);
}

__global__ void k_class_offsets(Work w) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (int i = NCLASS - 1; i >= 0; i--) { uint32_t c = w.ctl->class_count[i]; w.ctl->class_count[i] = run; run += c; }
}

__global__ void k_class_scatter(Plan p, Work w) {
  uint32_t ns = min((uint64_t)w.ctl->nsmall, p.cap_small);
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < ns; i += (uint64_t)gridDim.x * blockDim.x) {
    Bucket b = w.small[i];
    uint32_t pos = atomicAdd(&w.ctl->class_count[63 - __clzll(b.count)], 1u);
    w.small_ord[pos] = b;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.

// Probe input of the autotuner: record i gets key mix(i + salt) (uniform) or
// mix(mix(i + salt) % distinct + salt) (at most `distinct` different keys),
// and its index as payload; other words are zero.  mix is the SplitMix64
// output function (Steele, Lea and Flood 2014).
__device__ __forceinline__ uint64_t probe_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void k_probe_fill(uint32_t* rec, uint64_t n, uint32_t rw, uint32_t kw, uint64_t salt, uint64_t distinct) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t h = probe_mix(i + salt);
    if (distinct) h = probe_mix(h % distinct + salt);
    uint32_t* r = rec + i * rw;
    for (uint32_t w = 0; w < rw; w++) {
      uint32_t v = 0;
      if (w < kw) v = (uint32_t)(w & 1 ? (h >> 32) : h) ^ (w >= 2 ? (uint32_t)probe_mix(h + w) : 0u);
      else if (w == kw) v = (uint32_t)i;
      else if (w == kw + 1) v = (uint32_t)(i >> 32);
      r[w] = v;
    }
  }
}

void launch_probe_fill(void* rec, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, uint64_t salt, uint64_t distinct,
                       hipStream_t s) {
  uint32_t grid = (uint32_t)std::min<uint64_t>((n + WG - 1) / WG, 65536);
  if (grid == 0) return;
  k_probe_fill<<<grid, WG, 0, s>>>((uint32_t*)rec, n, rec_bytes / 4, (key_bytes + 3) / 4, salt, distinct);
}

void launch_init(const Work& w, hipStream_t s) {
  k_init<<<1, WG, 0, s>>>(w);
}

void launch_seed_single(const Plan& p, const Work& w, hipStream_t s) {
  k_seed_single<<<1, 64, 0, s>>>(p, w);
}

void launch_seed_segments(const Plan& p, const Work& w, const uint64_t* off, uint32_t S, hipStream_t s) {
  uint32_t g = (S + WG) / WG;
  k_check_segments<<<g, WG, 0, s>>>(p, w, off, S);
  k_seed_segments<<<g, WG, 0, s>>>(p, w, off, S);
}

void launch_level_prep(const Plan& p, const Work& w, uint32_t level, hipStream_t s) {
  k_prefix<<<1, WG, 0, s>>>(w.big + (uint64_t)level * p.cap_big, &w.ctl->nbig[level], p.cap_big,
                            w.tile_start + (uint64_t)level * (p.cap_big + 1), &w.ctl->ntiles[level],
                            &w.ctl->ticket[level], p.tile);
  k_clear_hist<<<p.grid_clear, WG, 0, s>>>(p, w, level);
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
  const uint64_t words = bytes / 8;
  if (!words) return;
  const uint64_t blocks = (words + WG - 1) / WG;
  const uint32_t g = (uint32_t)(blocks < 4096 ? blocks : 4096);
  k_zero_words<<<g, WG, 0, s>>>((uint64_t*)p, words);
}

void launch_level_hist(const Plan& p, const Work& w, uint32_t level, void* records, void* tmp, hipStream_t s) {
  const uint8_t* r0 = (const uint8_t*)records;
  const uint8_t* r1 = (const uint8_t*)tmp;
  switch (p.rw * 2 + (p.d_big > 8 ? 1 : 0)) {
#define RD_CASE(n)                                                                         \
  case 2 * n:                                                                              \
    if (p.key_bytes > 8) k_hist_wave<n, true><<<p.grid_hist, WG, 0, s>>>(p, w, level, r0, r1); \
    else k_hist_wave<n, false><<<p.grid_hist, WG, 0, s>>>(p, w, level, r0, r1);            \
    break;                                                                                 \
  case 2 * n + 1: k_hist<n, 11><<<p.grid_hist, WG, 0, s>>>(p, w, level, r0, r1); break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

void launch_level_scan(const Plan& p, const Work& w, uint32_t level, hipStream_t s) {
  // one workgroup per bucket at a time; latency-bound, so a large grid
  const uint32_t g = 4 * p.grid_clear;
  if (p.d_big > 8) k_scan<11><<<g, WG, 0, s>>>(p, w, level);
  else k_scan<8><<<g, WG, 0, s>>>(p, w, level);
}

void launch_tile_scan(const Plan& p, const Work& w, uint32_t level, hipStream_t s) {
  if (p.d_big > 8) k_tile_scan<11><<<p.grid_clear, WG, 0, s>>>(p, w, level);
  else k_tile_scan<8><<<p.grid_clear, WG, 0, s>>>(p, w, level);
}

void launch_level_scatter(const Plan& p, const Work& w, uint32_t level, void* records, void* tmp, hipStream_t s) {
  const uint8_t* r0 = (const uint8_t*)records;
  const uint8_t* r1 = (const uint8_t*)tmp;
  uint8_t* w0 = (uint8_t*)records;
  uint8_t* w1 = (uint8_t*)tmp;
  size_t stage = (size_t)p.tile * p.rec_bytes;
  // tiles of at most 32 words per thread take the variant with half the
  // registers; its workgroups are more per CU
  const bool small = (uint64_t)p.tile * p.rw <= 32ull * WG;
  const uint32_t grid = small ? 2 * p.grid_scatter : p.grid_scatter;
  switch (p.rw * 2 + (p.d_big > 8 ? 1 : 0)) {
#define RD_CASE(n)                                                                                              \
  case 2 * n:                                                                                                   \
    if (small) k_scatter<n, 8, true><<<grid, WG, stage, s>>>(p, w, level, r0, w0, r1, w1);                     \
    else k_scatter<n, 8, false><<<grid, WG, stage, s>>>(p, w, level, r0, w0, r1, w1);                          \
    break;                                                                                                      \
  case 2 * n + 1: k_scatter<n, 11, false><<<grid, WG, stage, s>>>(p, w, level, r0, w0, r1, w1); break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

void launch_order_small(const Plan& p, const Work& w, hipStream_t s) {
  k_class_count<<<p.grid_clear, WG, 0, s>>>(p, w);
  k_class_offsets<<<1, 64, 0, s>>>(w);
  k_class_scatter<<<p.grid_clear, WG, 0, s>>>(p, w);
}

void launch_copy(const Plan& p, const Work& w, void* records, const void* tmp, hipStream_t s) {
  k_prefix<<<1, WG, 0, s>>>(w.copy, &w.ctl->ncopy, p.cap_copy, w.copy_start, &w.ctl->copy_tiles,
                            &w.ctl->copy_ticket, p.tile);
  switch (p.rw) {
#define RD_CASE(n) case n: k_copy<n><<<p.grid_scatter, WG, 0, s>>>(p, w, (const uint8_t*)tmp, (uint8_t*)records); break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

}  // namespace rd
