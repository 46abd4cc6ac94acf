// k_inplace.hip -- MSD levels that partition every bucket within its own
// records, with no second buffer of the input's size.
//
// The paper sets its out-of-place distribution against in-place radix
// sorting (Sec. 2): there records are swapped into their bins, and a
// parallel version alternates a speculative permutation with a repair step
// until every record sits in its bin.  Here the unit that moves is a block
// of records of one digit (at most 512 bytes), so that every move is one
// coalesced transfer by one wavefront:
//
// 1. classify: a workgroup reads its stripe of a bucket tile by tile and
//    collects the records per digit in LDS buffers of one block; every full
//    block is written back at the stripe's front, which has already been
//    read.  What stays in the buffers at the stripe's end (less than a block
//    per digit) goes to a side buffer.
// 2. ranges: child v owns the block slots [f, e) that cover its records
//    (f = first slot starting inside it).  The full blocks inside that range
//    are moved to its front, so the range reads [unread blocks | free slots].
// 3. permute: wavefronts take unread blocks from the back of a range (read
//    cursor) and put each at the write cursor of its digit's range.  A slot
//    below that range's read cursor still holds an unread block, which is
//    taken out first and carried on (the swap of the speculative
//    permutation); both cursors of a range share one 64-bit word, so a slot
//    is either read or written first, never both.  A writer that lands on a
//    slot whose reader has not finished waits for the slot's bit.
// 4. cleanup: each child's edges -- less than a block at its head, the rest
//    after its last full block -- receive its leftovers and the part of its
//    last block that ran past its end (kept aside by that block's writer).
//
// A bucket of at most IP_MLB blocks is done by one workgroup from start to
// end (k_ip_medium), its buffers, cursors and bits in LDS.  The order of equal
// keys is not kept: the in-place sort is not stable.
#include "raduls_dev.hpp"
#include "raduls_kernels.hpp"

namespace rd {

namespace {

constexpr uint32_t IP_WAVES = IP_WG / 64;
constexpr uint32_t IP_PERM_WG = 256;               // threads of the permutation workgroups
// A range's blocks of its own digit are swapped to its front by its one
// workgroup only if at most this many blocks of the range are foreign
// (bounding the pairs it swaps); otherwise the permutation moves them all.
constexpr uint32_t IP_OWN_SWAP_MAX = 1u << 16;

__device__ __forceinline__ const Bucket* ip_list(const Plan& p, const Work& w, uint32_t level) {
  return w.big + (uint64_t)level * p.cap_big;
}

struct Dig {
  uint32_t shift, mask;
};
__device__ __forceinline__ Dig bucket_digit(const Plan& p, const KeyFmt& kf, uint32_t bit) {
  const uint32_t d = min(p.d_big, kf.kbits - bit);
  return Dig{kf.kbits - bit - d, (1u << d) - 1u};
}

__device__ __forceinline__ void wait_loads() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ uint64_t bcast64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Exclusive prefix over threads 0..IP_R-1 of a 1024-thread workgroup (the
// others pass 0); the total goes to *tot.  Two barriers.
__device__ __forceinline__ uint32_t scan_r(uint32_t x, uint32_t* tmp4, uint32_t* tot) {
  const uint32_t t = threadIdx.x;
  uint32_t wt;
  const uint32_t ex = wave_excl_scan(x, &wt);
  if (t < IP_R && lane_id() == 0) tmp4[t / 64] = wt;
  __syncthreads();
  uint32_t base = 0, total = 0;
#pragma unroll
  for (uint32_t q = 0; q < IP_R / 64; q++) {
    const uint32_t y = tmp4[q];
    base += q < t / 64 ? y : 0u;
    total += y;
  }
  __syncthreads();
  *tot = total;
  return base + ex;
}

// The same for 64-bit values.
__device__ __forceinline__ uint64_t scan_r64(uint64_t x, uint64_t* tmp4, uint64_t* tot) {
  const uint32_t t = threadIdx.x, l = lane_id();
  uint64_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up((unsigned long long)inc, o);
    if (l >= (uint32_t)o) inc += y;
  }
  if (t < IP_R && l == 63) tmp4[t / 64] = inc;
  __syncthreads();
  uint64_t base = 0, total = 0;
#pragma unroll
  for (uint32_t q = 0; q < IP_R / 64; q++) {
    const uint64_t y = tmp4[q];
    base += q < t / 64 ? y : 0ull;
    total += y;
  }
  __syncthreads();
  *tot = total;
  return base + inc - x;
}

// Exclusive scan in place of `count` (<= 16 * IP_WG) values in LDS by a
// 1024-thread workgroup; returns the total.  Two barriers.
__device__ __forceinline__ uint32_t scan_lds(uint32_t* a, uint32_t count, uint32_t* tmp16) {
  const uint32_t t = threadIdx.x;
  const uint32_t per = (count + IP_WG - 1) / IP_WG;
  const uint32_t lo = min(count, t * per), hi = min(lo + per, count);
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; i++) s += a[i];
  uint32_t wt;
  const uint32_t ex = wave_excl_scan(s, &wt);
  if (lane_id() == 0) tmp16[t / 64] = wt;
  __syncthreads();
  uint32_t base = 0, total = 0;
#pragma unroll
  for (uint32_t q = 0; q < IP_WAVES; q++) {
    const uint32_t y = tmp16[q];
    base += q < t / 64 ? y : 0u;
    total += y;
  }
  uint32_t run = base + ex;
  for (uint32_t i = lo; i < hi; i++) {
    const uint32_t c = a[i];
    a[i] = run;
    run += c;
  }
  __syncthreads();
  return total;
}

// Last index j in [0, n) with a[j] <= x (a non-decreasing, a[0] <= x).
__device__ __forceinline__ uint32_t last_le(const uint32_t* a, uint32_t n, uint32_t x) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (a[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---- blocks held by one wavefront -------------------------------------------
// A block of B records is WB = B * RW words; lane l holds words l and l + 64.
struct Blk {
  uint32_t a, b;
};

__device__ __forceinline__ Blk blk_load(const uint32_t* p, uint32_t WB, uint32_t lane) {
  Blk x{0u, 0u};
  if (lane < WB) x.a = p[lane];
  if (lane + 64 < WB) x.b = p[lane + 64];
  return x;
}

__device__ __forceinline__ void blk_store(uint32_t* p, Blk x, uint32_t WB, uint32_t lane) {
  if (lane < WB) p[lane] = x.a;
  if (lane + 64 < WB) p[lane + 64] = x.b;
}

// Digit of the block's first record (all its records share it).
template <int RW>
__device__ __forceinline__ uint32_t blk_digit(Blk x, const KeyFmt& kf, Dig g) {
  uint64_t lo = (uint32_t)__shfl((int)x.a, 0);
  if constexpr (RW > 1) lo |= (uint64_t)(uint32_t)__shfl((int)x.a, 1) << 32;
  uint64_t hi = 0;
  if constexpr (RW > 2) hi = (uint32_t)__shfl((int)x.a, 2);
  if constexpr (RW > 3) hi |= (uint64_t)(uint32_t)__shfl((int)x.a, 3) << 32;
  return __builtin_amdgcn_readfirstlane(key_digit(Key{lo & kf.mlo, hi & kf.mhi}, g.shift, g.mask, kf));
}

// Child ranges of one bucket: cursors, first slot, blocks and end (records
// relative to the bucket) of each child, and the read cursor's start.
struct Ranges {
  uint64_t* W;
  const uint32_t* rinit;
  const uint32_t* f;
  const uint32_t* F;
  const uint64_t* lim;
};

// Write a block of child v at slot s: the records inside the bucket go to
// the records, those past the child's end also to the child's aside area.
template <int RW>
__device__ __forceinline__ void put_block(Blk x, uint32_t* recw, uint64_t count, uint32_t s, uint32_t B,
                                          uint64_t lim, uint32_t* protw, uint32_t lane) {
  const uint32_t WB = B * RW;
  const uint64_t s0 = (uint64_t)s * B;
  const uint32_t alim = (uint32_t)min<uint64_t>(B, count - s0);  // records of the slot inside the bucket
  const uint32_t plo = (uint32_t)min<uint64_t>(B, lim - s0);     // first record past the child's end
  uint32_t* dst = recw + s0 * RW;
#pragma unroll
  for (uint32_t h = 0; h < 2; h++) {
    const uint32_t j = lane + 64 * h;
    if (j < WB) {
      const uint32_t val = h ? x.b : x.a;
      const uint32_t o = j / RW;
      if (o < alim) dst[j] = val;
      if (o >= plo) protw[j - plo * RW] = val;
    }
  }
}

// One wavefront moves blocks of the workgroup's own bucket (cursors and
// bits in LDS) with four chains at a time.  A chain without a block takes
// one from the back of a range (the wavefront visits every range once, its
// own 16 first, each until it is exhausted, so that all wavefronts help
// drain a child that holds most blocks); a chain with a block of digit v claims
// v's write slot: a slot still below v's read cursor holds an unread block,
// which is taken out first and carried on; a slot claimed by a reader is
// waited for through its bit (bounded).  Per round all chains' claims and
// block loads are issued before any is waited for, and read bits are set
// before any chain waits on one.
template <int RW>
__device__ void ip_drain_multi(const Ranges& rg, uint32_t first, uint32_t* recw, uint64_t count,
                               uint32_t B, Dig g, const KeyFmt& kf, uint32_t* done, uint32_t* protw0,
                               uint32_t spin_limit, uint32_t* err) {
  constexpr uint32_t NC = 4;
  const uint32_t lane = lane_id();
  const uint32_t WB = B * RW;
  const uint32_t PW = IP_BLOCK_BYTES / 4;
  const uint64_t nblk = (count + B - 1) / B;
  // visiting order: the wavefront's own ranges first, first + 16 b (b < 16),
  // then those of the next wavefront, and so on: visit k = 16 a + b goes to
  // range first + 16 b + a (mod 256), every range once
  constexpr uint32_t NW = IP_R / 16;
  auto range_of = [&](uint32_t k) -> uint32_t { return (first + 16u * (k % NW) + k / NW) % IP_R; };
  uint32_t visited = 0, ri = range_of(0);
  bool more = true;
  Blk x[NC], y[NC];
  uint32_t v[NC], slot[NC], mode[NC];
  uint64_t lim[NC];
  bool has[NC];
#pragma unroll
  for (uint32_t c = 0; c < NC; c++) {
    has[c] = false;
    v[c] = slot[c] = mode[c] = 0;
    lim[c] = 0;
    x[c] = y[c] = Blk{0u, 0u};
  }
  enum : uint32_t { NONE = 0, READ = 1, SWAP = 2, PLACE = 3 };
  for (;;) {
    uint32_t nneed = 0;
    bool busy = false;
#pragma unroll
    for (uint32_t c = 0; c < NC; c++) {
      nneed += has[c] ? 0u : 1u;
      busy = busy || has[c];
    }
    // ranges already drained are passed by a plain read of their word (a
    // hint: the claim below decides)
    while (nneed && more) {
      const uint64_t wv = bcast64(__shfl((unsigned long long)rg.W[ri], 0));
      if ((int64_t)(uint32_t)wv - (int64_t)IP_BIAS > (int64_t)(wv >> 32)) break;
      more = ++visited < IP_R;
      ri = range_of(visited);
    }
    if (!busy && !more) break;
    if (!more) nneed = 0;
    uint64_t rold = 0;
    if (nneed && lane == 0) rold = atomicAdd((unsigned long long*)&rg.W[ri], 0ull - nneed);
    uint64_t old[NC];
#pragma unroll
    for (uint32_t c = 0; c < NC; c++) {
      old[c] = 0;
      mode[c] = NONE;
      if (has[c]) {
        mode[c] = SWAP;
        if (lane == 0) old[c] = atomicAdd((unsigned long long*)&rg.W[v[c]], 1ull << 32);
      }
    }
    uint32_t rfirst = 0, ngot = 0;
    if (nneed) {
      const uint64_t o = bcast64(__shfl((unsigned long long)rold, 0));
      const int64_t wc = (int64_t)(o >> 32), rc = (int64_t)(uint32_t)o - (int64_t)IP_BIAS;
      const int64_t avail = rc - wc;
      ngot = avail <= 0 ? 0u : (uint32_t)min<int64_t>(avail, nneed);
      rfirst = (uint32_t)(rc - (int64_t)ngot);
      if (ngot && (uint64_t)rc > nblk) {  // cannot happen
        if (lane == 0) atomicOr(err, 4u);
        ngot = 0;
      }
      if (ngot < nneed) {  // range exhausted (it stays so): the next one
        more = ++visited < IP_R;
        ri = range_of(visited);
      }
    }
    uint32_t k = 0;
#pragma unroll
    for (uint32_t c = 0; c < NC; c++) {
      if (!has[c] && k < ngot) {
        mode[c] = READ;
        slot[c] = rfirst + k;
        x[c] = blk_load(recw + (uint64_t)slot[c] * WB, WB, lane);
        k++;
      }
      if (mode[c] != SWAP) continue;
      const uint64_t o = bcast64(__shfl((unsigned long long)old[c], 0));
      const int64_t rc = (int64_t)(uint32_t)o - (int64_t)IP_BIAS;
      const uint32_t ws = (uint32_t)(o >> 32);
      if (ws >= rg.f[v[c]] + rg.F[v[c]] || ws >= nblk) {  // cannot happen: drop the block, report
        if (lane == 0) atomicOr(err, 4u);
        mode[c] = NONE;
        has[c] = false;
        continue;
      }
      slot[c] = ws;
      lim[c] = rg.lim[v[c]];
      if ((int64_t)ws < rc) y[c] = blk_load(recw + (uint64_t)ws * WB, WB, lane);
      else mode[c] = PLACE;
    }
    wait_loads();
    if (ngot && lane == 0) {
      for (uint32_t j = 0; j < ngot; j++) atomicOr(&done[(rfirst + j) >> 5], 1u << ((rfirst + j) & 31));
    }
#pragma unroll
    for (uint32_t c = 0; c < NC; c++) {
      if (mode[c] != READ) continue;
      v[c] = blk_digit<RW>(x[c], kf, g);
      has[c] = true;
    }
#pragma unroll
    for (uint32_t c = 0; c < NC; c++) {
      if (mode[c] != SWAP && mode[c] != PLACE) continue;
      const uint32_t ws = slot[c];
      if (mode[c] == PLACE && ws < rg.rinit[v[c]]) {
        uint32_t spins = 0;
        for (;;) {
          uint32_t word = 0;
          if (lane == 0) word = __hip_atomic_load(&done[ws >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          word = __builtin_amdgcn_readfirstlane(__shfl(word, 0));
          if ((word >> (ws & 31)) & 1u) break;
          if (++spins > spin_limit) {
            if (lane == 0) atomicOr(err, 2u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      put_block<RW>(x[c], recw, count, ws, B, lim[c], protw0 + v[c] * PW, lane);
      if (mode[c] == SWAP) {
        x[c] = y[c];
        v[c] = blk_digit<RW>(y[c], kf, g);
      } else {
        has[c] = false;
      }
    }
  }
}

// ---- classification ---------------------------------------------------------

struct IpCls {
  uint32_t cnt[IP_R];   // records of each digit in the current tile
  uint32_t fill[IP_R];  // records in each digit's buffer
  uint32_t nbv[IP_R];   // blocks each digit completes in the current tile
  uint32_t blk[IP_R];   // the first of them (block index in the stripe)
  uint32_t tot[IP_R];   // records of each digit in the stripe
  uint32_t tmp4[IP_WAVES];
  uint32_t wpos;        // blocks written at the stripe's front
  uint32_t item;
};

// Rewrite records [s0, s1) of the bucket at P (s0 on a block boundary of
// the bucket) as whole blocks of one digit each from s0 on; the records
// that fill no block stay in `buf` (digit v: S.fill[v] records from record
// v * B).  OR of every key XOR a key of the bucket into vlo/vhi.
template <int RW>
__device__ void classify(uint8_t* rec, uint64_t P, uint64_t s0, uint64_t s1, Dig g, const KeyFmt& kf, uint32_t B,
                         uint32_t* buf, IpCls& S, uint64_t& vlo, uint64_t& vhi, uint8_t* bdig) {
  const uint32_t t = threadIdx.x;
  constexpr uint32_t IP_IPT = RW > 8 ? 2 : 4;  // records per thread of a tile
  constexpr uint32_t TILE = IP_IPT * IP_WG;
  if (t < IP_R) {
    S.cnt[t] = 0;
    S.fill[t] = 0;
    S.tot[t] = 0;
  }
  if (t == 0) S.wpos = 0;
  const Key ref = load_key<RW>(rec, P + s0, kf);  // any key of the bucket will do
  wait_loads();  // other wavefronts write this record's slot from the first tile on
  __syncthreads();
  for (uint64_t t0 = s0; t0 < s1; t0 += TILE) {
    Rec<RW> r[IP_IPT];
    uint32_t v[IP_IPT], q[IP_IPT];
#pragma unroll
    for (uint32_t u = 0; u < IP_IPT; u++) {
      const uint64_t i = t0 + u * IP_WG + t;
      if (i < s1) r[u] = load_rec<RW>(rec, P + i);
    }
#pragma unroll
    for (uint32_t u = 0; u < IP_IPT; u++) {
      const uint64_t i = t0 + u * IP_WG + t;
      const bool ok = i < s1;
      v[u] = 0;
      q[u] = 0;
      if (ok) {
        const Key k = rec_key<RW>(r[u], kf);
        vlo |= k.lo ^ ref.lo;
        vhi |= k.hi ^ ref.hi;
        v[u] = key_digit(k, g.shift, g.mask, kf);
      }
      // a wave whose records share one digit (runs of equal keys) takes its
      // ranks with one atomic instead of 64 on the same counter
      const uint64_t act = __ballot(ok);
      const uint32_t v0 = __shfl(v[u], 0);
      if (act == ~0ull && __ballot(v[u] == v0) == ~0ull) {
        uint32_t base = 0;
        if (lane_id() == 0) base = atomicAdd(&S.cnt[v0], 64u);
        q[u] = (uint32_t)__shfl(base, 0) + lane_id();
      } else if (ok) {
        q[u] = atomicAdd(&S.cnt[v[u]], 1u);
      }
    }
    // every word of the tile must be in registers before any wavefront
    // writes blocks, which may land inside this tile
    wait_loads();
    __syncthreads();
    uint32_t nb = 0, nf = 0, c = 0;
    if (t < IP_R) {
      c = S.cnt[t];
      const uint32_t f = S.fill[t];
      nb = (f + c) / B;
      nf = f + c - nb * B;
    }
    uint32_t total;
    const uint32_t ex = scan_r(nb, S.tmp4, &total);
    const uint32_t wp = S.wpos;
    if (t < IP_R) {
      S.blk[t] = wp + ex;
      S.nbv[t] = nb;
      S.tot[t] += c;
      S.cnt[t] = 0;
      // each block's digit, by its index from the stripe's first block
      if (bdig)
        for (uint32_t q = 0; q < nb; q++) bdig[wp + ex + q] = (uint8_t)t;
    }
    __syncthreads();
    if (t == 0) S.wpos = wp + total;
    // buffers of digits that complete a block go out first ...
    for (uint32_t idx = t; idx < IP_R * B; idx += IP_WG) {
      const uint32_t vv = idx / B, ss = idx - vv * B;
      if (S.nbv[vv] && ss < S.fill[vv])
        store_rec<RW>(rec, P + s0 + (uint64_t)S.blk[vv] * B + ss, lds_get<RW>(buf, vv * B + ss), false);
    }
    // ... with the records of this tile that complete blocks
#pragma unroll
    for (uint32_t u = 0; u < IP_IPT; u++) {
      const uint64_t i = t0 + u * IP_WG + t;
      if (i < s1) {
        const uint32_t pos = S.fill[v[u]] + q[u];
        const uint32_t nbu = S.nbv[v[u]];
        if (pos < nbu * B) {
          const uint32_t bi = pos / B;
          store_rec<RW>(rec, P + s0 + (uint64_t)(S.blk[v[u]] + bi) * B + (pos - bi * B), r[u], false);
          q[u] = 0xFFFFFFFFu;
        } else {
          q[u] = pos - nbu * B;
        }
      }
    }
    __syncthreads();
    // the rest refill the buffers
#pragma unroll
    for (uint32_t u = 0; u < IP_IPT; u++) {
      const uint64_t i = t0 + u * IP_WG + t;
      if (i < s1 && q[u] != 0xFFFFFFFFu) lds_put<RW>(buf, v[u] * B + q[u], r[u]);
    }
    if (t < IP_R) S.fill[t] = nf;
    __syncthreads();
  }
}

__device__ __forceinline__ void or_vary(const Work& w, uint32_t bi, uint64_t vlo, uint64_t vhi) {
  const uint64_t a = wave_or64(vlo), c = wave_or64(vhi);
  if (lane_id() == 0) {
    if (a) atomicOr((unsigned long long*)&w.vary[2 * bi], (unsigned long long)a);
    if (c) atomicOr((unsigned long long*)&w.vary[2 * bi + 1], (unsigned long long)c);
  }
}

// ---- level set-up ------------------------------------------------------------

// Sort the level's buckets into large ones (several stripes) and medium
// ones (one workgroup), and number the large ones' stripes.
__global__ __launch_bounds__(IP_WG) void k_ip_setup(Plan p, Work w, IpWork iw, uint32_t level) {
  __shared__ uint32_t tmp16[IP_WAVES];
  __shared__ uint32_t a[IP_WG], b[IP_WG], m[IP_WG];
  __shared__ uint32_t run_l, run_s, run_m;
  const uint32_t t = threadIdx.x;
  const Bucket* list = ip_list(p, w, level);
  const uint32_t nb = (uint32_t)min((uint64_t)w.ctl->nbig[level], p.cap_big);
  const uint64_t SL = (uint64_t)iw.slb * ip_block_records(p.rw);  // records per stripe
  const uint64_t ML = (uint64_t)iw.mlb * ip_block_records(p.rw);  // records of a one-workgroup bucket, at most
  if (t == 0) {
    run_l = run_s = run_m = 0;
    iw.ctl->stripe_ticket = 0;
    iw.ctl->medium_ticket = 0;
    iw.ctl->chunk_ticket = 0;
  }
  __syncthreads();
  bool bad = false;
  for (uint32_t c0 = 0; c0 < nb; c0 += IP_WG) {
    const uint32_t i = c0 + t;
    uint64_t cnt = i < nb ? list[i].count : 0;
    const bool lg = i < nb && cnt > ML;
    const uint64_t ns = lg ? (cnt + SL - 1) / SL : 0;
    if (ns > IP_MAX_STRIPES) bad = true;
    a[t] = lg ? 1u : 0u;
    b[t] = (uint32_t)min<uint64_t>(ns, IP_MAX_STRIPES);
    m[t] = (i < nb && !lg) ? 1u : 0u;
    __syncthreads();
    const uint32_t tl = scan_lds(a, IP_WG, tmp16);
    const uint32_t ts = scan_lds(b, IP_WG, tmp16);
    const uint32_t tm = scan_lds(m, IP_WG, tmp16);
    const uint32_t L0 = run_l, S0 = run_s, M0 = run_m;
    if (lg) {
      const uint32_t li = L0 + a[t];
      if (li < iw.cap_large) {
        iw.large[li] = i;
        iw.stripe_first[li] = S0 + b[t];
      } else {
        bad = true;
      }
    } else if (i < nb) {
      iw.medium[M0 + m[t]] = i;
    }
    __syncthreads();
    if (t == 0) {
      run_l = L0 + tl;
      run_s = S0 + ts;
      run_m = M0 + tm;
    }
    __syncthreads();
  }
  if (bad) atomicOr(&iw.ctl->error, 1u);
  __syncthreads();
  if (t == 0) {
    uint32_t nl = run_l, ns = run_s;
    if (nl > iw.cap_large || ns > iw.cap_stripes) {  // cannot happen with the plan's capacities
      atomicOr(&iw.ctl->error, 1u);
      nl = 0;
      ns = 0;
    }
    iw.ctl->nlarge = nl;
    iw.ctl->nstripes = ns;
    iw.ctl->nmedium = run_m;
    iw.ctl->nranges = nl * IP_R;
    if (nl) iw.stripe_first[nl] = ns;
  }
}

// ---- classification of the stripes of large buckets -------------------------

template <int RW>
__global__ __launch_bounds__(IP_WG) void k_ip_classify(Plan p, Work w, IpWork iw, uint32_t level, uint8_t* rec) {
  extern __shared__ __align__(16) uint32_t buf[];
  __shared__ IpCls S;
  const KeyFmt kf = make_keyfmt(p.key_bytes);
  const uint32_t B = ip_block_records(RW);
  const Bucket* list = ip_list(p, w, level);
  const uint32_t ns = iw.ctl->nstripes, nl = iw.ctl->nlarge;
  const uint32_t RS = 1u << p.d_big;
  const uint32_t t = threadIdx.x;
  const uint64_t SL = (uint64_t)iw.slb * B;
  for (;;) {
    if (t == 0) S.item = atomicAdd(&iw.ctl->stripe_ticket, 1u);
    __syncthreads();
    const uint32_t s = S.item;
    __syncthreads();
    if (s >= ns) break;
    const uint32_t lb = last_le(iw.stripe_first, nl, s);
    const uint32_t bi = iw.large[lb];
    const Bucket Bk = list[bi];
    const uint64_t s0 = (uint64_t)(s - iw.stripe_first[lb]) * SL;
    const uint64_t s1 = min(Bk.count, s0 + SL);
    const Dig g = bucket_digit(p, kf, Bk.bit);
    uint64_t vlo = 0, vhi = 0;
    classify<RW>(rec, Bk.begin, s0, s1, g, kf, B, buf, S, vlo, vhi, iw.bdig + Bk.begin / B + s0 / B);
    // leftovers aside, counts to the bucket's histogram
    uint8_t* side = iw.side + (uint64_t)s * IP_R * IP_BLOCK_BYTES;
    for (uint32_t idx = t; idx < IP_R * B; idx += IP_WG) {
      const uint32_t vv = idx / B, ss = idx - vv * B;
      if (ss < S.fill[vv]) store_rec<RW>(side + (uint64_t)vv * IP_BLOCK_BYTES, ss, lds_get<RW>(buf, vv * B + ss), false);
    }
    if (t < IP_R) {
      iw.lcnt[(uint64_t)s * IP_R + t] = (uint16_t)S.fill[t];
      if (S.tot[t]) atomicAdd((unsigned long long*)&w.hist[(uint64_t)bi * RS + t], (unsigned long long)S.tot[t]);
    }
    if (t == 0) iw.nbfull[s] = S.wpos;
    or_vary(w, bi, vlo, vhi);
    __syncthreads();
  }
}

// ---- a whole bucket by one workgroup ------------------------------------------

struct IpMed {
  uint64_t W[IP_R];
  uint64_t lim[IP_R];
  uint32_t base[IP_R], f[IP_R], F[IP_R], rinit[IP_R];
  uint32_t done[IP_MLB / 32];
};

template <int RW>
__global__ __launch_bounds__(IP_WG) void k_ip_medium(Plan p, Work w, IpWork iw, uint32_t level, uint8_t* rec) {
  extern __shared__ __align__(16) uint32_t buf[];
  __shared__ IpCls S;
  __shared__ IpMed M;
  const KeyFmt kf = make_keyfmt(p.key_bytes);
  const uint32_t B = ip_block_records(RW);
  const Bucket* list = ip_list(p, w, level);
  const uint32_t nm = iw.ctl->nmedium;
  const uint32_t RS = 1u << p.d_big;
  const uint32_t t = threadIdx.x, wave = t / 64, lane = lane_id();
  uint32_t* protw0 = reinterpret_cast<uint32_t*>(iw.mscratch + (uint64_t)blockIdx.x * IP_R * IP_BLOCK_BYTES);
  for (;;) {
    if (t == 0) S.item = atomicAdd(&iw.ctl->medium_ticket, 1u);
    __syncthreads();
    const uint32_t mi = S.item;
    __syncthreads();
    if (mi >= nm) break;
    const uint32_t bi = iw.medium[mi];
    const Bucket Bk = list[bi];
    const uint64_t P = Bk.begin, count = Bk.count;
    const Dig g = bucket_digit(p, kf, Bk.bit);
    uint64_t vlo = 0, vhi = 0;
    classify<RW>(rec, P, 0, count, g, kf, B, buf, S, vlo, vhi, nullptr);
    or_vary(w, bi, vlo, vhi);
    // children: bases, slot ranges, cursors (the full blocks are a prefix)
    const uint32_t c = t < IP_R ? S.tot[t] : 0u;
    uint32_t total;
    const uint32_t base = scan_r(c, S.tmp4, &total);
    const uint32_t nbf = S.wpos;
    if (t < IP_R) {
      if (c) w.hist[(uint64_t)bi * RS + t] = c;
      const uint32_t L = S.fill[t];
      const uint32_t f = (base + B - 1) / B, lim = base + c, e = (lim + B - 1) / B;
      const uint32_t Fr = f < nbf ? min(e, nbf) - f : 0u;
      // a bucket whose records all have one digit: its blocks are in place
      const uint32_t wstart = c == count ? f + Fr : f;
      M.W[t] = ((uint64_t)wstart << 32) | (uint64_t)(f + Fr + IP_BIAS);
      M.lim[t] = lim;
      M.base[t] = base;
      M.f[t] = f;
      M.F[t] = (c - L) / B;
      M.rinit[t] = f + Fr;
    }
    for (uint32_t i = t; i < (uint32_t)((count + 32ull * B - 1) / (32ull * B)); i += IP_WG) M.done[i] = 0;
    __syncthreads();
    const Ranges rg{M.W, M.rinit, M.f, M.F, M.lim};
    uint32_t* recw = reinterpret_cast<uint32_t*>(rec + P * (uint64_t)(4 * RW));
    ip_drain_multi<RW>(rg, wave, recw, count, B, g, kf, M.done, protw0, p.spin_limit, &iw.ctl->error);
    __syncthreads();
    // edges of each child: leftovers (LDS), then the part of its last block
    // past its end (aside area, written by other wavefronts of this group)
    for (uint32_t v = wave; v < IP_R; v += IP_WAVES) {
      const uint32_t L = S.fill[v];
      const uint32_t b0 = M.base[v], f = M.f[v], F = M.F[v];
      const uint32_t lim = (uint32_t)M.lim[v];
      const uint32_t E = (f + F) * B;
      const uint32_t head_end = F ? min(f * B, lim) : lim;
      const uint32_t tail0 = F ? min(E, lim) : lim;
      const uint32_t nh = (head_end - b0) + (lim - tail0);
      const uint32_t* pw = protw0 + v * (IP_BLOCK_BYTES / 4);
      for (uint32_t k = lane; k < nh; k += 64) {
        const uint32_t dst = k < head_end - b0 ? b0 + k : tail0 + (k - (head_end - b0));
        Rec<RW> r;
        if (k < L) {
          r = lds_get<RW>(buf, v * B + k);
        } else {
#pragma unroll
          for (int j = 0; j < RW; j++)
            r.w[j] = __hip_atomic_load(pw + (k - L) * RW + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        store_rec<RW>(rec, P + dst, r, false);
      }
    }
    __syncthreads();
  }
}

// ---- large buckets: children, ranges, permutation, cleanup -------------------

// Per child of each large bucket: count, leftovers, base, slot range.
__global__ __launch_bounds__(IP_WG) void k_ip_bucket(Plan p, Work w, IpWork iw, uint32_t level) {
  __shared__ uint32_t part[IP_WG];
  __shared__ uint64_t tmp64[4];
  const uint32_t nl = iw.ctl->nlarge;
  const uint32_t B = ip_block_records(p.rw);
  const uint32_t RS = 1u << p.d_big;
  const uint32_t t = threadIdx.x;
  for (uint32_t lb = blockIdx.x; lb < nl; lb += gridDim.x) {
    const uint32_t bi = iw.large[lb];
    const uint32_t sf = iw.stripe_first[lb], sn = iw.stripe_first[lb + 1] - sf;
    // leftovers of digit t % 256 over a quarter of the stripes each
    const uint32_t v = t % IP_R, qtr = t / IP_R;
    uint32_t L = 0;
    for (uint32_t j = qtr; j < sn; j += IP_WG / IP_R) L += iw.lcnt[(uint64_t)(sf + j) * IP_R + v];
    part[t] = L;
    __syncthreads();
    uint64_t cnt = 0;
    if (t < IP_R) {
      L = part[t] + part[t + IP_R] + part[t + 2 * IP_R] + part[t + 3 * IP_R];
      cnt = w.hist[(uint64_t)bi * RS + t];
    }
    uint64_t total;
    const uint64_t base = scan_r64(cnt, tmp64, &total);
    if (t < IP_R) {
      const uint64_t r = (uint64_t)lb * IP_R + t;
      const uint64_t lim = base + cnt;
      if ((cnt - L) % B) atomicOr(&iw.ctl->error, 4u);
      iw.rbase[r] = base;
      iw.rlim[r] = lim;
      iw.rf[r] = (uint32_t)((base + B - 1) / B);
      iw.re[r] = (uint32_t)((lim + B - 1) / B);
      iw.rF[r] = (uint32_t)((cnt - L) / B);
      iw.rL[r] = L;
    }
    __syncthreads();
  }
}

// Per child range of a large bucket: move its full blocks to its front, set
// its cursors, count its permutation chunks.
template <int RW>
__global__ __launch_bounds__(IP_WG) void k_ip_ranges(Plan p, Work w, IpWork iw, uint32_t level, uint8_t* rec) {
  __shared__ uint32_t hpre[IP_MAX_STRIPES + 1], mpre[IP_MAX_STRIPES + 1];
  __shared__ uint32_t tmp16[IP_WAVES];
  __shared__ uint32_t s_fr, s_h, s_pa, s_pb, s_na, s_nb, s_ca, s_cb;
  const uint32_t nr = iw.ctl->nranges;
  const uint32_t B = ip_block_records(RW), WB = B * RW;
  const Bucket* list = ip_list(p, w, level);
  const uint32_t t = threadIdx.x, wave = t / 64, lane = lane_id();
  const uint32_t SLB = iw.slb;
  for (uint32_t r = blockIdx.x; r < nr; r += gridDim.x) {
    const uint32_t lb = r / IP_R;
    const Bucket Bk = list[iw.large[lb]];
    const uint32_t sf = iw.stripe_first[lb];
    const uint32_t f = iw.rf[r], e = iw.re[r];
    const uint32_t sa = f / SLB, sz = e > f ? (e - 1) / SLB + 1 : sa;  // stripes meeting [f, e)
    const uint32_t nsr = sz - sa;
    // full slots of the range
    uint32_t fr = 0;
    for (uint32_t j = sa + t; j < sz; j += IP_WG) {
      const uint32_t lo = max(j * SLB, f), hi = min(j * SLB + iw.nbfull[sf + j], e);
      fr += hi > lo ? hi - lo : 0u;
    }
    fr = wave_sum32(fr);
    if (t == 0) s_fr = 0;
    __syncthreads();
    if (lane == 0 && fr) atomicAdd(&s_fr, fr);
    __syncthreads();
    const uint32_t Fr = s_fr;
    const uint32_t cut = f + Fr;
    // free slots below the cut, full slots above it, per stripe
    for (uint32_t j = sa + t; j < sz; j += IP_WG) {
      const uint32_t full_end = j * SLB + iw.nbfull[sf + j];
      const uint32_t hl = max(full_end, f), hh = min((j + 1) * SLB, cut);
      const uint32_t ml = max(j * SLB, cut), mh = min(full_end, e);
      hpre[j - sa] = hh > hl ? hh - hl : 0u;
      mpre[j - sa] = mh > ml ? mh - ml : 0u;
    }
    __syncthreads();
    const uint32_t H = scan_lds(hpre, nsr, tmp16);
    const uint32_t Mv = scan_lds(mpre, nsr, tmp16);
    if (H != Mv && t == 0) atomicOr(&iw.ctl->error, 4u);
    const uint32_t moves = min(H, Mv);
    uint32_t* recw = reinterpret_cast<uint32_t*>(rec + Bk.begin * (uint64_t)(4 * RW));
    uint8_t* bd = iw.bdig + Bk.begin / B;  // digit of each full block slot of the bucket
    for (uint32_t k = wave; k < moves; k += IP_WAVES) {
      const uint32_t jh = last_le(hpre, nsr, k), jm = last_le(mpre, nsr, k);
      const uint32_t sh = sa + jh, sm = sa + jm;
      const uint32_t hslot = max(sh * SLB + iw.nbfull[sf + sh], f) + (k - hpre[jh]);
      const uint32_t mslot = max(sm * SLB, cut) + (k - mpre[jm]);
      if (hslot >= cut || mslot < cut || mslot >= e) {  // cannot happen: refuse rather than move
        if (lane == 0) atomicOr(&iw.ctl->error, 4u);
        continue;
      }
      const Blk x = blk_load(recw + (uint64_t)mslot * WB, WB, lane);
      blk_store(recw + (uint64_t)hslot * WB, x, WB, lane);
      if (lane == 0) bd[hslot] = bd[mslot];
    }
    __syncthreads();
    // Blocks already of this range's digit need not move: they are swapped
    // to the range's front [f, f + O), and the cursors start past them
    // (with skewed keys most of a heavy child's blocks are its own).  The
    // prefix's foreign blocks and the rest's own blocks (as many of each)
    // are collected in two LDS queues as the two parts are scanned, and
    // swapped in pairs.
    const uint32_t v = r - lb * IP_R;
    auto digit_at = [&](uint32_t sl) -> uint32_t { return bd[sl]; };
    uint32_t own = 0;
    for (uint32_t s0 = f; s0 < cut; s0 += 4 * IP_WG) {
      uint32_t d4[4];
#pragma unroll
      for (uint32_t h = 0; h < 4; h++) {
        const uint32_t sl = s0 + h * IP_WG + t;
        d4[h] = sl < cut ? digit_at(sl) : ~0u;
      }
#pragma unroll
      for (uint32_t h = 0; h < 4; h++) own += d4[h] == v ? 1u : 0u;
    }
    own = wave_sum32(own);
    if (t == 0) {
      s_h = 0;
      s_pa = f;
      s_na = s_nb = 0;
    }
    __syncthreads();
    if (lane == 0 && own) atomicAdd(&s_h, own);
    __syncthreads();
    const uint32_t O0 = s_h;
    const bool own_ok = O0 > 0 && O0 < Fr && Fr - O0 <= IP_OWN_SWAP_MAX;
    const uint32_t O = (own_ok || O0 == Fr) ? O0 : 0u;  // blocks that stay in place
    if (t == 0) s_pb = f + O;
    uint32_t* qa = hpre;  // foreign blocks in [f, f + O)
    uint32_t* qb = mpre;  // own blocks in [f + O, cut)
    for (;;) {
      __syncthreads();
      const uint32_t pa = s_pa, pb = s_pb, na = s_na, nb = s_nb;
      // all own or none: nothing to swap; more than IP_OWN_SWAP_MAX foreign
      // blocks (the pairs one workgroup would swap): left to the permutation
      if (!own_ok || (pa >= f + O && pb >= cut && na == 0 && nb == 0)) break;
      if (t == 0) { s_ca = 0; s_cb = 0; }
      __syncthreads();
      const bool fa = na < IP_WG && pa < f + O, fb = nb < IP_WG && pb < cut;
      if (fa && pa + t < f + O && digit_at(pa + t) != v) qa[na + atomicAdd(&s_ca, 1u)] = pa + t;
      if (fb && pb + t < cut && digit_at(pb + t) == v) qb[nb + atomicAdd(&s_cb, 1u)] = pb + t;
      __syncthreads();
      const uint32_t na2 = na + s_ca, nb2 = nb + s_cb, k = min(na2, nb2);
      for (uint32_t j = wave; j < k; j += IP_WAVES) {
        const uint32_t sa_ = qa[j], sb_ = qb[j];
        const Blk x = blk_load(recw + (uint64_t)sa_ * WB, WB, lane);
        const Blk y = blk_load(recw + (uint64_t)sb_ * WB, WB, lane);
        blk_store(recw + (uint64_t)sa_ * WB, y, WB, lane);
        blk_store(recw + (uint64_t)sb_ * WB, x, WB, lane);
      }
      // drop the swapped pairs from the queues' fronts
      uint32_t ka[2], kb[2];
#pragma unroll
      for (uint32_t h = 0; h < 2; h++) {
        const uint32_t j = k + t + h * IP_WG;
        ka[h] = j < na2 ? qa[j] : 0u;
        kb[h] = j < nb2 ? qb[j] : 0u;
      }
      __syncthreads();
#pragma unroll
      for (uint32_t h = 0; h < 2; h++) {
        const uint32_t j = k + t + h * IP_WG;
        if (j < na2) qa[j - k] = ka[h];
        if (j < nb2) qb[j - k] = kb[h];
      }
      if (t == 0) {
        s_na = na2 - k;
        s_nb = nb2 - k;
        if (fa) s_pa = min(pa + IP_WG, f + O);
        if (fb) s_pb = min(pb + IP_WG, cut);
      }
    }
    if (t == 0) {
      iw.W[(uint64_t)r * IP_WSTRIDE] = ((uint64_t)(f + O) << 32) | (uint64_t)(cut + IP_BIAS);
      iw.rinit[r] = cut;
      iw.chunk_start[r] = (Fr - O + IP_CHUNK - 1) / IP_CHUNK;
    }
    __syncthreads();
  }
}

// Chunk offsets of the ranges, and a step coprime to the chunk count that
// spreads consecutive claims over the ranges.
__global__ __launch_bounds__(IP_WG) void k_ip_chunks(IpWork iw) {
  __shared__ uint32_t tmp16[IP_WAVES];
  __shared__ uint32_t run;
  const uint32_t nr = iw.ctl->nranges;
  const uint32_t t = threadIdx.x;
  if (t == 0) run = 0;
  __syncthreads();
  for (uint32_t c0 = 0; c0 < nr; c0 += 16 * IP_WG) {
    const uint32_t cnt = min(nr - c0, 16u * IP_WG);
    const uint32_t tot = scan_lds(iw.chunk_start + c0, cnt, tmp16);
    const uint32_t r0 = run;
    for (uint32_t i = t; i < cnt; i += IP_WG) iw.chunk_start[c0 + i] += r0;
    __syncthreads();
    if (t == 0) run = r0 + tot;
    __syncthreads();
  }
  if (t == 0) {
    const uint32_t n = run;
    iw.chunk_start[nr] = n;
    iw.ctl->nchunks = n;
    uint32_t s = n > 2 ? (uint32_t)((uint64_t)n * 5 / 8) | 1u : 1u;
    for (;; s++) {
      uint32_t a = s, b = n ? n : 1;
      while (b) { const uint32_t q = a % b; a = b; b = q; }
      if (a == 1) break;
    }
    iw.ctl->stride = s;
  }
}

// Permutation of the large buckets' blocks.  A wavefront runs IP_CHAINS
// chains at once, each carrying one block (the steps of ip_drain_multi): per
// round every chain issues its cursor claim -- a read claim on the wave's
// current range if it holds no block, a write claim on its block's digit
// otherwise -- then the block loads the claims call for, so that the
// latencies of the chains overlap.  Read bits are set before any chain of
// the round waits on one (a chain may wait on a slot that another chain of
// the same wave has just read).
constexpr uint32_t IP_CHAINS = 4;
static_assert(IP_CHAINS <= 32, "the slots of one read claim span at most two bit words");

template <int RW>
__global__ __launch_bounds__(IP_PERM_WG) void k_ip_permute(Plan p, Work w, IpWork iw, uint32_t level, uint8_t* rec) {
  const uint32_t nch = iw.ctl->nchunks, stride = iw.ctl->stride, nr = iw.ctl->nranges;
  const KeyFmt kf = make_keyfmt(p.key_bytes);
  const uint32_t B = ip_block_records(RW), WB = B * RW;
  const Bucket* list = ip_list(p, w, level);
  const uint32_t lane = lane_id();
  constexpr uint32_t NC = IP_CHAINS;
  constexpr uint64_t RB = 4 * RW;
  // the wave's current chunk: range ri of large bucket rlb (first record
  // rP, rcount records, digit rg), `quota` reads left
  uint32_t quota = 0, rlb = 0, ri = 0;
  uint64_t rP = 0, rcount = 0;
  Dig rg{0u, 0u};
  bool more = true;
  // chains: block x of digit v of large bucket lb; slot of this round; end
  // of the block's child
  Blk x[NC], y[NC];
  uint32_t v[NC], lbc[NC], slot[NC], mode[NC];
  uint64_t lim[NC];
  bool has[NC];
#pragma unroll
  for (uint32_t c = 0; c < NC; c++) {
    has[c] = false;
    v[c] = lbc[c] = slot[c] = mode[c] = 0;
    lim[c] = 0;
    x[c] = y[c] = Blk{0u, 0u};
  }
  enum : uint32_t { NONE = 0, READ = 1, SWAP = 2, PLACE = 3 };
  for (;;) {
    bool need = false, busy = false;
#pragma unroll
    for (uint32_t c = 0; c < NC; c++) {
      need = need || !has[c];
      busy = busy || has[c];
    }
    if (need && quota == 0 && more) {
      uint32_t t = 0;
      if (lane == 0) t = atomicAdd(&iw.ctl->chunk_ticket, 1u);
      t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
      if (t >= nch) {
        more = false;
      } else {
        const uint32_t cp = (uint32_t)(((uint64_t)t * stride) % nch);
        const uint32_t r = last_le(iw.chunk_start, nr, cp);
        rlb = r / IP_R;
        ri = r - rlb * IP_R;
        quota = IP_CHUNK;
        const Bucket Bk = list[iw.large[rlb]];
        rP = Bk.begin;
        rcount = Bk.count;
        rg = bucket_digit(p, kf, Bk.bit);
      }
    }
    if (!busy && quota == 0 && !more) break;
    // claims: the chains without a block share one read claim of up to
    // their number of slots; the others claim a write slot each
    uint32_t nneed = 0;
#pragma unroll
    for (uint32_t c = 0; c < NC; c++) nneed += has[c] ? 0u : 1u;
    nneed = min(nneed, quota);
    uint64_t rold = 0;
    if (nneed && lane == 0)
      rold = atomicAdd((unsigned long long*)&iw.W[((uint64_t)rlb * IP_R + ri) * IP_WSTRIDE], 0ull - nneed);
    uint64_t old[NC];
#pragma unroll
    for (uint32_t c = 0; c < NC; c++) {
      old[c] = 0;
      mode[c] = NONE;
      if (has[c]) {
        mode[c] = SWAP;
        if (lane == 0)
          old[c] = atomicAdd((unsigned long long*)&iw.W[((uint64_t)lbc[c] * IP_R + v[c]) * IP_WSTRIDE], 1ull << 32);
      }
    }
    // read slots rc - 1, rc - 2, ... down to the write cursor
    uint32_t rfirst = 0, ngot = 0;
    if (nneed) {
      quota -= nneed;
      const uint64_t o = bcast64(__shfl((unsigned long long)rold, 0));
      const int64_t wc = (int64_t)(o >> 32), rc = (int64_t)(uint32_t)o - (int64_t)IP_BIAS;
      const int64_t avail = rc - wc;
      ngot = avail <= 0 ? 0u : (uint32_t)min<int64_t>(avail, nneed);
      if (ngot < nneed) quota = 0;  // range exhausted: the rest of the chunk is void
      rfirst = (uint32_t)(rc - (int64_t)ngot);  // lowest slot read
      if (ngot && (uint64_t)rc > (rcount + B - 1) / B) {  // cannot happen
        if (lane == 0) atomicOr(&iw.ctl->error, 4u);
        ngot = 0;
        quota = 0;
      }
    }
    // decode, loads
    uint32_t k = 0;
#pragma unroll
    for (uint32_t c = 0; c < NC; c++) {
      if (!has[c] && k < ngot) {
        mode[c] = READ;
        lbc[c] = rlb;
        slot[c] = rfirst + k;
        x[c] = blk_load(reinterpret_cast<const uint32_t*>(rec + rP * RB) + (uint64_t)slot[c] * WB, WB, lane);
        k++;
      }
      if (mode[c] != SWAP) continue;
      // (a write cursor past its child's blocks cannot happen; the cleanup
      // checks every final cursor, and a slot past the bucket is refused)
      const uint64_t o = bcast64(__shfl((unsigned long long)old[c], 0));
      const int64_t rc = (int64_t)(uint32_t)o - (int64_t)IP_BIAS;
      const uint32_t ws = (uint32_t)(o >> 32);
      const Bucket Bk = list[iw.large[lbc[c]]];
      if (ws >= (Bk.count + B - 1) / B) {
        if (lane == 0) atomicOr(&iw.ctl->error, 4u);
        mode[c] = NONE;
        has[c] = false;
        continue;
      }
      slot[c] = ws;
      lim[c] = uniform64(iw.rlim[(uint64_t)lbc[c] * IP_R + v[c]]);
      if ((int64_t)ws < rc) y[c] = blk_load(reinterpret_cast<const uint32_t*>(rec + Bk.begin * RB) + (uint64_t)ws * WB, WB, lane);
      else mode[c] = PLACE;
    }
    wait_loads();
    // read bits first (the slots read are consecutive: at most two words)
    if (ngot && lane == 0) {
      const uint64_t b0 = rP / B + rfirst, b1 = b0 + ngot - 1;
      const uint32_t lo = (uint32_t)(b0 & 31), hi = (uint32_t)(b1 & 31);
      if ((b0 >> 5) == (b1 >> 5)) {
        atomicOr(&iw.done[b0 >> 5], (0xFFFFFFFFu >> (31 - hi)) & (0xFFFFFFFFu << lo));
      } else {
        atomicOr(&iw.done[b0 >> 5], 0xFFFFFFFFu << lo);
        atomicOr(&iw.done[b1 >> 5], 0xFFFFFFFFu >> (31 - hi));
      }
    }
#pragma unroll
    for (uint32_t c = 0; c < NC; c++) {
      if (mode[c] != READ) continue;
      v[c] = blk_digit<RW>(x[c], kf, rg);
      has[c] = true;
    }
    // then the writes
#pragma unroll
    for (uint32_t c = 0; c < NC; c++) {
      if (mode[c] != SWAP && mode[c] != PLACE) continue;
      const uint64_t ro = (uint64_t)lbc[c] * IP_R + v[c];
      const Bucket Bk = list[iw.large[lbc[c]]];
      uint32_t* recw = reinterpret_cast<uint32_t*>(rec + Bk.begin * RB);
      uint32_t* protw = reinterpret_cast<uint32_t*>(iw.prot + ro * IP_BLOCK_BYTES);
      const uint32_t ws = slot[c];
      if (mode[c] == PLACE && ws < iw.rinit[ro]) {
        // the slot's block was claimed by a reader: wait until it has it
        const uint64_t bi = Bk.begin / B + ws;
        uint32_t spins = 0;
        for (;;) {
          uint32_t word = 0;
          if (lane == 0) word = __hip_atomic_load(&iw.done[bi >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          word = __builtin_amdgcn_readfirstlane(__shfl(word, 0));
          if ((word >> (bi & 31)) & 1u) break;
          if (++spins > p.spin_limit) {
            if (lane == 0) atomicOr(&iw.ctl->error, 2u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      put_block<RW>(x[c], recw, Bk.count, ws, B, lim[c], protw, lane);
      if (mode[c] == SWAP) {
        x[c] = y[c];
        v[c] = blk_digit<RW>(y[c], kf, bucket_digit(p, kf, Bk.bit));
      } else {
        has[c] = false;
      }
    }
  }
}

// Edges of each child of a large bucket: its leftovers from every stripe,
// then the part of its last block past its end.
template <int RW>
__global__ __launch_bounds__(IP_WG) void k_ip_cleanup(Plan p, Work w, IpWork iw, uint32_t level, uint8_t* rec) {
  __shared__ uint32_t pre[IP_MAX_STRIPES + 1];
  __shared__ uint32_t tmp16[IP_WAVES];
  const uint32_t nr = iw.ctl->nranges;
  const uint32_t B = ip_block_records(RW);
  const Bucket* list = ip_list(p, w, level);
  const uint32_t t = threadIdx.x;
  for (uint32_t r = blockIdx.x; r < nr; r += gridDim.x) {
    const uint32_t lb = r / IP_R, v = r - lb * IP_R;
    const Bucket Bk = list[iw.large[lb]];
    const uint32_t sf = iw.stripe_first[lb], sn = iw.stripe_first[lb + 1] - sf;
    for (uint32_t j = t; j < sn; j += IP_WG) pre[j] = iw.lcnt[(uint64_t)(sf + j) * IP_R + v];
    __syncthreads();
    const uint32_t L = scan_lds(pre, sn, tmp16);
    const uint64_t b0 = iw.rbase[r], lim = iw.rlim[r];
    const uint32_t f = iw.rf[r], F = iw.rF[r];
    const uint64_t E = (uint64_t)(f + F) * B;
    const uint64_t head_end = F ? min((uint64_t)f * B, lim) : lim;
    const uint64_t tail0 = F ? min(E, lim) : lim;
    const uint64_t nh = (head_end - b0) + (lim - tail0);
    const uint64_t pc = F && E > lim ? E - lim : 0;
    // every block of the child was written: its write cursor ends at f + F
    if (t == 0 && (nh != L + pc || (uint32_t)(iw.W[(uint64_t)r * IP_WSTRIDE] >> 32) != f + F))
      atomicOr(&iw.ctl->error, 4u);
    const uint8_t* pr = iw.prot + (uint64_t)r * IP_BLOCK_BYTES;
    for (uint64_t k = t; k < nh; k += IP_WG) {
      const uint64_t dst = k < head_end - b0 ? b0 + k : tail0 + (k - (head_end - b0));
      Rec<RW> x;
      if (k < L) {
        const uint32_t j = last_le(pre, sn, (uint32_t)k);
        x = load_rec<RW>(iw.side + ((uint64_t)(sf + j) * IP_R + v) * IP_BLOCK_BYTES, k - pre[j]);
      } else {
        x = load_rec<RW>(pr, k - L);
      }
      store_rec<RW>(rec, Bk.begin + dst, x, false);
    }
    __syncthreads();
  }
}

}  // namespace

// ---- launchers -------------------------------------------------------------------

// set-up and classification of the stripes of the large buckets
void launch_ip_classify(const Plan& p, const Work& w, const IpWork& iw, uint32_t level, void* records, int cus,
                        hipStream_t s) {
  uint8_t* rec = (uint8_t*)records;
  const size_t lds = (size_t)IP_R * IP_BLOCK_BYTES;
  k_ip_setup<<<1, IP_WG, 0, s>>>(p, w, iw, level);
  switch (p.rw) {
#define RD_CASE(n) case n: k_ip_classify<n><<<cus, IP_WG, lds, s>>>(p, w, iw, level, rec); break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

// the buckets one workgroup partitions from start to end
void launch_ip_medium(const Plan& p, const Work& w, const IpWork& iw, uint32_t level, void* records, hipStream_t s) {
  uint8_t* rec = (uint8_t*)records;
  const size_t lds = (size_t)IP_R * IP_BLOCK_BYTES;
  switch (p.rw) {
#define RD_CASE(n) case n: k_ip_medium<n><<<iw.grid_medium, IP_WG, lds, s>>>(p, w, iw, level, rec); break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

// children of the large buckets, routing, child ranges, permutation chunks
void launch_ip_prepare(const Plan& p, const Work& w, const IpWork& iw, uint32_t level, void* records, int cus,
                       hipStream_t s) {
  uint8_t* rec = (uint8_t*)records;
  k_ip_bucket<<<cus, IP_WG, 0, s>>>(p, w, iw, level);
  launch_level_scan(p, w, level, s);
  switch (p.rw) {
#define RD_CASE(n) case n: k_ip_ranges<n><<<2 * cus, IP_WG, 0, s>>>(p, w, iw, level, rec); break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
  k_ip_chunks<<<1, IP_WG, 0, s>>>(iw);
  launch_zero(iw.done, (size_t)((iw.done_words + 1) / 2) * 8, s);
}

void launch_ip_permute(const Plan& p, const Work& w, const IpWork& iw, uint32_t level, void* records, int cus,
                       hipStream_t s) {
  uint8_t* rec = (uint8_t*)records;
  switch (p.rw) {
#define RD_CASE(n) case n: k_ip_permute<n><<<8 * cus, IP_PERM_WG, 0, s>>>(p, w, iw, level, rec); break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

void launch_ip_cleanup(const Plan& p, const Work& w, const IpWork& iw, uint32_t level, void* records, int cus,
                       hipStream_t s) {
  uint8_t* rec = (uint8_t*)records;
  switch (p.rw) {
#define RD_CASE(n) case n: k_ip_cleanup<n><<<4 * cus, IP_WG, 0, s>>>(p, w, iw, level, rec); break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

}  // namespace rd
