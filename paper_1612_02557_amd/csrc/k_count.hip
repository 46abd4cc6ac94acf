// k_count.hip -- duplicate removal with counts over key-ordered records.
//
// The k-mer counting application of the paper (Sec. 5) sorts the k-mers of
// a bin and then removes duplicates; here the second step is one pass over
// the sorted records.  A record starts a run when its key differs from the
// previous record's; run j's first record goes to uniq[j] and its length to
// counts[j].
//
// One workgroup takes one tile of records (tile ids from an atomic ticket,
// so every tile's predecessors are running or done).  Per tile: the head
// flags (ballots per wavefront row), the number of heads h and the index of
// its last head; the heads before the tile (H) and the last head before it
// (P) come from a decoupled look-back over the tiles' (h, last head) pairs,
// combined as (H1 + H2, last2 if the second part has a head, else last1),
// one wavefront reading 64 earlier tiles' words at a time.
// Each head then writes its record to uniq[H + rank] and the length of the
// run before it (its index minus the previous head's), so every count is
// written exactly once, by a plain store; the tile holding the last record
// also writes the last run's length and the number of runs.
//
// uniq may be the input itself: a tile writes only below its own heads'
// indices, and only after every earlier tile has published, i.e. has
// finished reading its records.
#include "raduls_dev.hpp"
#include "raduls_kernels.hpp"

namespace rd {

namespace {

// Look-back words, four per tile: the tile's own (heads, last head + 1) and
// the inclusive pair of this and all earlier tiles.  Every word carries its
// own ready bit (the top bit), so a pair is read as ready when both of its
// words are, and the words are plain relaxed device-scope atomics: no cache
// write-back or invalidation between the XCDs' L2s is needed.  A tile that
// gave up on its wait publishes a poisoned inclusive pair, and tiles after
// it give up at once.
constexpr uint64_t RL_READY = 1ull << 63;
constexpr uint64_t RL_POISON = 1ull << 62;
constexpr uint64_t RL_VAL = RL_POISON - 1;

// records per thread of a tile: up to 64 words of records in registers
__host__ __device__ constexpr uint32_t runs_rows(uint32_t rw) { return rw <= 4 ? 16u : (64u / rw >= 2 ? 64u / rw : 2u); }
template <int RW>
constexpr uint32_t runs_per_thread() {
  return runs_rows(RW);
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}


template <int RW>
__global__ __launch_bounds__(WG) void k_runs(const uint8_t* src, uint64_t n, KeyFmt kf,
                                             uint8_t* uniq, uint64_t* __restrict__ counts,
                                             uint64_t* __restrict__ num_runs, RunCtl* __restrict__ ctl,
                                             uint64_t* __restrict__ st, uint32_t spin_limit) {
  constexpr uint32_t E = runs_per_thread<RW>();
  constexpr uint32_t T = E * WG;
  constexpr uint32_t NS = E * NWAVES;  // segments: (row, wavefront) in record order
  static_assert(NS <= 64, "one wavefront scans the segments");
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_cnt[NS];    // heads of each segment, then the heads before it in the tile
  __shared__ uint64_t s_last[NS];   // last head of each segment + 1, then of the segments before it
  __shared__ uint64_t s_H, s_P;     // heads before the tile, last head before it + 1
  __shared__ uint32_t s_ok;

  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
  if (tid == 0) s_tile = atomicAdd(&ctl->ticket, 1u);
  __syncthreads();
  const uint64_t tile = s_tile;
  const uint64_t base = tile * T;

  Rec<RW> rec[E];
  uint64_t hb[E];  // ballot of head flags of each row
#pragma unroll
  for (uint32_t e = 0; e < E; e++) {
    const uint64_t i = base + e * WG + tid;
    const bool valid = i < n;
    if (valid) rec[e] = load_rec<RW>(src, i);
    else {
#pragma unroll
      for (int q = 0; q < RW; q++) rec[e].w[q] = 0;
    }
  }
#pragma unroll
  for (uint32_t e = 0; e < E; e++) {
    const uint64_t i = base + e * WG + tid;
    const bool valid = i < n;
    const Key k = rec_key(rec[e], kf);
    // previous record's key: the lane below, or a load for lane 0
    Key pk;
    pk.lo = __shfl_up(k.lo, 1);
    pk.hi = __shfl_up(k.hi, 1);
    if (lane == 0 && valid && i > 0) pk = load_key<RW>(src, i - 1, kf);
    const bool head = valid && (i == 0 || ((k.lo ^ pk.lo) | (k.hi ^ pk.hi)) != 0);
    hb[e] = __ballot(head);
    if (lane == 0) {
      const uint32_t s = e * NWAVES + wave;
      s_cnt[s] = (uint32_t)__popcll(hb[e]);
      s_last[s] = hb[e] ? base + e * WG + wave * 64 + (63 - __clzll(hb[e])) + 1 : 0ull;
    }
  }
  // every load of the tile has returned before the tile publishes (uniq may
  // be the input: later tiles write below their heads only after that)
#pragma unroll
  for (uint32_t e = 0; e < E; e++) {
#pragma unroll
    for (int q = 0; q < RW; q++) asm volatile("" : : "v"(rec[e].w[q]));
  }
  __syncthreads();

  if (wave == 0) {
    // heads before each segment (exclusive sum) and the last head before it
    // (exclusive max: head indices grow with the segment order)
    const uint32_t c = lane < NS ? s_cnt[lane] : 0u;
    const uint64_t l = lane < NS ? s_last[lane] : 0ull;
    uint32_t tot;
    const uint32_t ex = wave_excl_scan(c, &tot);
    uint64_t mx = l;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t y = __shfl_up(mx, o);
      if (lane >= (uint32_t)o) mx = y > mx ? y : mx;
    }
    const uint64_t lp = __shfl(mx, 63);  // last head of the tile + 1 (0: none)
    uint64_t exl = __shfl_up(mx, 1);
    if (lane == 0) exl = 0;
    if (lane < NS) { s_cnt[lane] = ex; s_last[lane] = exl; }

    const uint64_t h = tot;
    uint64_t* my = st + 4 * tile;
    uint64_t H = 0, P = 0;
    bool ok = true;
    if (tile == 0) {
      if (lane == 0) {
        atomic_store_agent(&my[3], RL_READY | lp);
        atomic_store_agent(&my[2], RL_READY | h);
      }
    } else {
      if (lane == 0) {
        atomic_store_agent(&my[1], RL_READY | lp);
        atomic_store_agent(&my[0], RL_READY | h);
      }
      // look back over a window of 64 earlier tiles at once (lane L reads
      // tile j0 - L): the nearest tile with an inclusive word ends the walk
      // when every tile between it and this one has published its own pair
      uint64_t j0 = tile - 1;
      uint32_t spins = 0;
      bool done = false;
      while (!done) {
        // bounded wait: past the limit the tile gives up, flags the error
        // and poisons its inclusive word so that the tiles after it stop too
        if (spins >= spin_limit) { ok = false; break; }
        const bool exists = j0 >= (uint64_t)lane;
        const uint64_t j = exists ? j0 - lane : 0;
        // before tile 0: an empty inclusive prefix
        uint64_t w = exists ? atomic_load_agent(&st[4 * j + 2]) : RL_READY;
        uint64_t pw = exists ? atomic_load_agent(&st[4 * j + 3]) : RL_READY;
        const bool inc = (w & pw & RL_READY) != 0;
        if (!inc) {
          w = atomic_load_agent(&st[4 * j + 0]);
          pw = atomic_load_agent(&st[4 * j + 1]);
        }
        const bool ready = (w & pw & RL_READY) != 0;
        pw &= RL_VAL;
        const uint64_t incm = __ballot(inc);
        const uint64_t waiting = __ballot(!ready);
        const uint32_t first = incm ? (uint32_t)(__ffsll((long long)incm) - 1) : 64u;
        const uint64_t below = first >= 63 ? ~0ull : ((2ull << first) - 1);  // lanes 0..first
        if (waiting & below) {  // a tile before the nearest inclusive one is not ready
          ++spins;
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        if (first < 64 && __shfl(w, (int)first) & RL_POISON) { ok = false; break; }
        const bool use = lane <= first;
        H += wave_sum64(use ? (w & RL_VAL) : 0ull);
        if (!P) {
          const uint64_t pm = __ballot(use && pw != 0);
          if (pm) P = __shfl(pw, (int)(__ffsll((long long)pm) - 1));
        }
        done = first < 64;
        j0 -= 64;
      }
      if (lane == 0) {
        if (ok) {
          atomic_store_agent(&my[3], RL_READY | (lp ? lp : P));
          atomic_store_agent(&my[2], RL_READY | (H + h));
        } else {
          atomicOr(&ctl->error, 1u);
          atomic_store_agent(&my[3], RL_READY);
          atomic_store_agent(&my[2], RL_READY | RL_POISON);
        }
      }
    }
    if (lane == 0) {
      s_H = H;
      s_P = P;
      s_ok = ok ? 1u : 0u;
      if (ok && base + T >= n) {
        // the tile of the last record: the last run and the number of runs
        const uint64_t U = H + h;
        const uint64_t start = (lp ? lp : P) - 1;
        counts[U - 1] = n - start;
        *num_runs = U;
      }
    }
  }
  __syncthreads();
  if (!s_ok) return;
  const uint64_t H = s_H, P = s_P;
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (uint32_t e = 0; e < E; e++) {
    if (!((hb[e] >> lane) & 1ull)) continue;
    const uint32_t s = e * NWAVES + wave;
    const uint64_t i = base + e * WG + tid;
    const uint64_t j = H + s_cnt[s] + (uint64_t)__popcll(hb[e] & lt);
    store_rec<RW>(uniq, j, rec[e], false);
    if (j == 0) continue;  // the first record: no run before it
    const uint64_t below = hb[e] & lt;
    uint64_t prev;
    if (below) prev = base + e * WG + wave * 64 + (63 - __clzll(below));
    else if (s_last[s]) prev = s_last[s] - 1;
    else prev = P - 1;
    counts[j - 1] = i - prev;
  }
}

}  // namespace

uint64_t runs_tiles(uint64_t n, uint32_t rec_bytes) {
  const uint64_t T = (uint64_t)runs_rows(rec_bytes / 4) * WG;
  return (n + T - 1) / T;
}

size_t runs_workspace_bytes(uint64_t n, uint32_t rec_bytes) { return 256 + (size_t)(runs_tiles(n, rec_bytes) + 1) * 32; }

void launch_runs(const void* src, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, void* uniq, uint64_t* counts,
                 uint64_t* num_runs, void* ws, uint32_t spin_limit, hipStream_t s) {
  if (n == 0) {
    launch_zero(num_runs, 8, s);
    return;
  }
  launch_zero(ws, runs_workspace_bytes(n, rec_bytes), s);
  RunCtl* ctl = (RunCtl*)ws;
  uint64_t* st = (uint64_t*)((uint8_t*)ws + 256);
  const KeyFmt kf = make_keyfmt(key_bytes);
  const uint8_t* in = (const uint8_t*)src;
  uint8_t* out = (uint8_t*)uniq;
  switch (rec_bytes / 4) {
#define RD_CASE(m)                                                                                          \
  case m: {                                                                                                 \
    const uint32_t grid = (uint32_t)runs_tiles(n, rec_bytes);                                               \
    k_runs<m><<<grid, WG, 0, s>>>(in, n, kf, out, counts, num_runs, ctl, st, spin_limit);                   \
    break;                                                                                                  \
  }
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

}  // namespace rd
