// k_search.hip -- batched pattern-prefix search over a suffix array.
//
// The paper's second application (Sec. 5): many patterns are looked up in a
// suffix array (the text's suffixes in lexicographic order).  Searched one
// by one, each pattern costs a binary search over the whole array; with the
// patterns (or their prefixes) sorted first, each search runs in a range
// narrowed by its neighbours' results.
//
// Here a query is a record whose key (k = key_bytes <= 16 bytes) holds the
// pattern's first k characters reversed, so the key, read as a little-endian
// integer, is the big-endian integer of the k characters: key order is the
// string order, and comparing a query with a suffix is comparing that key
// with the big-endian integer of the suffix's first k characters (zero past
// the end of the text; text characters are non-zero).  For each query,
// lo = the number of suffixes whose k-prefix is below it and hi = the number
// at or below it, so sa[lo, hi) are the suffixes that start with it.
//
// One workgroup takes 256 consecutive queries, one per thread.  If they are
// in ascending order (checked per tile) every one of them lies in
// [lower bound of the first, upper bound of the last), which one wavefront
// finds by a 64-way search (each lane probes one position per round);
// every thread then binary-searches its own query inside that range only.
// Tiles out of order, or all tiles when narrowing is switched off, search
// the whole array.
#include "raduls_dev.hpp"
#include "raduls_kernels.hpp"

namespace rd {

namespace {

struct U128 {
  uint64_t lo, hi;
};

__device__ __forceinline__ bool u128_less(U128 a, U128 b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }

// Big-endian integer of text[i, i + k), zero past the end of the text.
__device__ __forceinline__ U128 suffix_prefix(const uint8_t* __restrict__ text, uint64_t N, uint64_t i, uint32_t k) {
  U128 v{0, 0};
  for (uint32_t j = 0; j < k; j++) {
    const uint64_t c = i + j < N ? (uint64_t)text[i + j] : 0ull;
    const uint32_t s = 8 * (k - 1 - j);  // bit position of character j
    if (s >= 64) v.hi |= c << (s - 64);
    else v.lo |= c << s;
  }
  return v;
}

// Does the suffix at rank m come before the query (below it, or, for an
// upper bound, at or below it)?
__device__ __forceinline__ bool before(const uint8_t* text, uint64_t N, const uint32_t* sa, uint64_t m, uint32_t k,
                                       U128 q, bool upper) {
  const U128 p = suffix_prefix(text, N, sa[m], k);
  return upper ? !u128_less(q, p) : u128_less(p, q);
}

// First rank in [L, R) whose suffix does not come before the query (R if
// none), by bisection.
__device__ __forceinline__ uint64_t bisect(const uint8_t* text, uint64_t N, const uint32_t* sa, uint64_t L, uint64_t R,
                                           uint32_t k, U128 q, bool upper) {
  while (L < R) {
    const uint64_t m = L + (R - L) / 2;
    if (before(text, N, sa, m, k, q, upper)) L = m + 1;
    else R = m;
  }
  return L;
}

// The same by one wavefront (every lane has the same query): each round,
// lane l probes the end of the l-th of 64 equal parts of [L, R); the parts
// wholly before the query are skipped.
__device__ __forceinline__ uint64_t bisect_wave(const uint8_t* text, uint64_t N, const uint32_t* sa, uint64_t L,
                                                uint64_t R, uint32_t k, U128 q, bool upper) {
  const uint32_t lane = lane_id();
  while (R - L > 64) {
    const uint64_t len = R - L;
    const uint64_t p = L + (len * (lane + 1)) / 65;  // probes strictly inside [L, R), increasing with the lane
    const uint64_t bm = __ballot(before(text, N, sa, p, k, q, upper));
    const uint32_t c = (uint32_t)__popcll(bm);     // probes before the query: lanes 0 .. c-1
    const uint64_t nL = c ? L + (len * c) / 65 + 1 : L;
    const uint64_t nR = c < 64 ? L + (len * (c + 1)) / 65 : R;
    L = nL;
    R = nR > nL ? nR : nL;
  }
  // at most 64 ranks left: one probe each
  const uint64_t p = L + lane;
  const bool b = p < R && before(text, N, sa, p, k, q, upper);
  return L + (uint64_t)__popcll(__ballot(b));
}

template <int RW>
__global__ __launch_bounds__(WG) void k_prefix_search(const uint8_t* __restrict__ text, uint64_t N,
                                                      const uint32_t* __restrict__ sa,
                                                      const uint8_t* __restrict__ queries, uint64_t nq, KeyFmt kf,
                                                      uint32_t k, uint64_t* __restrict__ lo_out,
                                                      uint64_t* __restrict__ hi_out, uint32_t narrow) {
  __shared__ uint64_t s_q[2 * WG];
  __shared__ uint32_t s_unsorted;
  __shared__ uint64_t s_L, s_R;
  const uint32_t t = threadIdx.x;
  const uint64_t i = (uint64_t)blockIdx.x * WG + t;
  const uint64_t last = min(nq, (uint64_t)(blockIdx.x + 1) * WG) - 1;  // last query of the tile
  const bool valid = i < nq;
  U128 q{0, 0};
  if (valid) {
    const Key key = load_key<RW>(queries, i, kf);
    q = U128{key.lo, key.hi};
  }
  uint64_t L = 0, R = N;
  if (narrow) {
    if (t == 0) s_unsorted = 0;
    s_q[2 * t] = q.lo;
    s_q[2 * t + 1] = q.hi;
    __syncthreads();
    if (valid && t > 0 && u128_less(q, U128{s_q[2 * t - 2], s_q[2 * t - 1]})) s_unsorted = 1;
    __syncthreads();
    if (!s_unsorted) {
      if (t < 64) {
        const uint32_t tl = (uint32_t)(last - (uint64_t)blockIdx.x * WG);
        const U128 qf{s_q[0], s_q[1]}, ql{s_q[2 * tl], s_q[2 * tl + 1]};
        const uint64_t a = bisect_wave(text, N, sa, 0, N, k, qf, false);
        const uint64_t b = bisect_wave(text, N, sa, a, N, k, ql, true);
        if (t == 0) { s_L = a; s_R = b; }
      }
      __syncthreads();
      L = s_L;
      R = s_R;
    }
  }
  if (!valid) return;
  const uint64_t lo = bisect(text, N, sa, L, R, k, q, false);
  const uint64_t hi = bisect(text, N, sa, lo, R, k, q, true);
  lo_out[i] = lo;
  hi_out[i] = hi;
}

}  // namespace

void launch_prefix_search(const void* text, uint64_t N, const uint32_t* sa, const void* queries, uint64_t nq,
                          uint32_t rec_bytes, uint32_t key_bytes, uint64_t* lo, uint64_t* hi, uint32_t narrow,
                          hipStream_t s) {
  if (nq == 0) return;
  const KeyFmt kf = make_keyfmt(key_bytes);
  const uint32_t grid = (uint32_t)((nq + WG - 1) / WG);
  const uint8_t* tx = (const uint8_t*)text;
  const uint8_t* qr = (const uint8_t*)queries;
  switch (rec_bytes / 4) {
#define RD_CASE(m)                                                                                       \
  case m:                                                                                                \
    k_prefix_search<m><<<grid, WG, 0, s>>>(tx, N, sa, qr, nq, kf, key_bytes, lo, hi, narrow);            \
    break;
    RD_CASE(1) RD_CASE(2) RD_CASE(3) RD_CASE(4) RD_CASE(5) RD_CASE(6) RD_CASE(7) RD_CASE(8)
    RD_CASE(9) RD_CASE(10) RD_CASE(11) RD_CASE(12) RD_CASE(13) RD_CASE(14) RD_CASE(15) RD_CASE(16)
#undef RD_CASE
    default: break;
  }
}

}  // namespace rd
