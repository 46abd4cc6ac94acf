/*
 * oracle_sort.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU reference for what the GPU sorter
 * computes.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file's library; the product path never does.
 * It shares no code, header, helper or table with the GPU library.
 *
 * Record model (paper, Sec. 1 and the experiments of Sec. 4: a record is a
 * key followed by data, e.g. 8-byte key + 8-byte data):
 *   a record is rec_bytes bytes; its key is bytes [0, key_bytes) read as an
 *   unsigned little-endian integer (byte key_bytes-1 most significant); bytes
 *   [key_bytes, rec_bytes) are payload and travel with the key unchanged.
 *
 * Result: the records permuted into ascending key order, STABLY (records with
 * equal keys keep their input order).  The paper's finishing sorts are not
 * stable, so several outputs would be valid there; this reference pins the
 * stable one, which is unique.
 *
 * Method (paper, Sec. 1): least-significant-digit radix sort with radix
 * R = 256 (one byte per digit, Sec. 3.1), each pass a stable counting sort
 * made of two traversals: the first counts how often each digit value
 * occurs, then the number of keys with a smaller digit gives each value's
 * first output slot, and the second traversal moves every record to the
 * next free slot of its digit value.  Stability of each pass is what makes
 * the LSD order correct.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- one stable counting pass on key byte `b` (Sec. 1) ----------------- */
static void counting_pass_byte(const uint8_t* src, uint8_t* dst, uint64_t n,
                               uint32_t r, uint32_t b) {
  uint64_t count[256];
  uint64_t next[256];
  memset(count, 0, sizeof count);
  /* traversal 1: histogram of digit values */
  for (uint64_t i = 0; i < n; i++) count[src[i * r + b]] += 1;
  /* number of keys whose digit is smaller = first slot of each value */
  uint64_t run = 0;
  for (int v = 0; v < 256; v++) { next[v] = run; run += count[v]; }
  /* traversal 2: distribute, in input order (stable) */
  for (uint64_t i = 0; i < n; i++) {
    uint32_t v = src[i * r + b];
    memcpy(dst + next[v] * r, src + i * r, r);
    next[v] += 1;
  }
}

/*
 * oracle_sort: sort n records of r bytes in place by their k-byte key,
 * ascending, stable.  Returns 0, or -1 if scratch memory is unavailable or
 * the arguments are inconsistent (k == 0 or k > r).
 */
int oracle_sort(uint8_t* rec, uint64_t n, uint32_t r, uint32_t k) {
  if (k == 0 || k > r) return -1;
  if (n < 2) return 0;
  uint8_t* tmp = (uint8_t*)malloc(n * r);
  if (!tmp) return -1;
  uint8_t* src = rec;
  uint8_t* dst = tmp;
  for (uint32_t b = 0; b < k; b++) {   /* least significant byte first */
    counting_pass_byte(src, dst, n, r, b);
    uint8_t* t = src; src = dst; dst = t;
  }
  if (src != rec) memcpy(rec, src, n * r);
  free(tmp);
  return 0;
}

/* ---- the T-thread variant (same output) ---------------------------------
 * Each thread counts digit values over its own contiguous chunk; thread t's
 * first slot for value v is (all records with a smaller value) + (records
 * with value v in the chunks of threads before t).  Chunks are distributed in
 * input order, so the pass stays stable and the output is identical to the
 * single-thread pass.
 */
typedef struct {
  const uint8_t* src;
  uint8_t* dst;
  uint64_t lo, hi;
  uint32_t r, b;
  uint64_t count[256];
  uint64_t next[256];
  int phase;
} chunk_job;

static void* chunk_worker(void* arg) {
  chunk_job* j = (chunk_job*)arg;
  if (j->phase == 0) {
    memset(j->count, 0, sizeof j->count);
    for (uint64_t i = j->lo; i < j->hi; i++) j->count[j->src[i * j->r + j->b]] += 1;
  } else {
    for (uint64_t i = j->lo; i < j->hi; i++) {
      uint32_t v = j->src[i * j->r + j->b];
      memcpy(j->dst + j->next[v] * j->r, j->src + i * j->r, j->r);
      j->next[v] += 1;
    }
  }
  return NULL;
}

static int run_phase(chunk_job* jobs, uint32_t T) {
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * T);
  if (!th) return -1;
  uint32_t started = 0;
  for (uint32_t t = 0; t < T; t++) {
    if (pthread_create(&th[t], NULL, chunk_worker, &jobs[t]) != 0) break;
    started++;
  }
  for (uint32_t t = 0; t < started; t++) pthread_join(th[t], NULL);
  /* chunks whose thread could not be started run here, so the pass completes */
  for (uint32_t t = started; t < T; t++) chunk_worker(&jobs[t]);
  free(th);
  return 0;
}

int oracle_sort_threads(uint8_t* rec, uint64_t n, uint32_t r, uint32_t k, uint32_t T) {
  if (k == 0 || k > r) return -1;
  if (T <= 1) return oracle_sort(rec, n, r, k);
  if (n < 2) return 0;
  uint8_t* tmp = (uint8_t*)malloc(n * r);
  chunk_job* jobs = (chunk_job*)calloc(T, sizeof(chunk_job));
  if (!tmp || !jobs) { free(tmp); free(jobs); return -1; }
  uint8_t* src = rec;
  uint8_t* dst = tmp;
  for (uint32_t b = 0; b < k; b++) {
    for (uint32_t t = 0; t < T; t++) {
      jobs[t].src = src; jobs[t].dst = dst; jobs[t].r = r; jobs[t].b = b;
      jobs[t].lo = n * t / T; jobs[t].hi = n * (t + 1) / T; jobs[t].phase = 0;
    }
    if (run_phase(jobs, T)) { free(tmp); free(jobs); return -1; }
    uint64_t run = 0;
    for (int v = 0; v < 256; v++)
      for (uint32_t t = 0; t < T; t++) { jobs[t].next[v] = run; run += jobs[t].count[v]; }
    for (uint32_t t = 0; t < T; t++) jobs[t].phase = 1;
    if (run_phase(jobs, T)) { free(tmp); free(jobs); return -1; }
    uint8_t* x = src; src = dst; dst = x;
  }
  if (src != rec) memcpy(rec, src, n * r);
  free(tmp);
  free(jobs);
  return 0;
}

/* ---- digit of the key integer, bit by bit -------------------------------
 * digit(i) = floor(K_i / 2^shift) mod 2^bits, K_i the little-endian key of
 * record i.  Bits at or above 8*k read as zero.
 */
static uint32_t key_digit(const uint8_t* rec, uint32_t k, uint32_t shift, uint32_t bits) {
  uint32_t v = 0;
  for (uint32_t j = 0; j < bits; j++) {
    uint32_t pos = shift + j;
    uint32_t bit = 0;
    if (pos < 8 * k) bit = (rec[pos / 8] >> (pos % 8)) & 1u;
    v |= bit << j;
  }
  return v;
}

/*
 * oracle_digit_histogram: counts[v] = number of records whose digit
 * (shift, bits) equals v, v in [0, 2^bits).  The first traversal of a
 * counting pass (Sec. 1), for one digit anywhere in the key.
 */
int oracle_digit_histogram(const uint8_t* rec, uint64_t n, uint32_t r, uint32_t k,
                           uint32_t shift, uint32_t bits, uint64_t* counts) {
  if (k == 0 || k > r || bits == 0 || bits > 16) return -1;
  memset(counts, 0, sizeof(uint64_t) << bits);
  for (uint64_t i = 0; i < n; i++) counts[key_digit(rec + i * r, k, shift, bits)] += 1;
  return 0;
}

/*
 * oracle_partition: one stable counting pass (Sec. 1) on the digit
 * (shift, bits): out = the records of `in` ordered by digit value, records
 * with the same digit value in input order.  This is the split that one MSD
 * level applies to a bin (Sec. 1, last paragraph; Sec. 3.2-3.4).
 */
int oracle_partition(const uint8_t* in, uint8_t* out, uint64_t n, uint32_t r, uint32_t k,
                     uint32_t shift, uint32_t bits) {
  if (k == 0 || k > r || bits == 0 || bits > 16) return -1;
  uint64_t R = 1ull << bits;
  uint64_t* next = (uint64_t*)calloc(R, sizeof(uint64_t));
  if (!next) return -1;
  oracle_digit_histogram(in, n, r, k, shift, bits, next);
  uint64_t run = 0;
  for (uint64_t v = 0; v < R; v++) { uint64_t c = next[v]; next[v] = run; run += c; }
  for (uint64_t i = 0; i < n; i++) {
    uint32_t v = key_digit(in + i * r, k, shift, bits);
    memcpy(out + next[v] * r, in + i * r, r);
    next[v] += 1;
  }
  free(next);
  return 0;
}

/*
 * oracle_sort_segments: each segment [off[s], off[s+1]) sorted on its own
 * (the definition of a batch of independent arrays).
 */
int oracle_sort_segments(uint8_t* rec, const uint64_t* off, uint32_t S, uint32_t r, uint32_t k) {
  for (uint32_t s = 0; s < S; s++) {
    if (off[s + 1] < off[s]) return -1;
    int rc = oracle_sort(rec + off[s] * r, off[s + 1] - off[s], r, k);
    if (rc) return rc;
  }
  return 0;
}

/*
 * oracle_count_runs: duplicate removal with counting over records already in
 * key order -- the second half of the k-mer counting application of Sec. 5,
 * where the k-mers of a bin are sorted and then their duplicates removed.
 * A run is a maximal stretch of consecutive records whose keys (bytes
 * [0, k)) are identical.  For the j-th run, uniq receives its first record
 * (all r bytes; with a stable sort that is the earliest input record of that
 * key) and counts[j] its length.  *u receives the number of runs.  uniq and
 * counts must hold n entries.  Returns 0, or -1 on inconsistent arguments.
 */
int oracle_count_runs(const uint8_t* sorted, uint64_t n, uint32_t r, uint32_t k,
                      uint8_t* uniq, uint64_t* counts, uint64_t* u) {
  if (k == 0 || k > r) return -1;
  uint64_t runs = 0;
  for (uint64_t i = 0; i < n; i++) {
    const uint8_t* x = sorted + i * r;
    if (i == 0 || memcmp(x, x - r, k) != 0) {  /* a new key starts a run */
      memcpy(uniq + runs * r, x, r);
      counts[runs] = 0;
      runs += 1;
    }
    counts[runs - 1] += 1;
  }
  *u = runs;
  return 0;
}
