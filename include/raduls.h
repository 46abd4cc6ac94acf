/*
 * raduls.h -- C interface of an MI355X (gfx950) most-significant-digit radix
 * sorter of fixed-size records, after RADULS (Kokot, Deorowicz,
 * Debudaj-Grabysz, "Sorting Data on Ultra-Large Scale with RADULS", arXiv
 * 1612.02557).
 *
 * Conventions shared by every call
 * --------------------------------
 * Record model (paper, Sec. 1 and Sec. 4): a record is rec_bytes bytes; its
 * key is the unsigned little-endian integer in bytes [0, key_bytes) (byte
 * key_bytes-1 is most significant); bytes [key_bytes, rec_bytes) are payload
 * and move with the key unchanged.  Sorting is ascending by key and STABLE:
 * records with equal keys keep their input order.  (The paper's own finishing
 * sorts are not stable; this library always produces the stable order, which
 * is the unique correct output.)
 *
 * Supported shapes: 1 <= key_bytes <= 16, key_bytes <= rec_bytes,
 * rec_bytes a multiple of 4 and at most 64; record arrays 16-byte aligned.
 *
 * Pointers named "device" point to GPU memory (hipMalloc or a framework
 * allocator); pointers named "host" point to ordinary CPU memory.  `stream`
 * is a hipStream_t passed as void* (NULL = the legacy default stream).  Work
 * is enqueued on that stream and the calls return without waiting for it,
 * unless stated otherwise.
 *
 * Ownership: the caller owns every buffer it passes.  The library owns a
 * per-device workspace (bucket lists, histograms, tile offsets, queues)
 * that grows on demand and is freed by raduls_release().  Calls on different
 * streams of one device serialise on that workspace (the library orders them
 * with an event); calls from several host threads are serialised by a mutex.
 *
 * Errors: every call validates its arguments before any device work, so a
 * call that returns RADULS_EINVAL or RADULS_EUNSUPPORTED has modified
 * nothing.  RADULS_EHIP reports a HIP runtime failure (buffer contents are
 * then undefined); raduls_last_error_message() gives the HIP message.
 */
#ifndef RADULS_H
#define RADULS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum raduls_status {
  RADULS_OK = 0,
  RADULS_EINVAL = -1,       /* bad argument (null pointer, overlap, sizes) */
  RADULS_ENOMEM = -2,       /* workspace allocation failed; inputs untouched */
  RADULS_EHIP = -3,         /* HIP runtime error */
  RADULS_EUNSUPPORTED = -4, /* shape outside the supported range */
  RADULS_EMODEL = -5,       /* model blob rejected; the heuristic stays in use */
  RADULS_EDEVICE = -6       /* a device-side check failed (see raduls_sync_check) */
};

/* Procedures a bucket can be given (paper, Sec. 3.2-3.5, mapped to the GPU):
 * RADIX    one more radix pass by one workgroup through memory, children
 *          handled recursively (the paper's per-bin radix split, Sec. 3.4);
 * LSD      the remaining digits sorted inside the workgroup's LDS by stable
 *          counting passes (a bin that fits fast memory, Sec. 3.4);
 * BITONIC  comparison sort inside LDS (the tiny-bin comparison sort, Sec. 3.5);
 * RANK     one wavefront ranks up to 32 records by all-pairs comparison (the
 *          insertion-sort slot for bins of at most 32, Sec. 3.5);
 * BIG      a multi-workgroup pass (the big-bin pass, Sec. 3.3). */
enum raduls_proc { RADULS_PROC_RADIX = 0, RADULS_PROC_LSD = 1, RADULS_PROC_BITONIC = 2,
                   RADULS_PROC_RANK = 3, RADULS_PROC_BIG = 4 };

/* Scheduler modes for the choice between RADIX, LSD and BITONIC. */
enum raduls_sched { RADULS_SCHED_HEURISTIC = 0, /* the paper's thresholds (Sec. 3.2-3.5) */
                    RADULS_SCHED_LEARNED = 1,   /* the loaded network; heuristic fallback */
                    RADULS_SCHED_FORCED = 2 };  /* always `forced_proc` where feasible */

/* Tunable parameters.  None of them changes the output bytes. */
typedef struct raduls_tuning {
  uint32_t big_digit_bits;    /* digit width of multi-workgroup levels, 1..11 */
  uint32_t block_digit_bits;  /* digit width of one-workgroup radix passes, 1..11 */
  uint32_t tile_records;      /* records per tile of a multi-workgroup pass, 256..8192, power of 2 */
  uint32_t lds_finish_max;    /* largest bucket finished inside LDS (0 = as large as LDS allows) */
  uint32_t bitonic_max;       /* largest bucket the bitonic finish accepts (0 = the LDS capacity) */
  uint32_t workgroups_per_cu; /* resident workgroups per CU assumed by the big threshold, 1..8 */
  uint64_t big_min;           /* big buckets hold more than big_min records (and see big_rule) */
  uint32_t nontemporal;       /* 1: non-temporal stores for scattered output */
  uint32_t big_rule;          /* 0: also more than 2N/(3W) (Sec. 3.2, W = resident workgroups);
                                 1: big_min alone (the default, with big_min = 2 tiles) */
  uint32_t job_records;       /* children of a radix pass are grouped into finishing jobs of at
                                 most this many records (0 = the LDS capacity) */
  uint32_t reg_finish;        /* 1: keys of at most 8 bytes are finished by 1024-thread workgroups
                                 holding up to 17K records in registers (buckets that size leave
                                 the levels); 0: by the LDS procedures of at most the LDS capacity */
} raduls_tuning;

/* One row per scheduled bucket when tracing is on (64 bytes). */
typedef struct raduls_trace_row {
  float features[9];     /* the scheduler network's inputs for this bucket */
  uint32_t chosen;       /* procedure that produced the output */
  uint32_t count;        /* records in the bucket */
  uint32_t observed;     /* bit p set: time_ticks[p] was measured */
  uint32_t time_ticks[3];/* elapsed 100 MHz ticks of RADIX, LSD, BITONIC */
  uint32_t flags;        /* bit 0: counterfactual sample (every feasible procedure timed);
                            bit 1: one wavefront ran the job (RADIX not feasible there) */
} raduls_trace_row;

typedef struct raduls_stats {
  double last_ms;            /* device time of the last sort call (0 if not timed) */
  uint64_t last_records;
  uint32_t last_levels;      /* multi-workgroup levels launched */
  uint32_t sched_mode;
  uint64_t workspace_bytes;  /* bytes held by the workspace of the current device */
  uint64_t model_params;     /* parameters of the loaded network (0 = none) */
  uint64_t graph_cache_entries;
} raduls_stats;

/* ---- sorting ------------------------------------------------------------ */

/* Sort n records in `records` (device) by key, ascending and stable (paper,
 * Sec. 1: MSD radix sort with recursion per bin, Sec. 3).  `tmp` (device) is
 * scratch of the same size, n*rec_bytes bytes, not overlapping `records`; its
 * contents are undefined afterwards.  n <= 1 returns RADULS_OK at once. */
int raduls_sort(void* records, void* tmp, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes,
                void* stream);

/* Sort n records in `records` (device, 16-byte aligned) by key, ascending,
 * with no caller buffer besides the records: the in-place MSD variant the
 * paper sets its method against (Sec. 2, in-place radix sorting with a
 * speculative permutation and a repair step).  Each level partitions every
 * bucket within its own records, moving whole blocks of records of one
 * digit (at most 512 bytes each); buckets then finish in registers in
 * place.  NOT stable: records with equal keys end in an unspecified order
 * (the result's keys are those of raduls_sort, its records a permutation of
 * the input).  The library's own workspace
 * (raduls_inplace_workspace_bytes) replaces the n*rec_bytes of `tmp`.
 * n <= 1 returns RADULS_OK at once.  Same argument checks and error codes as
 * raduls_sort; device-side failures (a bounded wait that gave up, a
 * capacity or cursor check) are reported by raduls_sync_check. */
int raduls_sort_inplace(void* records, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, void* stream);

/* Bytes of library workspace a raduls_sort_inplace of n records uses
 * (0 for an unsupported shape). */
size_t raduls_inplace_workspace_bytes(uint64_t n, uint32_t rec_bytes, uint32_t key_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sort as raduls_sort, with the same arguments, results and argument
 * checks, but its workspace is one fixed array of
 * RADULS_NOALLOC_SCRATCH_BYTES per GPU inside the library (held until the
 * process ends) and it calls no allocating routine.  A sort whose workspace
 * (about raduls_workspace_bytes(n, ...)) does not fit that array returns
 * RADULS_EUNSUPPORTED before any device work; 2^22 records of up to 32 bytes
 * fit.  The caller still passes `records` and `tmp`.  All calls on one GPU
 * share the array, so calls that overlap on one GPU (different streams, or
 * threads) race and must be ordered by the caller.  The learned scheduler is
 * used only if its network is already on the device (after a raduls_sort
 * with it); otherwise the heuristic runs.  Tracing is off.  Device-side
 * failures are reported by raduls_sync_check. */
#define RADULS_NOALLOC_SCRATCH_BYTES (64ull << 20)
int raduls_sort_noalloc(void* records, void* tmp, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes,
                        void* stream);

/* Sort each segment [seg_offsets[s], seg_offsets[s+1]) of `records`
 * independently (a batch of independent arrays), in one launch sequence that
 * the library captures once per shape into a HIP graph and replays.
 * seg_offsets (device, num_segs+1 entries) must start at 0, be non-decreasing
 * and end at total_records; this is checked on the device, and a violation
 * leaves the data unmodified and is reported by raduls_sync_check(). */
int raduls_sort_segmented(void* records, void* tmp, const uint64_t* seg_offsets,
                          uint32_t num_segs, uint64_t total_records, uint32_t rec_bytes,
                          uint32_t key_bytes, void* stream);

/* One stable counting pass (paper, Sec. 1: histogram, offsets of smaller
 * digits, distribution) on the digit floor(key / 2^shift) mod 2^bits, with
 * 1 <= bits <= 11 and shift < 8*key_bytes: `out` (device) receives the
 * records of `in` (device) ordered by that digit, equal digits in input
 * order.  This is one MSD level on a single bucket, run by the same
 * multi-workgroup histogram, offset-scan and scatter kernels the sort
 * uses.  If `counts` (device, 2^bits uint64) is not NULL it receives the
 * histogram. */
int raduls_partition(const void* in, void* out, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes,
                     uint32_t shift, uint32_t bits, uint64_t* counts, void* stream);

/* Duplicate removal with counts over records in key order (paper, Sec. 5:
 * a k-mer counter sorts the k-mers of a bin and removes the duplicates).
 * A run is a maximal stretch of consecutive records of `sorted` (device, n
 * records) with identical keys.  For the j-th run (in record order)
 * uniq[j] (device, room for n records) receives its first record, all
 * rec_bytes bytes, and counts[j] (device, room for n uint64) its length;
 * *num_runs (device uint64) receives the number of runs U.  Entries at U and
 * beyond are left as they were.  uniq may be `sorted` itself (the runs are
 * then compacted in place) or must not overlap it; counts and num_runs
 * overlap nothing.  Buffers of records are 16-byte aligned, counts and
 * num_runs 8-byte aligned.  One pass over the records (a decoupled
 * look-back over tiles); stream-ordered, nothing is allocated after the
 * first call of a size.  A look-back wait that gives up is reported by
 * raduls_sync_check() (RADULS_EDEVICE); the outputs are then incomplete. */
int raduls_count_runs(const void* sorted, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, void* uniq,
                      uint64_t* counts, uint64_t* num_runs, void* stream);

/* raduls_sort of `records` followed by raduls_count_runs on them: the
 * distinct keys in ascending order with their multiplicities (k-mer
 * counting, Sec. 5).  uniq may be `records`, `tmp` (free once the sort is
 * done) or a buffer apart from both; records keep the sorted order unless
 * uniq is `records`. */
int raduls_sort_count(void* records, void* tmp, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, void* uniq,
                      uint64_t* counts, uint64_t* num_runs, void* stream);

/* Pattern-prefix search over a suffix array (paper, Sec. 5: patterns are
 * looked up in a suffix array by binary search; with the patterns, or their
 * prefixes, sorted first, the searches run in narrowed ranges).
 * text (device, text_len bytes, 1 <= text_len < 2^32): the text; sa (device,
 * text_len uint32): its suffix array, i.e. the suffix start positions in
 * lexicographic order (any order in which the k-prefixes defined below do
 * not decrease will do).  queries (device, nq records of rec_bytes, 16-byte
 * aligned): the key of query i (key_bytes = k <= 16 bytes) holds k pattern
 * characters reversed -- key byte k-1 is the first character -- so that key
 * order is string order.  The k-prefix of suffix j is text[j, j+k) with
 * zero bytes past the end of the text.  lo[i] (device uint64) receives the
 * number of suffixes whose k-prefix is below query i's characters and hi[i]
 * the number at or below them: sa[lo[i], hi[i]) are the suffixes that start
 * with them.  Results do not depend on the query order; queries in
 * ascending key order (as raduls_sort leaves them) are searched in ranges
 * narrowed per 256 consecutive queries, unless `flags` holds
 * RADULS_SEARCH_NO_NARROWING (every query searched over the whole array).
 * lo and hi overlap nothing.  Stream-ordered; allocates nothing. */
#define RADULS_SEARCH_NO_NARROWING 1u
int raduls_prefix_search(const void* text, uint64_t text_len, const uint32_t* sa, const void* queries, uint64_t nq,
                         uint32_t rec_bytes, uint32_t key_bytes, uint64_t* lo, uint64_t* hi, uint32_t flags,
                         void* stream);

/* raduls_sort of the query records (stable, by key) followed by
 * raduls_prefix_search on them: lo/hi follow the sorted order, and a
 * payload carrying each pattern's id maps them back. */
int raduls_sort_search(void* queries, void* tmp, uint64_t nq, uint32_t rec_bytes, uint32_t key_bytes, const void* text,
                       uint64_t text_len, const uint32_t* sa, uint64_t* lo, uint64_t* hi, void* stream);

/* Wait for `stream` and report device-side failures of earlier calls on this
 * device (RADULS_EDEVICE: invalid segment offsets).  Clears the flags. */
int raduls_sync_check(void* stream);

/* ---- scheduling, tuning, tracing ---------------------------------------- */

int raduls_set_scheduler(int mode, int forced_proc);
int raduls_get_scheduler(int* mode, int* forced_proc);

/* Load the scheduler network from a host blob: header "RDLSMLP1", uint32
 * F, H, P (must be 9, 32, 3), then F*H+H+H*H+H+P*H+P float32 parameters in
 * the order W1 (HxF row-major), b1, W2, b2, W3, b3, then feature means and
 * scales (2*F float32) and a uint32 checksum (FNV-1a of everything before
 * it).  Rejected blobs return RADULS_EMODEL and leave the current model. */
int raduls_load_model(const void* host_blob, size_t bytes);
/* A bucket whose features, normalized by the blob's means and scales, are
 * not all within +-RADULS_MLP_OOD_Z lies outside the network's training
 * range (the scales are the training features' standard deviations): the
 * heuristic decides it. */
#define RADULS_MLP_OOD_Z 4.0f
int raduls_unload_model(void);

/* Set the tuning of all later sorts; NULL returns to the defaults and
 * forgets the autotuner's results. */
int raduls_set_tuning(const raduls_tuning* host_tuning);
int raduls_get_tuning(raduls_tuning* host_tuning);
int raduls_default_tuning(uint32_t rec_bytes, uint32_t key_bytes, uint64_t n,
                          raduls_tuning* host_tuning);
/* Autotuner (the paper picked its constants by experiment, Sec. 3.2-3.5).
 * A coordinate search from the defaults: register finishing on or off,
 * level digit width (8..11 bits), tile size, finishing-job size, resident
 * workgroups per CU, big-bucket rule and non-temporal stores, each in turn
 * taking the value that times best with the others fixed.  Each candidate
 * is timed on two probe inputs of min(max(n_hint, 2^16), 2^27) records that
 * it generates on the device (uniform keys; keys with 4096 distinct values;
 * payload = index), the median of three timed sorts each.  The result is
 * kept for (rec_bytes, key_bytes, floor(log2 n_hint)) and used by every
 * later sort of that shape and size class (unless raduls_set_tuning set a
 * tuning, which takes precedence); a second call for the same class returns
 * at once.  Allocates and frees 4 * n * rec_bytes bytes of probe buffers
 * (ENOMEM if that fails, nothing then changed) and waits for `stream`.  No
 * tuning changes the bytes a sort produces. */
int raduls_tune(uint32_t rec_bytes, uint32_t key_bytes, uint64_t n_hint, void* stream);
/* The tuning a sort of n records of this shape would use now (the one set
 * by raduls_set_tuning, else the autotuner's result for the shape class,
 * else the defaults). */
int raduls_effective_tuning(uint32_t rec_bytes, uint32_t key_bytes, uint64_t n,
                            raduls_tuning* host_tuning);

/* Record one raduls_trace_row per scheduled bucket into `rows` (device,
 * `capacity` rows); every `sample_period`-th eligible bucket (0 = none) is
 * run under each procedure in turn and all three times are recorded.  The
 * output bytes do not change.  rows == NULL turns tracing off.  The number
 * of rows written (which may exceed capacity; extra rows are dropped) is read
 * with raduls_trace_count, which waits for the stream. */
int raduls_set_trace(void* rows, uint64_t capacity, uint32_t sample_period);
int raduls_trace_count(uint64_t* host_count, void* stream);

int raduls_get_stats(raduls_stats* host_stats);
/* 1: time every sort with events (raduls_get_stats().last_ms); 2: also time
 * each launch group of raduls_sort (raduls_phase_times); 0: off. */
int raduls_set_timing(int on);
/* Device milliseconds of each launch group of the last raduls_sort run with
 * timing mode 2, waiting for it: index 0 setup; for level l (0..19) 1+4l
 * tile ranges and histogram reset, 2+4l histogram, 3+4l scan, 4+4l scatter
 * (raduls_sort_inplace: 1+4l set-up and the one-workgroup buckets, 2+4l
 * classification of the stripes, 3+4l children, ranges and cleanup, 4+4l
 * block permutation);
 * 81 queue ordering, 82 single-workgroup queue pass, 83 single-workgroup
 * jobs pass, 84 copy-back.  `count` entries of host_ms are written (85 cover
 * every phase). */
#define RADULS_PHASES 85
int raduls_phase_times(double* host_ms, uint32_t count);
/* Records handled by each stage of the last sort, waiting for the device:
 * [2l] records in level l's buckets (histogram reads), [2l+1] records that
 * level moved (scatter) -- for raduls_sort_inplace: the records of the
 * buckets split into stripes among workgroups, the others being partitioned
 * by one workgroup each -- l = 0..19; [40] records queued for the
 * single-workgroup kernel, [41] records in tiny buckets, [42] records copied
 * back from tmp, [43] records through one-workgroup radix passes (a record
 * counts once per pass), [44] records finished by wavefront jobs, [45]
 * records finished by workgroup jobs, [46] records finished as tiny buckets,
 * [47] the largest job finished in registers (0: the workgroup jobs ran in
 * LDS).  `count` entries are written (48 cover all). */
int raduls_last_work(uint64_t* host_out, uint32_t count);

/* Bytes of library workspace a sort of n records needs (beyond the caller's
 * records and tmp). */
size_t raduls_workspace_bytes(uint64_t n, uint32_t rec_bytes, uint32_t key_bytes);

const char* raduls_status_string(int status);
const char* raduls_last_error_message(void);

/* Free the workspace and cached graphs of every device. */
void raduls_release(void);

/* ---- scheduler-network training kernels (float32) ----------------------- */
/* All arrays are device, row-major.  F = 9 inputs, H = 32 hidden, P = 3
 * outputs; theta holds RADULS_MLP_PARAMS floats in the layout of
 * raduls_load_model.  The network is a two-hidden-layer ReLU perceptron;
 * the loss is the masked mean squared error sum(M*(Y-T)^2)/sum(M) (0 when
 * sum(M) = 0).  Reductions run in a fixed order, so results are
 * deterministic. */
#define RADULS_MLP_F 9
#define RADULS_MLP_H 32
#define RADULS_MLP_P 3
#define RADULS_MLP_PARAMS (RADULS_MLP_F * RADULS_MLP_H + RADULS_MLP_H + \
                           RADULS_MLP_H * RADULS_MLP_H + RADULS_MLP_H + \
                           RADULS_MLP_P * RADULS_MLP_H + RADULS_MLP_P)

/* Y[B,P] = network(X[B,F]). */
int raduls_mlp_forward(const float* X, const float* theta, float* Y, uint32_t batch, void* stream);
/* loss[0] and grad[RADULS_MLP_PARAMS] of the masked MSE for targets T[B,P]
 * and mask M[B,P] (back-propagation). */
int raduls_mlp_loss_grad(const float* X, const float* T, const float* M, const float* theta,
                         float* grad, float* loss, uint32_t batch, void* stream);
/* One Adam step (Kingma and Ba 2015) at step t >= 1 on theta, moments m, v. */
int raduls_mlp_adam(float* theta, const float* grad, float* m, float* v, uint32_t t, float lr,
                    float beta1, float beta2, float eps, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RADULS_H */
