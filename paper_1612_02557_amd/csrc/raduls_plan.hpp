// raduls_plan.hpp -- launch plan and workspace layout shared by host and kernels.
#pragma once
#include <stdint.h>

#include "../../include/raduls.h"

namespace rd {

// Multi-workgroup list entry and queued single-workgroup bucket (32 bytes).
struct Bucket {
  uint64_t begin;   // first record
  uint64_t count;   // records
  uint64_t parent;  // records of the parent bucket (narrowing factor, Sec. 3.5)
  uint32_t bit;     // leading key bits already resolved
  uint32_t flags;   // bit 0: data in tmp; bit 1: skip the scatter (set by the scan)
};
constexpr uint32_t BF_TMP = 1u;
constexpr uint32_t BF_SKIP = 2u;
constexpr uint32_t BF_ROOT = 4u;  // deferred job that is a queued bucket (one more radix pass allowed)
constexpr uint32_t BF_GROUP = 8u; // finishing job made of several consecutive children

constexpr uint32_t LMAX = 20;        // multi-workgroup levels a plan may launch
constexpr uint32_t TSCAN_CH = 32;    // tiles per chunk of the tile-offset scan
constexpr uint32_t TINY_MAX = 32;    // buckets this small go to one wavefront (Sec. 3.5: N <= 32)
constexpr uint32_t SMALL_LDS_BYTES = 80 * 1024;  // dynamic LDS of the single-workgroup kernel
constexpr uint32_t NCLASS = 40;      // size classes of the queued buckets (floor(log2(count)))

// Finishing jobs held in registers (k_finish.hip): a 1024-thread workgroup
// holds fin_records_per_thread(rw) records per thread (at most 68 words),
// sorts composites of (key bits below a 12-bit digit, index) in LDS.
constexpr uint32_t FIN_THREADS = 1024;
constexpr uint32_t FIN_DIGIT_BITS = 12;
__host__ __device__ constexpr uint32_t fin_records_per_thread(uint32_t rw) { return 68 / rw < 17 ? 68 / rw : 17; }
// Keys above 8 bytes: 128-bit composites (16 bytes of LDS each), so at most
// 8 records per thread.
__host__ __device__ constexpr uint32_t fin_records_per_thread_wide(uint32_t rw) { return 68 / rw < 8 ? 68 / rw : 8; }
// composite bits of a job of keys with `kbits` bits
__host__ __device__ constexpr uint32_t fin_comp_bits(uint32_t kbits) { return kbits > 64 ? 128u : 64u; }
constexpr uint32_t FIN_MAX_RECORDS = 17 * FIN_THREADS;
constexpr uint32_t FIN_LDS_BYTES = 147712;  // composites of the largest job and 2^12 16-bit counters
constexpr uint32_t FIN_LDS_BIG = 544;       // > FIN_MAX_RECORDS / 33: sub-bins above 32 records
constexpr uint32_t FIN_STATIC_LDS = 16128;  // upper bound of the kernel's static LDS (with the dynamic part: 160 KiB)
static_assert(FIN_LDS_BYTES >= 8 * FIN_MAX_RECORDS + 4 * ((1u << FIN_DIGIT_BITS) / 2 + 1), "LDS of a finishing job");
static_assert(FIN_MAX_RECORDS < 65536, "16-bit counters and slots");
static_assert(FIN_LDS_BYTES >= 16 * 8 * FIN_THREADS + 4 * ((1u << FIN_DIGIT_BITS) / 2 + 1), "LDS of a wide finishing job");

// Device control block: list sizes, tickets, flags.  Cleared at the start of
// every sort by the init kernel.
struct Ctl {
  uint32_t nbig[LMAX + 1];     // entries of each multi-workgroup list
  uint32_t ticket[LMAX + 1];   // tile tickets of each level's scatter
  uint32_t cticket[LMAX + 1];  // chunk tickets of each level's tile-offset scan
  uint64_t ntiles[LMAX + 1];   // tiles of each list (set by the prefix kernel)
  uint32_t nsmall;             // queued single-workgroup buckets
  uint32_t ntiny;              // queued tiny buckets
  uint32_t ncopy;              // buckets to copy from tmp to records
  uint32_t small_head;         // queue cursors of the persistent kernels
  uint32_t tiny_head;
  uint32_t nwg;                // deferred workgroup jobs
  uint32_t wg_head;
  uint32_t class_count[NCLASS];
  uint64_t copy_tiles;
  uint32_t copy_ticket;
  uint32_t error;              // bit 0: bad segment offsets, bit 1: look-back wait limit (the
                               // scatters that follow are skipped), bit 2: a finishing job the
                               // register kernel cannot take (never queued by the routing)
  uint32_t overflow;           // bit 0 big list, 1 small, 2 tiny, 3 copy, 4 stack, 5 deferred jobs
  uint32_t epoch;              // look-back epoch of level 0 of this sort
  uint32_t pad;
  // records handled by the single-workgroup kernels: [0] one-workgroup radix
  // passes (each pass counts its bucket), [1] wavefront jobs of the queue
  // pass, [2] workgroup jobs of the jobs pass, [3] tiny buckets
  unsigned long long stage_records[4];
};

// Control block of the run-counting pass (k_count.hip), zeroed per call.
struct RunCtl {
  uint32_t ticket;  // tiles handed out
  uint32_t error;   // bit 0: look-back wait limit (the outputs are incomplete)
};

struct Plan {
  uint64_t n;              // records in all
  uint64_t t_big;          // buckets above this are multi-workgroup (Sec. 3.2: 2N/3T)
  uint64_t cap_big;        // entries per multi-workgroup list
  uint64_t cap_small;      // entries of the single-workgroup queue
  uint64_t cap_tiny;
  uint64_t cap_copy;
  uint64_t cap_wg;         // deferred workgroup jobs
  uint64_t max_tiles;      // tiles of one level, upper bound
  uint32_t rec_bytes, key_bytes, rw;
  uint32_t d_big, d_block; // digit widths
  uint32_t tile;           // records per tile of a multi-workgroup pass
  uint32_t c_fin;          // largest bucket finished in LDS
  uint32_t bitonic_max;
  uint32_t nontemporal;
  uint32_t lmax;           // levels launched
  uint32_t grid_hist, grid_scatter, grid_small, grid_clear;
  uint32_t stack_cap;      // entries per workgroup stack
  uint32_t block_tile;     // records per tile of a one-workgroup pass
  uint32_t wave_cap;       // largest bucket one wavefront finishes
  uint32_t job_window;     // children are grouped by windows of this many records
  uint32_t sched_mode, forced_proc;
  uint32_t segmented;
  uint32_t epoch;          // look-back epoch of level 0 (level l uses epoch + l)
  uint32_t sample_period;  // counterfactual sampling period (0 = none)
  uint32_t has_model;
  uint32_t partition;      // 1: one level on one bucket, children not routed
  uint32_t partition_bit;  // resolved bits of that bucket
  uint32_t spin_limit;     // polls a look-back wait makes before it gives up
  uint32_t fin_max;        // largest job finished in registers (0: jobs go to the LDS path)
  uint32_t grid_fin;       // workgroups of the register-finishing kernel
  uint32_t inplace;        // 1: levels partition in place (no tmp; children stay in the records)
  uint64_t trace_cap;
};

// Device pointers of the workspace.
struct Work {
  Ctl* ctl;
  Bucket* big;         // (LMAX + 1) lists of cap_big entries
  uint64_t* tile_start;       // (LMAX + 1) x (cap_big + 1)
  uint64_t* hist;             // cap_big x 2^d_big (per level, reused)
  uint64_t* vary;             // cap_big x 2 (OR of key XOR reference key)
  uint64_t* status;           // tile digit offsets, max_tiles x 2^d_big, then the chunk look-back words
  uint32_t* tcnt;             // tile digit counts, max_tiles x 2^d_big
  uint32_t* tbucket;          // list entry of each tile of the level (set by the offset scan)
  uint64_t* cstatus;          // look-back words of the tile-offset scan, (max_tiles / TSCAN_CH + 2) x 2^d_big
  Bucket* small;       // cap_small
  Bucket* small_ord;   // cap_small, ordered largest class first
  uint64_t* tiny;             // cap_tiny packed tiny buckets
  Bucket* copy;        // cap_copy
  uint64_t* copy_start;       // cap_copy + 1
  Bucket* stacks;      // grid_small x stack_cap
  Bucket* wgjobs;             // cap_wg deferred workgroup jobs
  const float* model;         // scheduler network + feature normalisation, or null
  raduls_trace_row* trace;
  uint64_t* trace_count;
  uint64_t* counts_out;       // partition: histogram for the caller, or null
  uint32_t* epoch_counter;    // look-back epochs handed out so far
};

// ---- in-place levels (k_inplace.hip) ---------------------------------------
// A level partitions each of its buckets within its own records.  Records
// are moved in blocks of ip_block_records(rw) records (at most 512 bytes):
// each stripe of a bucket is first rewritten as whole blocks of one digit
// each, which then move to their children's ranges; the few records that
// do not fill a block (at most a block per digit and stripe) wait in a side
// buffer and fill the children's edges at the end.
constexpr uint32_t IP_WG = 1024;          // threads of the in-place workgroups
constexpr uint32_t IP_R = 256;            // digits of a level (8 bits)
constexpr uint32_t IP_BLOCK_BYTES = 512;  // bytes of a block, at most
constexpr uint32_t IP_SLB = 32768;        // blocks per stripe of a bucket split among workgroups (more for n above 2^28 blocks)
constexpr uint32_t IP_MLB = 147456;       // blocks of a bucket done by one workgroup, at most (its read bits fill 18 KiB of LDS)
constexpr uint32_t IP_MAX_STRIPES = 8192; // stripes of one bucket, at most
constexpr uint32_t IP_CHUNK = 64;         // block reads per claim of the permutation
constexpr uint32_t IP_BIAS = 1u << 30;    // added to the read cursor so that extra decrements never borrow
constexpr uint32_t IP_WSTRIDE = 16;       // 64-bit words between the cursor words of two ranges (one per cache line)
__host__ __device__ constexpr uint32_t ip_block_records(uint32_t rw) { return IP_BLOCK_BYTES / (4 * rw); }

struct IpCtl {
  uint32_t nlarge;         // buckets of the level split into stripes
  uint32_t nmedium;        // buckets of the level partitioned by one workgroup
  uint32_t nstripes;       // stripes of the large buckets
  uint32_t nranges;        // child ranges of the large buckets (256 each)
  uint32_t stripe_ticket, medium_ticket, chunk_ticket;
  uint32_t nchunks, stride;
  uint32_t error;          // bit 0: capacity, bit 1: wait limit, bit 2: cursor out of its range
};

struct IpWork {
  IpCtl* ctl;
  uint32_t* large;         // cap_large: list entry of each large bucket
  uint32_t* stripe_first;  // cap_large + 1: first stripe of each large bucket
  uint32_t* medium;        // cap_big: list entry of each medium bucket
  uint32_t* nbfull;        // cap_stripes: blocks written by each stripe
  uint16_t* lcnt;          // cap_stripes x IP_R: records left over per stripe and digit
  uint8_t* side;           // cap_stripes x IP_R x IP_BLOCK_BYTES: those records
  uint8_t* prot;           // cap_ranges x IP_BLOCK_BYTES: records of a child's last block past the child's end
  uint64_t* W;             // cap_ranges x IP_WSTRIDE: write cursor << 32 | (read cursor + IP_BIAS), in block slots
  uint64_t* rbase;         // cap_ranges: first record of each child, relative to its bucket
  uint64_t* rlim;          // cap_ranges: end of each child, relative to its bucket
  uint32_t* rf;            // cap_ranges: first block slot starting inside the child
  uint32_t* re;            // cap_ranges: end of the child's slots
  uint32_t* rF;            // cap_ranges: blocks of the child's digit
  uint32_t* rL;            // cap_ranges: records of the child left over in the stripes
  uint32_t* rinit;         // cap_ranges: read cursor before the permutation
  uint32_t* chunk_start;   // cap_ranges + 1: permutation chunks of each range (prefix)
  uint32_t* done;          // done_words: one bit per block of the records, set once its reader has it
  uint8_t* bdig;           // done_words x 32: digit of each full block of a large bucket (by block index)
  uint8_t* mscratch;       // grid_medium x IP_R x IP_BLOCK_BYTES: protruding records of the medium kernel
  uint64_t cap_large, cap_stripes, cap_ranges, done_words;
  uint32_t grid_medium;
  uint32_t slb;            // blocks per stripe (IP_SLB, longer for huge n, shorter only in tests)
  uint32_t mlb;            // blocks of a bucket one workgroup takes, at most (IP_MLB; the stripe in tests)
};

}  // namespace rd
