// synth_gen.hip -- device twin of synth/gen.py (seeded synthetic records).
// Holds only input generation; none of the sorting method.  Each record is a
// pure function of (stream bases, global index), so any range regenerates
// on its own and matches the host generator byte for byte.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <stdint.h>

namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;
constexpr uint64_t MIX_T_UNIFORM = 1ull << 52;
constexpr uint64_t MIX_T_ZIPF = 7205759403792793ull;

struct Bases {
  uint64_t key, key_hi, zipf, mix, salt_lo, salt_hi;
  uint64_t payload[16];
  uint64_t p24;
  uint64_t genome, kmerpos, kmererr;  // k-mer keys: stream bases
  uint64_t windows, bases;            // start positions W, bases per k-mer K
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t val(uint64_t base, uint64_t i) { return mix64(base + (i + 1) * GAMMA); }

__global__ void k_fill(uint32_t* out, uint64_t i0, uint64_t count, uint32_t r, uint32_t k, int dist, int pay_index,
                       Bases B, const double* cdf, uint32_t m) {
  uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t >= count) return;
  uint64_t i = i0 + t;
  uint64_t lo = val(B.key, i), hi = val(B.key_hi, i);
  int code = dist;  // 0 uniform, 1 zipf, 2 prefix, 3 mix, 4 k-mers
  if (dist == 3) {
    uint64_t c = val(B.mix, i) >> 11;
    code = c < MIX_T_UNIFORM ? 0 : (c < MIX_T_ZIPF ? 1 : 2);
  }
  if (code == 1) {
    double x = (double)(val(B.zipf, i) >> 11) * (1.0 / 9007199254740992.0);
    uint32_t a = 0, b = m;  // first index with cdf[idx] > x
    while (a < b) {
      uint32_t mid = (a + b) / 2;
      if (cdf[mid] <= x) a = mid + 1; else b = mid;
    }
    uint64_t j = (uint64_t)(a < m ? a : m - 1) + 1;
    lo = mix64(j ^ B.salt_lo);
    hi = mix64(j ^ B.salt_hi);
  } else if (code == 4) {
    // bits [2p, 2p + 2K) of the genome, 32 bases per stream word
    const uint64_t K = B.bases;
    const uint64_t b = 2 * (val(B.kmerpos, i) % B.windows);
    const uint64_t w0 = b >> 6, s = b & 63;
    const uint64_t g0 = val(B.genome, w0), g1 = val(B.genome, w0 + 1), g2 = val(B.genome, w0 + 2);
    lo = s ? (g0 >> s) | (g1 << (64 - s)) : g0;
    hi = s ? (g1 >> s) | (g2 << (64 - s)) : g1;
    if (2 * K <= 64) {
      hi = 0;
      if (2 * K < 64) lo &= (1ull << (2 * K)) - 1;
    } else if (2 * K < 128) {
      hi &= (1ull << (2 * K - 64)) - 1;
    }
    const uint64_t e = val(B.kmererr, i);
    if ((e >> 58) == 0) {  // one substituted base
      const uint64_t q = (e & 0xFFFF) % K;
      const uint64_t flip = ((e >> 16) % 3 + 1) << ((2 * q) & 63);
      if (q < 32) lo ^= flip; else hi ^= flip;
    }
  } else if (code == 2) {
    const uint64_t mask40 = (1ull << 40) - 1;
    if (k == 8) lo = (B.p24 << 40) | (lo & mask40);
    else hi = (B.p24 << 40) | (hi & mask40);
  }
  // assemble the record bytes as words
  uint8_t bytes[64];
  for (uint32_t q = 0; q < 8; q++) { bytes[q] = (uint8_t)(lo >> (8 * q)); bytes[8 + q] = (uint8_t)(hi >> (8 * q)); }
  uint8_t rec[64];
  for (uint32_t q = 0; q < k; q++) rec[q] = bytes[q];
  uint32_t pl = r - k;
  for (uint32_t w = 0; 8 * w < pl; w++) {
    uint64_t v = (w == 0 && pay_index) ? i : val(B.payload[w], i);
    for (uint32_t q = 0; q < 8 && 8 * w + q < pl; q++) rec[k + 8 * w + q] = (uint8_t)(v >> (8 * q));
  }
  uint32_t* dst = out + t * (r / 4);
  for (uint32_t q = 0; q < r / 4; q++)
    dst[q] = rec[4 * q] | ((uint32_t)rec[4 * q + 1] << 8) | ((uint32_t)rec[4 * q + 2] << 16) |
             ((uint32_t)rec[4 * q + 3] << 24);
}

}  // namespace

extern "C" int synth_fill(void* out, uint64_t i0, uint64_t count, uint32_t rec_bytes, uint32_t key_bytes, int dist,
                          int payload_index, const uint64_t* bases, const double* cdf, uint32_t m, void* stream) {
  if (rec_bytes % 4 || rec_bytes > 64 || key_bytes > 16 || key_bytes > rec_bytes) return -1;
  if (count == 0) return 0;
  Bases B;
  B.key = bases[0]; B.key_hi = bases[1]; B.zipf = bases[2]; B.mix = bases[3];
  B.salt_lo = bases[4]; B.salt_hi = bases[5];
  for (int w = 0; w < 16; w++) B.payload[w] = bases[6 + w];
  B.p24 = bases[22];
  B.genome = bases[23]; B.kmerpos = bases[24]; B.kmererr = bases[25];
  B.windows = bases[26]; B.bases = bases[27];
  if (dist == 4 && (B.windows == 0 || B.bases == 0 || B.bases > 4ull * key_bytes)) return -1;
  (void)hipGetLastError();  // report this call's launches only
  // a launch covers fewer than 2^32 work-items: fill 2^30 records per launch
  const uint64_t step = 1ull << 30;
  for (uint64_t a = 0; a < count; a += step) {
    const uint64_t c = count - a < step ? count - a : step;
    const uint64_t blocks = (c + 255) / 256;
    hipLaunchKernelGGL(k_fill, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream,
                       (uint32_t*)out + a * (rec_bytes / 4), i0 + a, c, rec_bytes, key_bytes, dist, payload_index, B,
                       cdf, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      fprintf(stderr, "synth_fill: %s\n", hipGetErrorString(e));
      return -3;
    }
  }
  return 0;
}
