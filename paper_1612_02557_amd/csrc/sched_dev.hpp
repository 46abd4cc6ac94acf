// sched_dev.hpp -- per-bucket procedure choice on the device.
//
// The heuristic restates the paper's thresholds (Sec. 3.2-3.5) over the GPU
// procedures; the learned mode evaluates a small network (one thread per
// bucket) that predicts each procedure's log-time and takes the cheapest
// feasible one, falling back to the heuristic on a missing model, a
// non-finite prediction, or a bucket outside the network's training range
// (a normalized feature beyond RADULS_MLP_OOD_Z).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "raduls_plan.hpp"

namespace rd {

constexpr uint32_t P_RADIX = 0, P_LSD = 1, P_BITONIC = 2, P_RANK = 3;
constexpr uint32_t MLP_F = RADULS_MLP_F, MLP_H = RADULS_MLP_H, MLP_P = RADULS_MLP_P;
constexpr uint32_t MLP_NPARAM = RADULS_MLP_PARAMS;
// model buffer: parameters, then feature means, then feature scales
constexpr uint32_t MLP_MODEL_FLOATS = MLP_NPARAM + 2 * MLP_F;

constexpr uint32_t H_TINY = 384;        // Sec. 3.5
constexpr uint32_t H_TINY_NARROW = 32;  // Sec. 3.5
constexpr uint32_t H_NARROW = 16;       // Sec. 3.5, sqrt(R)

__device__ __forceinline__ float log2f_u64(uint64_t x) { return __log2f((float)x); }

// The nine network inputs of a bucket.
__device__ __forceinline__ void bucket_features(float* f, uint64_t m, uint64_t parent, uint32_t bit,
                                                uint32_t kbits, uint32_t rec_bytes, uint32_t key_bytes) {
  float lm = log2f_u64(m);
  float lp = log2f_u64(parent > m ? parent : m);
  f[0] = lm;
  f[1] = lp;
  f[2] = lp - lm;
  f[3] = (float)(kbits - bit) / 64.0f;
  f[4] = (float)bit / 64.0f;
  f[5] = (float)rec_bytes / 64.0f;
  f[6] = (float)key_bytes / 16.0f;
  f[7] = __log2f((float)m * (float)rec_bytes) - 16.0f;
  f[8] = (lp - lm) > 4.0f ? 1.0f : 0.0f;
}

// Feasible procedures (bit p set) for a bucket of m records.
__device__ __forceinline__ uint32_t feasible_mask(const Plan& p, uint64_t m, uint32_t bit, uint32_t kbits,
                                                  bool allow_radix) {
  uint32_t mask = 0;
  if (allow_radix) mask |= 1u << P_RADIX;
  if (m <= p.c_fin) mask |= 1u << P_LSD;
  // the bitonic composite holds the unresolved key bits and a local index
  uint32_t ib = 64 - __clzll(m - 1);
  if (m <= p.bitonic_max && (kbits - bit) + ib <= 128) mask |= 1u << P_BITONIC;
  return mask;
}

// Paper rules (Sec. 3.5: tiny bins < 384 keys, < 32 when the narrowing
// factor parent/current exceeds 16, get a comparison sort; Sec. 3.4: other
// bins get another radix pass, in fast memory when they fit there)
// restricted to the feasible procedures.
__device__ __forceinline__ uint32_t heuristic_proc(uint64_t m, uint64_t parent, uint32_t feas) {
  uint64_t tiny = (parent > (uint64_t)H_NARROW * m) ? H_TINY_NARROW : H_TINY;
  if (m < tiny && (feas & (1u << P_BITONIC))) return P_BITONIC;
  if (feas & (1u << P_RADIX)) return P_RADIX;
  if (feas & (1u << P_LSD)) return P_LSD;
  return P_BITONIC;
}

// Network prediction, one thread.  Returns the masked argmin, or 0xFFFFFFFF
// if any prediction is not finite.  W2T: the layer-2 matrix is stored
// transposed (element (j, i) at i * H + j), the layout of the copy in LDS.
template <bool W2T = false>
__device__ __forceinline__ uint32_t mlp_choose(const float* __restrict__ model, const float* feat, uint32_t feas) {
  const float* W1 = model;
  const float* b1 = W1 + MLP_H * MLP_F;
  const float* W2 = b1 + MLP_H;
  const float* b2 = W2 + MLP_H * MLP_H;
  const float* W3 = b2 + MLP_H;
  const float* b3 = W3 + MLP_P * MLP_H;
  const float* mean = model + MLP_NPARAM;
  const float* scale = mean + MLP_F;
  float x[MLP_F];
  bool ood = false;
#pragma unroll
  for (uint32_t i = 0; i < MLP_F; i++) {
    x[i] = (feat[i] - mean[i]) / scale[i];
    ood = ood || !(fabsf(x[i]) <= RADULS_MLP_OOD_Z);
  }
  if (ood) return 0xFFFFFFFFu;  // outside the training range: the heuristic decides
  float h1[MLP_H];
#pragma unroll 4
  for (uint32_t j = 0; j < MLP_H; j++) {
    float a = b1[j];
#pragma unroll
    for (uint32_t i = 0; i < MLP_F; i++) a = fmaf(W1[j * MLP_F + i], x[i], a);
    h1[j] = a > 0.0f ? a : 0.0f;
  }
  float y[MLP_P];
#pragma unroll
  for (uint32_t q = 0; q < MLP_P; q++) y[q] = b3[q];
  for (uint32_t j = 0; j < MLP_H; j++) {
    float a = b2[j];
#pragma unroll
    for (uint32_t i = 0; i < MLP_H; i++) a = fmaf(W2[W2T ? i * MLP_H + j : j * MLP_H + i], h1[i], a);
    a = a > 0.0f ? a : 0.0f;
#pragma unroll
    for (uint32_t q = 0; q < MLP_P; q++) y[q] = fmaf(W3[q * MLP_H + j], a, y[q]);
  }
  uint32_t best = 0xFFFFFFFFu;
  float bv = 0.0f;
#pragma unroll
  for (uint32_t q = 0; q < MLP_P; q++) {
    if (!isfinite(y[q])) return 0xFFFFFFFFu;
    if ((feas >> q) & 1u) {
      if (best == 0xFFFFFFFFu || y[q] < bv) { best = q; bv = y[q]; }
    }
  }
  return best;
}

// The same network evaluated by one whole wavefront for one bucket: lane j <
// H owns hidden unit j of both layers, layer 2 reads the first layer's units
// lane by lane, and the outputs are summed across lanes.  About 100
// instructions instead of the ~1400 of the one-thread form.  All lanes must
// be active; every lane returns the same choice (0xFFFFFFFF on a non-finite
// prediction).
template <bool W2T = false>
__device__ __forceinline__ uint32_t mlp_choose_wave(const float* __restrict__ model, const float* feat, uint32_t feas) {
  const float* W1 = model;
  const float* b1 = W1 + MLP_H * MLP_F;
  const float* W2 = b1 + MLP_H;
  const float* b2 = W2 + MLP_H * MLP_H;
  const float* W3 = b2 + MLP_H;
  const float* b3 = W3 + MLP_P * MLP_H;
  const float* mean = model + MLP_NPARAM;
  const float* scale = mean + MLP_F;
  const uint32_t j = __lane_id() & (MLP_H - 1);
  const bool own = __lane_id() < MLP_H;
  float x[MLP_F];
  bool ood = false;
#pragma unroll
  for (uint32_t i = 0; i < MLP_F; i++) {
    x[i] = (feat[i] - mean[i]) / scale[i];
    ood = ood || !(fabsf(x[i]) <= RADULS_MLP_OOD_Z);
  }
  if (ood) return 0xFFFFFFFFu;  // the same in every lane
  float a = b1[j];
#pragma unroll
  for (uint32_t i = 0; i < MLP_F; i++) a = fmaf(W1[j * MLP_F + i], x[i], a);
  const float h1 = a > 0.0f ? a : 0.0f;
  float a2 = b2[j];
#pragma unroll
  for (uint32_t i = 0; i < MLP_H; i++) a2 = fmaf(W2[W2T ? i * MLP_H + j : j * MLP_H + i], __shfl(h1, (int)i), a2);
  const float h2 = own && a2 > 0.0f ? a2 : 0.0f;
  uint32_t best = 0xFFFFFFFFu;
  float bv = 0.0f;
  bool finite = true;
#pragma unroll
  for (uint32_t q = 0; q < MLP_P; q++) {
    float y = own ? W3[q * MLP_H + j] * h2 : 0.0f;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) y += __shfl_xor(y, o);
    y += b3[q];
    finite = finite && isfinite(y);
    if ((feas >> q) & 1u) {
      if (best == 0xFFFFFFFFu || y < bv) { best = q; bv = y; }
    }
  }
  return finite ? best : 0xFFFFFFFFu;
}

// Procedure for a bucket of 32 < m records (single thread).
template <bool W2T = false>
__device__ __forceinline__ uint32_t choose_proc(const Plan& p, const float* model, uint64_t m, uint64_t parent,
                                                uint32_t bit, uint32_t kbits, uint32_t feas) {
  if (feas == 0) return P_LSD;
  if (__popc(feas) == 1) return __ffs(feas) - 1;
  if (p.sched_mode == RADULS_SCHED_FORCED) {
    if (p.forced_proc < MLP_P && ((feas >> p.forced_proc) & 1u)) return p.forced_proc;
  } else if (p.sched_mode == RADULS_SCHED_LEARNED && model) {
    float f[MLP_F];
    bucket_features(f, m, parent, bit, kbits, p.rec_bytes, p.key_bytes);
    uint32_t c = mlp_choose<W2T>(model, f, feas);
    if (c != 0xFFFFFFFFu) return c;
  }
  return heuristic_proc(m, parent, feas);
}

// choose_proc for a whole wavefront deciding one bucket (all lanes active,
// same arguments in every lane).
template <bool W2T = false>
__device__ __forceinline__ uint32_t choose_proc_wave(const Plan& p, const float* model, uint64_t m, uint64_t parent,
                                                     uint32_t bit, uint32_t kbits, uint32_t feas) {
  if (feas == 0) return P_LSD;
  if (__popc(feas) == 1) return __ffs(feas) - 1;
  if (p.sched_mode == RADULS_SCHED_LEARNED && model) {
    float f[MLP_F];
    bucket_features(f, m, parent, bit, kbits, p.rec_bytes, p.key_bytes);
    uint32_t c = mlp_choose_wave<W2T>(model, f, feas);
    if (c != 0xFFFFFFFFu) return c;
    return heuristic_proc(m, parent, feas);
  }
  return choose_proc<W2T>(p, model, m, parent, bit, kbits, feas);
}

}  // namespace rd
