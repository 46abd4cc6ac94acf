// raduls_kernels.hpp -- host-side launchers of the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "raduls_plan.hpp"

namespace rd {

void launch_init(const Work& w, hipStream_t s);
// zero `bytes` (a multiple of 8) at device address p with a fill kernel
void launch_zero(void* p, size_t bytes, hipStream_t s);
void launch_probe_fill(void* rec, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, uint64_t salt, uint64_t distinct,
                       hipStream_t s);
void launch_seed_single(const Plan& p, const Work& w, hipStream_t s);
void launch_seed_segments(const Plan& p, const Work& w, const uint64_t* off, uint32_t S, hipStream_t s);
void launch_level_prep(const Plan& p, const Work& w, uint32_t level, hipStream_t s);
void launch_level_hist(const Plan& p, const Work& w, uint32_t level, void* records, void* tmp, hipStream_t s);
void launch_level_scan(const Plan& p, const Work& w, uint32_t level, hipStream_t s);
void launch_tile_scan(const Plan& p, const Work& w, uint32_t level, hipStream_t s);
void launch_level_scatter(const Plan& p, const Work& w, uint32_t level, void* records, void* tmp, hipStream_t s);
void launch_order_small(const Plan& p, const Work& w, hipStream_t s);
void launch_small(const Plan& p, const Work& w, void* records, void* tmp, hipStream_t s);
void launch_small_jobs(const Plan& p, const Work& w, void* records, void* tmp, hipStream_t s);
void launch_fin_jobs(const Plan& p, const Work& w, void* records, void* tmp, hipStream_t s);
void launch_copy(const Plan& p, const Work& w, void* records, const void* tmp, hipStream_t s);
// one in-place level (k_inplace.hip), in this order: set-up and
// classification; the one-workgroup buckets; children, routing, ranges;
// permutation; cleanup
void launch_ip_classify(const Plan& p, const Work& w, const IpWork& iw, uint32_t level, void* records, int cus,
                        hipStream_t s);
void launch_ip_medium(const Plan& p, const Work& w, const IpWork& iw, uint32_t level, void* records, hipStream_t s);
void launch_ip_prepare(const Plan& p, const Work& w, const IpWork& iw, uint32_t level, void* records, int cus,
                       hipStream_t s);
void launch_ip_permute(const Plan& p, const Work& w, const IpWork& iw, uint32_t level, void* records, int cus,
                       hipStream_t s);
void launch_ip_cleanup(const Plan& p, const Work& w, const IpWork& iw, uint32_t level, void* records, int cus,
                       hipStream_t s);

// runs of equal keys in key-ordered records (k_count.hip); the workspace
// holds the control block and the look-back words
size_t runs_workspace_bytes(uint64_t n, uint32_t rec_bytes);
uint64_t runs_tiles(uint64_t n, uint32_t rec_bytes);
void launch_runs(const void* src, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, void* uniq, uint64_t* counts,
                 uint64_t* num_runs, void* ws, uint32_t spin_limit, hipStream_t s);

// pattern-prefix search over a suffix array (k_search.hip)
void launch_prefix_search(const void* text, uint64_t N, const uint32_t* sa, const void* queries, uint64_t nq,
                          uint32_t rec_bytes, uint32_t key_bytes, uint64_t* lo, uint64_t* hi, uint32_t narrow,
                          hipStream_t s);

// scheduler network
void launch_mlp_forward(const float* X, const float* theta, float* Y, uint32_t B, hipStream_t s);
void launch_mlp_loss_grad(const float* X, const float* T, const float* M, const float* theta, float* grad,
                          float* loss, float* scratch, uint32_t B, hipStream_t s);
void launch_mlp_adam(float* theta, const float* grad, float* m, float* v, uint32_t t, float lr, float b1,
                     float b2, float eps, hipStream_t s);

// scratch floats the loss/gradient launcher needs for a batch
size_t mlp_scratch_floats(uint32_t B);

// LDS bytes the single-workgroup kernel needs for a plan
uint32_t small_dynamic_lds(const Plan& p);

}  // namespace rd
