// k_mlp.hip -- training kernels of the scheduler network (float32).
//
// Network: a1 = W1 x + b1, h1 = relu(a1), a2 = W2 h1 + b2, h2 = relu(a2),
// y = W3 h2 + b3.  Loss: masked mean squared error sum(M (y-t)^2) / sum(M).
// Gradients by back-propagation; the ReLU derivative is 1 where a > 0.
// Every sum over the batch runs in index order in one thread, so repeated
// runs give identical bits.
#include "raduls_kernels.hpp"
#include "sched_dev.hpp"

namespace rd {

constexpr uint32_t F = MLP_F, H = MLP_H, P = MLP_P;
constexpr uint32_t OFF_W1 = 0, OFF_B1 = OFF_W1 + H * F, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
                   OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + P * H;
// per-sample scratch: x, h1, da1, h2, da2, dy, loss term
constexpr uint32_t S_X = 0, S_H1 = S_X + F, S_DA1 = S_H1 + H, S_H2 = S_DA1 + H, S_DA2 = S_H2 + H, S_DY = S_DA2 + H,
                   S_L = S_DY + P, S_STRIDE = S_L + 1;

size_t mlp_scratch_floats(uint32_t B) { return (size_t)B * S_STRIDE + 64; }

__device__ __forceinline__ void mlp_forward_one(const float* __restrict__ th, const float* x, float* a1, float* a2,
                                                float* y) {
  for (uint32_t j = 0; j < H; j++) {
    float a = th[OFF_B1 + j];
    for (uint32_t i = 0; i < F; i++) a = fmaf(th[OFF_W1 + j * F + i], x[i], a);
    a1[j] = a;
  }
  for (uint32_t j = 0; j < H; j++) {
    float a = th[OFF_B2 + j];
    for (uint32_t i = 0; i < H; i++) a = fmaf(th[OFF_W2 + j * H + i], a1[i] > 0.0f ? a1[i] : 0.0f, a);
    a2[j] = a;
  }
  for (uint32_t q = 0; q < P; q++) {
    float a = th[OFF_B3 + q];
    for (uint32_t i = 0; i < H; i++) a = fmaf(th[OFF_W3 + q * H + i], a2[i] > 0.0f ? a2[i] : 0.0f, a);
    y[q] = a;
  }
}

__global__ void k_mlp_forward(const float* X, const float* th, float* Y, uint32_t B) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float x[F], a1[H], a2[H], y[P];
  for (uint32_t i = 0; i < F; i++) x[i] = X[(size_t)b * F + i];
  mlp_forward_one(th, x, a1, a2, y);
  for (uint32_t q = 0; q < P; q++) Y[(size_t)b * P + q] = y[q];
}

// sum(M) in index order (one thread); stored at scratch[B * S_STRIDE].
__global__ void k_mlp_mask_sum(const float* M, uint32_t B, float* scratch) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.0f;
  for (size_t i = 0; i < (size_t)B * P; i++) s += M[i];
  scratch[(size_t)B * S_STRIDE] = s;
}

// Forward and backward vectors of one sample.
__global__ void k_mlp_sample(const float* X, const float* T, const float* M, const float* th, uint32_t B,
                             float* scratch) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float msum = scratch[(size_t)B * S_STRIDE];
  float* s = scratch + (size_t)b * S_STRIDE;
  float x[F], a1[H], a2[H], y[P];
  for (uint32_t i = 0; i < F; i++) { x[i] = X[(size_t)b * F + i]; s[S_X + i] = x[i]; }
  mlp_forward_one(th, x, a1, a2, y);
  float dy[P];
  float lterm = 0.0f;
  for (uint32_t q = 0; q < P; q++) {
    float mk = M[(size_t)b * P + q];
    float d = mk > 0.0f ? y[q] - T[(size_t)b * P + q] : 0.0f;
    lterm += mk * d * d;
    dy[q] = msum > 0.0f ? 2.0f * mk * d / msum : 0.0f;
    s[S_DY + q] = dy[q];
  }
  s[S_L] = lterm;
  float da2[H];
  for (uint32_t j = 0; j < H; j++) {
    float g = 0.0f;
    for (uint32_t q = 0; q < P; q++) g = fmaf(th[OFF_W3 + q * H + j], dy[q], g);
    da2[j] = a2[j] > 0.0f ? g : 0.0f;
    s[S_H2 + j] = a2[j] > 0.0f ? a2[j] : 0.0f;
    s[S_DA2 + j] = da2[j];
  }
  for (uint32_t i = 0; i < H; i++) {
    float g = 0.0f;
    for (uint32_t j = 0; j < H; j++) g = fmaf(th[OFF_W2 + j * H + i], da2[j], g);
    s[S_DA1 + i] = a1[i] > 0.0f ? g : 0.0f;
    s[S_H1 + i] = a1[i] > 0.0f ? a1[i] : 0.0f;
  }
}

// One thread per parameter (plus one for the loss): sum over the batch in
// index order.
__global__ void k_mlp_reduce(uint32_t B, const float* scratch, float* grad, float* loss) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > MLP_NPARAM) return;
  uint32_t u, v;   // grad = sum_b s[u] * (v == 0xFFFF ? 1 : s[v])
  const uint32_t ONE = 0xFFFFu;
  if (k == MLP_NPARAM) {
    float L = 0.0f;
    for (uint32_t b = 0; b < B; b++) L += scratch[(size_t)b * S_STRIDE + S_L];
    const float msum = scratch[(size_t)B * S_STRIDE];
    loss[0] = msum > 0.0f ? L / msum : 0.0f;
    return;
  }
  if (k < OFF_B1) { u = S_DA1 + (k - OFF_W1) / F; v = S_X + (k - OFF_W1) % F; }
  else if (k < OFF_W2) { u = S_DA1 + (k - OFF_B1); v = ONE; }
  else if (k < OFF_B2) { u = S_DA2 + (k - OFF_W2) / H; v = S_H1 + (k - OFF_W2) % H; }
  else if (k < OFF_W3) { u = S_DA2 + (k - OFF_B2); v = ONE; }
  else if (k < OFF_B3) { u = S_DY + (k - OFF_W3) / H; v = S_H2 + (k - OFF_W3) % H; }
  else { u = S_DY + (k - OFF_B3); v = ONE; }
  float g = 0.0f;
  for (uint32_t b = 0; b < B; b++) {
    const float* s = scratch + (size_t)b * S_STRIDE;
    g = v == ONE ? g + s[u] : fmaf(s[u], s[v], g);
  }
  grad[k] = g;
}

__global__ void k_mlp_adam(float* th, const float* g, float* m, float* v, uint32_t n, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float gk = g[k];
  float mk = b1 * m[k] + (1.0f - b1) * gk;
  float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  float mh = mk / c1;
  float vh = vk / c2;
  th[k] -= lr * mh / (sqrtf(vh) + eps);
}

void launch_mlp_forward(const float* X, const float* theta, float* Y, uint32_t B, hipStream_t s) {
  k_mlp_forward<<<(B + 127) / 128, 128, 0, s>>>(X, theta, Y, B);
}

void launch_mlp_loss_grad(const float* X, const float* T, const float* M, const float* theta, float* grad, float* loss,
                          float* scratch, uint32_t B, hipStream_t s) {
  k_mlp_mask_sum<<<1, 64, 0, s>>>(M, B, scratch);
  if (B) k_mlp_sample<<<(B + 127) / 128, 128, 0, s>>>(X, T, M, theta, B, scratch);
  k_mlp_reduce<<<(MLP_NPARAM + 1 + 127) / 128, 128, 0, s>>>(B, scratch, grad, loss);
}

void launch_mlp_adam(float* theta, const float* grad, float* m, float* v, uint32_t t, float lr, float b1, float b2,
                     float eps, hipStream_t s) {
  // bias corrections 1 - beta^t, computed on the host in double precision
  float c1 = (float)(1.0 - pow((double)b1, (double)t));
  float c2 = (float)(1.0 - pow((double)b2, (double)t));
  k_mlp_adam<<<(MLP_NPARAM + 127) / 128, 128, 0, s>>>(theta, grad, m, v, MLP_NPARAM, lr, b1, b2, eps, c1, c2);
}

}  // namespace rd
