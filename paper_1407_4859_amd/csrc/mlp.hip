// Cost-model network kernels: forward, backward (mean squared error) and
// Adam, fp32, for the fixed shape 16 -> 64 -> 64 -> 64 -> 1 with ReLU.
//
// The paper weights its shortest path with a measured tuning profile of
// section times (section 2, third paragraph).  The learned model predicts
// that profile instead; these kernels train and evaluate it on the device.
// The matrices are tiny (a batch of a few hundred rows by 64), so every
// layer is one launch with one thread per output element and a fixed
// summation order: results are deterministic from run to run.
#include "adha_impl.h"

namespace adha {

constexpr int kIn = ADHA_N_FEATURES, kH = 64;
constexpr int kW0 = 0, kB0 = kW0 + kH * kIn, kW1 = kB0 + kH, kB1 = kW1 + kH * kH, kW2 = kB1 + kH,
              kB2 = kW2 + kH * kH, kW3 = kB2 + kH, kB3 = kW3 + kH, kParams = kB3 + 1;
static_assert(kParams == ADHA_MLP_PARAMS, "parameter count");

// Y[b][o] = act(sum_i X[b][i] * W[o][i] + bias[o]); Z (pre-activation) kept if non-null.
__global__ void mlp_layer_kernel(const float *__restrict__ X, const float *__restrict__ W,
                                 const float *__restrict__ bias, float *__restrict__ Z,
                                 float *__restrict__ Y, uint32_t B, uint32_t in, uint32_t out, int relu) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * out) return;
  const uint32_t b = t / out, o = t % out;
  float acc = bias[o];
  for (uint32_t i = 0; i < in; ++i) acc = fmaf(X[b * in + i], W[o * in + i], acc);
  if (Z) Z[t] = acc;
  Y[t] = relu ? fmaxf(acc, 0.0f) : acc;
}

// delta[b] = 2/B * (y[b] - target[b]); loss = mean of squares (one thread, fixed order).
__global__ void mlp_out_delta_kernel(const float *__restrict__ y, const float *__restrict__ target,
                                     float *__restrict__ delta, float *__restrict__ loss, uint32_t B) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) delta[b] = 2.0f / (float)B * (y[b] - target[b]);
  if (loss && b == 0) {
    float s = 0.0f;
    for (uint32_t i = 0; i < B; ++i) {
      const float d = y[i] - target[i];
      s = fmaf(d, d, s);
    }
    *loss = s / (float)B;
  }
}

// dW[o][i] = sum_b delta[b][o] * A[b][i];  db[o] = sum_b delta[b][o].
__global__ void mlp_wgrad_kernel(const float *__restrict__ delta, const float *__restrict__ A,
                                 float *__restrict__ dW, float *__restrict__ db, uint32_t B,
                                 uint32_t in, uint32_t out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < out * in) {
    const uint32_t o = t / in, i = t % in;
    float acc = 0.0f;
    for (uint32_t b = 0; b < B; ++b) acc = fmaf(delta[b * out + o], A[b * in + i], acc);
    dW[t] = acc;
  } else if (t < out * in + out) {
    const uint32_t o = t - out * in;
    float acc = 0.0f;
    for (uint32_t b = 0; b < B; ++b) acc += delta[b * out + o];
    db[o] = acc;
  }
}

// dprev[b][i] = (sum_o delta[b][o] * W[o][i]) * (Zprev[b][i] > 0).
__global__ void mlp_back_kernel(const float *__restrict__ delta, const float *__restrict__ W,
                                const float *__restrict__ Zprev, float *__restrict__ dprev, uint32_t B,
                                uint32_t in, uint32_t out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * in) return;
  const uint32_t b = t / in, i = t % in;
  float acc = 0.0f;
  for (uint32_t o = 0; o < out; ++o) acc = fmaf(delta[b * out + o], W[o * in + i], acc);
  dprev[t] = Zprev[t] > 0.0f ? acc : 0.0f;
}

__global__ void mlp_adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                                float *__restrict__ v, uint32_t n, float lr, float b1, float b2, float eps,
                                float c1, float c2) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static dim3 blocks_for(uint64_t n) { return dim3((uint32_t)((n + 255) / 256)); }

// Scratch layout for one forward + backward: Z1..Z3, A1..A3 [B][64], y [B],
// delta3 [B], d2, d1, d0 [B][64].
size_t mlp_scratch_floats(uint32_t B) { return (size_t)B * (6 * kH + 2 + 3 * kH); }

static void forward_into(const float *P, const float *x, uint32_t B, float *Z1, float *A1, float *Z2,
                         float *A2, float *Z3, float *A3, float *y, hipStream_t st) {
  hipLaunchKernelGGL(mlp_layer_kernel, blocks_for((uint64_t)B * kH), dim3(256), 0, st, x, P + kW0, P + kB0, Z1, A1, B, kIn, kH, 1);
  hipLaunchKernelGGL(mlp_layer_kernel, blocks_for((uint64_t)B * kH), dim3(256), 0, st, A1, P + kW1, P + kB1, Z2, A2, B, kH, kH, 1);
  hipLaunchKernelGGL(mlp_layer_kernel, blocks_for((uint64_t)B * kH), dim3(256), 0, st, A2, P + kW2, P + kB2, Z3, A3, B, kH, kH, 1);
  hipLaunchKernelGGL(mlp_layer_kernel, blocks_for(B), dim3(256), 0, st, A3, P + kW3, P + kB3, (float *)nullptr, y, B, kH, 1, 0);
}

adha_status mlp_forward(Ctx *ctx, const float *params, const float *x, uint32_t B, float *y, hipStream_t st) {
  (void)ctx;
  if (B == 0) return ADHA_OK;
  float *tmp = nullptr;
  ADHA_HIP(hipMallocAsync((void **)&tmp, (size_t)B * kH * 6 * sizeof(float), st));
  forward_into(params, x, B, tmp, tmp + B * kH, tmp + 2 * B * kH, tmp + 3 * B * kH, tmp + 4 * B * kH,
               tmp + 5 * B * kH, y, st);
  hipError_t e = hipGetLastError();
  (void)hipFreeAsync(tmp, st);
  if (e != hipSuccess) return fail(ADHA_ERR_DEVICE, "mlp forward launch failed: %s", hipGetErrorString(e));
  return ADHA_OK;
}

adha_status mlp_backward(Ctx *ctx, const float *P, const float *x, const float *target, uint32_t B, float *grad,
                         float *loss, float *s, size_t scratch_floats, hipStream_t st) {
  (void)ctx;
  if (B == 0) return fail(ADHA_ERR_INVALID, "batch must be positive");
  if (mlp_scratch_floats(B) > scratch_floats)
    return fail(ADHA_ERR_INVALID, "backward scratch holds %zu floats, a batch of %u needs %zu", scratch_floats, B,
                mlp_scratch_floats(B));
  float *Z1 = s, *A1 = Z1 + B * kH, *Z2 = A1 + B * kH, *A2 = Z2 + B * kH, *Z3 = A2 + B * kH,
        *A3 = Z3 + B * kH, *y = A3 + B * kH, *d3 = y + B, *d2 = d3 + B, *d1 = d2 + B * kH, *d0 = d1 + B * kH;
  forward_into(P, x, B, Z1, A1, Z2, A2, Z3, A3, y, st);
  hipLaunchKernelGGL(mlp_out_delta_kernel, blocks_for(B), dim3(256), 0, st, y, target, d3, loss, B);
  // layer 3 (64 -> 1)
  hipLaunchKernelGGL(mlp_wgrad_kernel, blocks_for(kH + 1), dim3(256), 0, st, d3, A3, grad + kW3, grad + kB3, B, kH, 1);
  hipLaunchKernelGGL(mlp_back_kernel, blocks_for((uint64_t)B * kH), dim3(256), 0, st, d3, P + kW3, Z3, d2, B, kH, 1);
  // layer 2 (64 -> 64)
  hipLaunchKernelGGL(mlp_wgrad_kernel, blocks_for(kH * kH + kH), dim3(256), 0, st, d2, A2, grad + kW2, grad + kB2, B, kH, kH);
  hipLaunchKernelGGL(mlp_back_kernel, blocks_for((uint64_t)B * kH), dim3(256), 0, st, d2, P + kW2, Z2, d1, B, kH, kH);
  // layer 1 (64 -> 64)
  hipLaunchKernelGGL(mlp_wgrad_kernel, blocks_for(kH * kH + kH), dim3(256), 0, st, d1, A1, grad + kW1, grad + kB1, B, kH, kH);
  hipLaunchKernelGGL(mlp_back_kernel, blocks_for((uint64_t)B * kH), dim3(256), 0, st, d1, P + kW1, Z1, d0, B, kH, kH);
  // layer 0 (16 -> 64)
  hipLaunchKernelGGL(mlp_wgrad_kernel, blocks_for(kH * kIn + kH), dim3(256), 0, st, d0, x, grad + kW0, grad + kB0, B, kIn, kH);
  ADHA_HIP(hipGetLastError());
  return ADHA_OK;
}

adha_status mlp_adam(Ctx *ctx, float *params, const float *grad, float *m, float *v, float lr, float b1, float b2,
                     float eps, uint32_t t, hipStream_t st) {
  (void)ctx;
  if (t == 0) return fail(ADHA_ERR_INVALID, "Adam step count starts at 1");
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(mlp_adam_kernel, blocks_for(kParams), dim3(256), 0, st, params, grad, m, v, (uint32_t)kParams,
                     lr, b1, b2, eps, c1, c2);
  ADHA_HIP(hipGetLastError());
  return ADHA_OK;
}

}  // namespace adha
