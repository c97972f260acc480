// A small multilayer perceptron, trained and evaluated on the GPU, for the
// learned recipe/tile picker: n_in -> hidden -> hidden -> n_out, ReLU after
// both hidden layers, FP32.  It predicts the log-time of every candidate
// (recipe, tile) of a contraction from features of its layout; the plan takes
// the fastest legal prediction, and the paper's class rules stay the
// fallback.
//
// Kernels: dense forward (matrix product + bias + ReLU fused), masked
// mean-squared-error gradient, weight/bias gradients (one thread per weight,
// summing over the batch in order: deterministic), input gradient with the
// ReLU mask, and Adam.  Weights are stored row-major W[i][o].
#include <vector>

#include "kernels.hpp"

namespace tc {
namespace {

__global__ __launch_bounds__(256) void dense_fwd_kernel(const float* __restrict__ X, const float* __restrict__ W,
                                                        const float* __restrict__ b, float* __restrict__ Y, int B,
                                                        int I, int O, int relu) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * O) return;
  const int row = (int)(t / O), o = (int)(t % O);
  const float* x = X + (int64_t)row * I;
  float acc = b[o];
  for (int i = 0; i < I; ++i) acc = fmaf(x[i], W[(int64_t)i * O + o], acc);
  Y[t] = relu && acc < 0.f ? 0.f : acc;
}

// sums[0] = sum M (Y - T)^2, sums[1] = sum M over all B*O entries (one
// workgroup, fixed reduction order).
__global__ __launch_bounds__(256) void masked_sums_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                          const float* __restrict__ M, int64_t n,
                                                          float* __restrict__ sums) {
  __shared__ float s0[256], s1[256];
  float a = 0.f, c = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const float d = Y[i] - T[i];
    a = fmaf(M[i] * d, d, a);
    c += M[i];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sums[1] = s1[0];
    sums[0] = s1[0] > 0.f ? s0[0] / s1[0] : 0.f;  // the loss
  }
}

// dY = 2 M (Y - T) / sum M
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                       const float* __restrict__ M, const float* __restrict__ sums,
                                                       float* __restrict__ dY, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float cnt = sums[1] > 0.f ? sums[1] : 1.f;
  dY[i] = 2.f * M[i] * (Y[i] - T[i]) / cnt;
}

// dW[i][o] = sum_b Xin[b][i] dZ[b][o] (i < I);  db[o] = sum_b dZ[b][o] (i == I)
__global__ __launch_bounds__(256) void dense_wgrad_kernel(const float* __restrict__ Xin, const float* __restrict__ dZ,
                                                          float* __restrict__ dW, float* __restrict__ db, int B,
                                                          int I, int O) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)(I + 1) * O) return;
  const int i = (int)(t / O), o = (int)(t % O);
  float acc = 0.f;
  if (i < I) {
    for (int r = 0; r < B; ++r) acc = fmaf(Xin[(int64_t)r * I + i], dZ[(int64_t)r * O + o], acc);
    dW[(int64_t)i * O + o] = acc;
  } else {
    for (int r = 0; r < B; ++r) acc += dZ[(int64_t)r * O + o];
    db[o] = acc;
  }
}

// dX[b][i] = (sum_o dZ[b][o] W[i][o]) * (Hin[b][i] > 0): the gradient at the
// pre-activation of the previous layer (Hin is its ReLU output).
__global__ __launch_bounds__(256) void dense_xgrad_kernel(const float* __restrict__ dZ, const float* __restrict__ W,
                                                          const float* __restrict__ Hin, float* __restrict__ dX,
                                                          int B, int I, int O) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * I) return;
  const int r = (int)(t / I), i = (int)(t % I);
  float acc = 0.f;
  for (int o = 0; o < O; ++o) acc = fmaf(dZ[(int64_t)r * O + o], W[(int64_t)i * O + o], acc);
  dX[t] = Hin[t] > 0.f ? acc : 0.f;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t mlp_forward(const MlpDims& d, const float* params, const float* X, float* H1, float* H2, float* Y, int B,
                       hipStream_t s) {
  const float* W0 = params;
  const float* b0 = W0 + (int64_t)d.n_in * d.hidden;
  const float* W1 = b0 + d.hidden;
  const float* b1 = W1 + (int64_t)d.hidden * d.hidden;
  const float* W2 = b1 + d.hidden;
  const float* b2 = W2 + (int64_t)d.hidden * d.n_out;
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(blocks_for((int64_t)B * d.hidden)), dim3(256), 0, s, X, W0, b0, H1, B,
                     d.n_in, d.hidden, 1);
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(blocks_for((int64_t)B * d.hidden)), dim3(256), 0, s, H1, W1, b1, H2, B,
                     d.hidden, d.hidden, 1);
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(blocks_for((int64_t)B * d.n_out)), dim3(256), 0, s, H2, W2, b2, Y, B,
                     d.hidden, d.n_out, 0);
  return hipGetLastError();
}

hipError_t mlp_backward(const MlpDims& d, const float* params, const float* X, const float* T, const float* M,
                        const MlpScratch& w, float* grads, float* sums, int B, hipStream_t s) {
  const float* W1 = params + (int64_t)d.n_in * d.hidden + d.hidden;
  const float* W2 = W1 + (int64_t)d.hidden * d.hidden + d.hidden;
  float* gW0 = grads;
  float* gb0 = gW0 + (int64_t)d.n_in * d.hidden;
  float* gW1 = gb0 + d.hidden;
  float* gb1 = gW1 + (int64_t)d.hidden * d.hidden;
  float* gW2 = gb1 + d.hidden;
  float* gb2 = gW2 + (int64_t)d.hidden * d.n_out;
  const int64_t ny = (int64_t)B * d.n_out;
  hipLaunchKernelGGL(masked_sums_kernel, dim3(1), dim3(256), 0, s, w.Y, T, M, ny, sums);
  hipLaunchKernelGGL(mse_grad_kernel, dim3(blocks_for(ny)), dim3(256), 0, s, w.Y, T, M, sums, w.dY, ny);
  hipLaunchKernelGGL(dense_wgrad_kernel, dim3(blocks_for((int64_t)(d.hidden + 1) * d.n_out)), dim3(256), 0, s, w.H2,
                     w.dY, gW2, gb2, B, d.hidden, d.n_out);
  hipLaunchKernelGGL(dense_xgrad_kernel, dim3(blocks_for((int64_t)B * d.hidden)), dim3(256), 0, s, w.dY, W2, w.H2,
                     w.dH2, B, d.hidden, d.n_out);
  hipLaunchKernelGGL(dense_wgrad_kernel, dim3(blocks_for((int64_t)(d.hidden + 1) * d.hidden)), dim3(256), 0, s, w.H1,
                     w.dH2, gW1, gb1, B, d.hidden, d.hidden);
  hipLaunchKernelGGL(dense_xgrad_kernel, dim3(blocks_for((int64_t)B * d.hidden)), dim3(256), 0, s, w.dH2, W1, w.H1,
                     w.dH1, B, d.hidden, d.hidden);
  hipLaunchKernelGGL(dense_wgrad_kernel, dim3(blocks_for((int64_t)(d.n_in + 1) * d.hidden)), dim3(256), 0, s, X,
                     w.dH1, gW0, gb0, B, d.n_in, d.hidden);
  return hipGetLastError();
}

hipError_t mlp_adam(float* params, const float* grads, float* m, float* v, int64_t n, float lr, int step,
                    hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, s, params, grads, m, v, n, lr, b1, b2, eps, c1,
                     c2);
  return hipGetLastError();
}

}  // namespace tc
