// Matrix-vector, inner-product and outer-product recipes (paper Sec. 2.2 and
// Sec. 3.2: Class 2 -> GEMV, Class 1 -> DOT, all contracted indices sliced ->
// a sum of GERs).  These contractions move many bytes per flop, so the
// kernels are built around coalescing rather than matrix cores:
//
//  * outputs-along-lanes (GEMV-N, fused GER sum): one thread owns one output
//    entry and walks the contracted index; consecutive lanes own consecutive
//    entries along the index that is stride-1 in memory, so each step of the
//    walk is one coalesced row of the matrix operand.  Summing the rank-1
//    updates in registers writes C once instead of once per update.
//  * k-along-lanes (GEMV-T, DOT): a wavefront owns one output entry (or one
//    segment of its contracted range); lanes stride along the contracted
//    stride-1 index and combine with a cross-lane reduction.  When few
//    outputs exist, the contracted range is cut into segments whose partial
//    sums go to the workspace and a second pass adds them in a fixed order
//    (deterministic).
#include <algorithm>

#include "lanes.hpp"

namespace tc {
namespace {

// One thread per (output entry, contracted segment); blockIdx.y is the
// segment.  seg == 1 writes C; otherwise the partial sum goes to
// part[s * total + o] (consecutive outputs adjacent).
__global__ __launch_bounds__(256) void lanes_over_outputs_kernel(GettParams p, int n_fastest, int64_t total,
                                                                 int64_t seg, int64_t seg_len,
                                                                 double* __restrict__ part) {
  const int64_t s = blockIdx.y;
  const int64_t k0 = s * seg_len;
  const int64_t k1 = k0 + seg_len < p.K ? k0 + seg_len : p.K;
  // grid-stride over the outputs: any output count fits the grid limits
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    int64_t m, n, l;
    if (n_fastest) {
      n = o % p.N;
      const int64_t r = o / p.N;
      m = r % p.M;
      l = r / p.M;
    } else {
      m = o % p.M;
      const int64_t r = o / p.M;
      n = r % p.N;
      l = r / p.N;
    }
    const double* __restrict__ A = p.A + off_at(p.aL, l) + off_at(p.aM, m);
    const double* __restrict__ B = p.B + off_at(p.bL, l) + off_at(p.bN, n);
    const double v = lanes_out_dot(A, B, p.aK, p.bK, k0, k1);
    if (seg > 1) {
      part[s * total + o] = v;
      continue;
    }
    double* dst = p.C + off_at(p.cL, l) + off_at(p.cM, m) + off_at(p.cN, n);
    *dst = p.beta == 0.0 ? p.alpha * v : p.alpha * v + p.beta * *dst;
  }
}

// Second pass of the segmented form: output o adds its partial sums in segment order.
__global__ __launch_bounds__(256) void sum_out_partials_kernel(GettParams p, int n_fastest, int64_t total,
                                                               int64_t seg, const double* __restrict__ part) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int64_t s = 0; s < seg; ++s) v += part[s * total + o];
    int64_t m, n, l;
    if (n_fastest) {
      n = o % p.N;
      const int64_t r = o / p.N;
      m = r % p.M;
      l = r / p.M;
    } else {
      m = o % p.M;
      const int64_t r = o / p.M;
      n = r % p.N;
      l = r / p.N;
    }
    double* dst = p.C + off_at(p.cL, l) + off_at(p.cM, m) + off_at(p.cN, n);
    *dst = p.beta == 0.0 ? p.alpha * v : p.alpha * v + p.beta * *dst;
  }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One wavefront per (output entry, contracted segment).  seg == 1 writes C;
// otherwise the partial sum goes to part[o * seg + s].
__global__ __launch_bounds__(256) void lanes_over_k_kernel(GettParams p, int64_t outputs, int64_t seg,
                                                           int64_t seg_len, double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = outputs * seg, stride = (int64_t)gridDim.x * (blockDim.x / 64);
  // grid-stride over (output, segment) pairs, uniform per wavefront
  for (int64_t w = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); w < waves; w += stride) {
    const int64_t o = w / seg, s = w % seg;
    const int64_t m = o % p.M;
    const int64_t r = o / p.M;
    const int64_t n = r % p.N;
    const int64_t l = r / p.N;
    const double* __restrict__ A = p.A + off_at(p.aL, l) + off_at(p.aM, m);
    const double* __restrict__ B = p.B + off_at(p.bL, l) + off_at(p.bN, n);
    const int64_t k0 = s * seg_len;
    const int64_t k1 = k0 + seg_len < p.K ? k0 + seg_len : p.K;
    const double v = wave_sum(lanes_k_dot(A, B, p.aK, p.bK, k0, k1, lane));
    if (lane != 0) continue;
    if (seg == 1) {
      double* dst = p.C + off_at(p.cL, l) + off_at(p.cM, m) + off_at(p.cN, n);
      *dst = p.beta == 0.0 ? p.alpha * v : p.alpha * v + p.beta * *dst;
    } else {
      part[o * seg + s] = v;
    }
  }
}

// Second pass: output o (one workgroup) adds its seg partial sums.  Thread t
// takes segments t, t+256, ... in order, then a fixed LDS tree combines the
// 256 sums, so the result does not depend on timing.
__global__ __launch_bounds__(256) void sum_partials_kernel(GettParams p, int64_t outputs, int64_t seg,
                                                           const double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t o = blockIdx.x;
  if (o >= outputs) return;
  double acc = 0.0;
  for (int64_t s = threadIdx.x; s < seg; s += 256) acc += part[o * seg + s];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double v = red[0];
  const int64_t m = o % p.M;
  const int64_t r = o / p.M;
  const int64_t n = r % p.N;
  const int64_t l = r / p.N;
  double* dst = p.C + off_at(p.cL, l) + off_at(p.cM, m) + off_at(p.cN, n);
  *dst = p.beta == 0.0 ? p.alpha * v : p.alpha * v + p.beta * *dst;
}

}  // namespace

hipError_t launch_lanes_over_outputs(const GettParams& p, bool n_fastest, int64_t seg, double* part, hipStream_t s) {
  const int64_t total = p.M * p.N * p.L;
  if (total == 0) return hipSuccess;
  if (seg < 1 || !part) seg = 1;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, kMaxGridBlocks);
  if (seg > 65535) return hipErrorInvalidConfiguration;
  const int64_t seg_len = (p.K + seg - 1) / seg;
  hipLaunchKernelGGL(lanes_over_outputs_kernel, dim3((unsigned)blocks, (unsigned)seg), dim3(256), 0, s, p,
                     n_fastest ? 1 : 0, total, seg, seg_len, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || seg == 1) return e;
  hipLaunchKernelGGL(sum_out_partials_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n_fastest ? 1 : 0, total,
                     seg, part);
  return hipGetLastError();
}

int64_t out_segments(int64_t outputs, int64_t K) {
  const int64_t blocks = (outputs + 255) / 256;
  const int64_t target_blocks = 256 * 4;
  if (blocks >= target_blocks || K < 512) return 1;
  int64_t seg = (target_blocks + blocks - 1) / blocks;
  const int64_t max_seg = K / 256;
  if (seg > max_seg) seg = max_seg;
  return seg < 1 ? 1 : seg;
}

hipError_t launch_lanes_over_k(const GettParams& p, int64_t seg, double* part, hipStream_t s) {
  const int64_t outputs = p.M * p.N * p.L;
  if (outputs == 0) return hipSuccess;
  if (seg < 1) seg = 1;
  const int64_t seg_len = (p.K + seg - 1) / seg;
  const int64_t waves = outputs * seg;
  const int64_t blocks = std::min<int64_t>((waves + 3) / 4, kMaxGridBlocks);
  hipLaunchKernelGGL(lanes_over_k_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, outputs, seg, seg_len, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || seg == 1) return e;
  if (outputs > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)outputs), dim3(256), 0, s, p, outputs, seg, part);
  return hipGetLastError();
}

int64_t k_segments(int64_t outputs, int64_t K) {
  // Enough wavefronts to cover the chip (about 8 per SIMD), but segments of at
  // least 4096 contracted indices so that the second pass stays negligible.
  const int64_t target_waves = 256 * 4 * 8;
  if (outputs >= target_waves || K <= 8192) return 1;
  int64_t seg = (target_waves + outputs - 1) / outputs;
  const int64_t max_seg = K / 4096;
  if (seg > max_seg) seg = max_seg;
  return seg < 1 ? 1 : seg;
}

}  // namespace tc
