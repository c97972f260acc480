// Storage reordering (the COPY of the paper's COPY+GEMM, Sec. 3.1 F1) and
// the beta-scaling used when a contraction has an empty sum.
//
// The permute stages 32 x 32 tiles through LDS: a tile spans X's stride-1
// mode (so reads are coalesced) and Y's stride-1 mode (so writes are), the
// transposition happening in LDS.  Unlike the paper's slice-by-slice copy,
// the whole operand is reordered in one pass, so every byte is read once and
// written once (its footnote on amortising the copy over all slices).
#include <algorithm>

#include "kernels.hpp"

namespace tc {
namespace {

constexpr int T = 32;

struct PermPlan {
  const double* X;
  double* Y;
  int nout;                  // modes other than a and b
  int64_t oext[kMaxRank];
  int64_t osx[kMaxRank];
  int64_t osy[kMaxRank];
  int64_t ea, eb;            // extents of the tile modes
  int64_t sxa, sxb, sya, syb;
  int64_t ta, tb;            // tiles along a and b
};

__global__ __launch_bounds__(256) void permute_tile_kernel(PermPlan p) {
  __shared__ double tile[T][T + 1];
  int64_t bid = blockIdx.x;
  const int64_t ia = bid % p.ta;
  bid /= p.ta;
  const int64_t ib = bid % p.tb;
  int64_t outer = bid / p.tb;
  int64_t ox = 0, oy = 0;
  for (int i = 0; i < p.nout; ++i) {
    int64_t v = outer % p.oext[i];
    outer /= p.oext[i];
    ox += v * p.osx[i];
    oy += v * p.osy[i];
  }
  const int tx = threadIdx.x & (T - 1), ty = threadIdx.x / T;  // 32 x 8
  const int64_t a0 = ia * T, b0 = ib * T;
#pragma unroll
  for (int r = 0; r < T; r += 8) {
    int64_t a = a0 + tx, b = b0 + ty + r;
    if (a < p.ea && b < p.eb) tile[ty + r][tx] = p.X[ox + a * p.sxa + b * p.sxb];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < T; r += 8) {
    int64_t a = a0 + ty + r, b = b0 + tx;
    if (a < p.ea && b < p.eb) p.Y[oy + a * p.sya + b * p.syb] = tile[tx][ty + r];
  }
}

// X and Y share their fastest mode: plain strided copy, one element per thread.
__global__ __launch_bounds__(256) void permute_flat_kernel(PermuteParams p, int64_t total) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e, ox = 0, oy = 0;
    for (int d = 0; d < p.rank; ++d) {
      int64_t v = i % p.ext[d];
      i /= p.ext[d];
      ox += v * p.sx[d];
      oy += v * p.sy[d];
    }
    p.Y[oy] = p.X[ox];
  }
}

__global__ __launch_bounds__(256) void scale_kernel(double* C, Offs cM, Offs cN, Offs cL, int64_t M, int64_t N,
                                                    int64_t total, double beta) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t n = i % N;
    int64_t r = i / N;
    int64_t m = r % M;
    int64_t l = r / M;
    double* d = C + off_at(cM, m) + off_at(cN, n) + off_at(cL, l);
    *d = beta == 0.0 ? 0.0 : beta * *d;
  }
}

}  // namespace

hipError_t launch_permute(const PermuteParams& p, hipStream_t s) {
  int64_t total = 1;
  for (int d = 0; d < p.rank; ++d) total *= p.ext[d];
  if (total == 0) return hipSuccess;
  // a: the mode X reads fastest; b: the mode Y writes fastest
  int a = -1, b = -1;
  for (int d = 0; d < p.rank; ++d) {
    if (p.ext[d] <= 1) continue;
    if (a < 0 || p.sx[d] < p.sx[a]) a = d;
    if (b < 0 || p.sy[d] < p.sy[b]) b = d;
  }
  if (a < 0 || a == b) {
    // reorder the modes so that the shared fast mode decodes first
    PermuteParams q = p;
    if (a > 0) {
      std::swap(q.ext[0], q.ext[a]);
      std::swap(q.sx[0], q.sx[a]);
      std::swap(q.sy[0], q.sy[a]);
    }
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, kMaxGridBlocks);
    hipLaunchKernelGGL(permute_flat_kernel, dim3((unsigned)blocks), dim3(256), 0, s, q, total);
    return hipGetLastError();
  }
  PermPlan pp{};
  pp.X = p.X;
  pp.Y = p.Y;
  pp.ea = p.ext[a];
  pp.eb = p.ext[b];
  pp.sxa = p.sx[a];
  pp.sxb = p.sx[b];
  pp.sya = p.sy[a];
  pp.syb = p.sy[b];
  pp.ta = (pp.ea + T - 1) / T;
  pp.tb = (pp.eb + T - 1) / T;
  int64_t outer = 1;
  for (int d = 0; d < p.rank; ++d) {
    if (d == a || d == b) continue;
    pp.oext[pp.nout] = p.ext[d];
    pp.osx[pp.nout] = p.sx[d];
    pp.osy[pp.nout] = p.sy[d];
    pp.nout++;
    outer *= p.ext[d];
  }
  int64_t blocks = pp.ta * pp.tb * outer;
  if (blocks > 0xffffffffLL / 256) return hipErrorInvalidConfiguration;  // total threads below 2^32
  hipLaunchKernelGGL(permute_tile_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pp);
  return hipGetLastError();
}

hipError_t launch_scale(double* C, Offs cM, Offs cN, Offs cL, int64_t M, int64_t N, int64_t L, double beta,
                        hipStream_t s) {
  int64_t total = M * N * L;
  if (total == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, kMaxGridBlocks);
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks), dim3(256), 0, s, C, cM, cN, cL, M, N, total, beta);
  return hipGetLastError();
}

}  // namespace tc
