// Slab engine for batch-dominated contractions, shared by the one-contraction
// kernel (batched.hip) and the persistent batch kernel.  See batched.hip.
#pragma once

#include "kernels.hpp"

namespace tc {

// Decode linear index r of a slab over the operand's modes (sorted by global
// stride): returns the global offset inside the slab and the LDS offset.
__device__ inline void slab_decode(const SlabDesc& d, int r, int64_t* g, int* s) {
  int64_t go = 0;
  int so = 0;
#pragma unroll 4
  for (int i = 0; i < d.n; ++i) {
    const int v = r % d.ext[i];
    r /= d.ext[i];
    go += (int64_t)v * d.gstr[i];
    so += v * d.lstr[i];
  }
  *g = go;
  *s = so;
}

// Copy the slabs of P batch indices (starting at l0, at most L - l0 of them)
// of one operand into LDS (slab size `size` doubles per point).
__device__ inline void slab_load(const double* __restrict__ X, const Offs& xl, const SlabDesc& d, int64_t l0,
                                 int np, int P, double* __restrict__ lds, int tid, int nt) {
  const int total = np * d.size;
  for (int e = tid; e < total; e += nt) {
    int p, r;
    if (d.batch_fast) {
      p = e % np;
      r = e / np;
    } else {
      p = e / d.size;
      r = e % d.size;
    }
    int64_t g;
    int s;
    slab_decode(d, r, &g, &s);
    lds[p * d.size + s] = X[off_at(xl, l0 + p) + g];
  }
  (void)P;
}

// One task: the slabs of batch indices l0 .. l0+P-1.  The layout comes by
// reference (kernel argument or global memory, never a local copy, so that
// the descriptor arrays are not moved to scratch); pointers and scalars apart.
__device__ inline void batched_slab(const BatchedParams& bp, const double* __restrict__ A,
                                    const double* __restrict__ B, double* __restrict__ C, double alpha,
                                    double beta, int64_t l0, double* smem) {
  const int tid = threadIdx.x;
  const int P = bp.P;
  const int np = (int)(bp.L - l0 < P ? bp.L - l0 : P);
  const int sA = bp.a.size, sB = bp.b.size, sC = bp.c.size;
  double* As = smem;
  double* Bs = As + P * sA;
  double* Cs = Bs + P * sB;
  slab_load(A, bp.aL, bp.a, l0, np, P, As, tid, blockDim.x);
  slab_load(B, bp.bL, bp.b, l0, np, P, Bs, tid, blockDim.x);
  __syncthreads();
  // outputs in canonical order [p][m][n]; n fastest
  const int M = bp.M, N = bp.N, K = bp.K;
  for (int o = tid; o < np * sC; o += blockDim.x) {
    const int p = o / sC, mn = o % sC;
    const int m = mn / N, n = mn % N;
    const double* a = As + p * sA + m * K;
    const double* b = Bs + p * sB + n * K;
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc += a[k] * b[k];
    Cs[o] = acc;
  }
  __syncthreads();
  const int total = np * sC;
  for (int e = tid; e < total; e += blockDim.x) {
    int p, r;
    if (bp.c.batch_fast) {
      p = e % np;
      r = e / np;
    } else {
      p = e / sC;
      r = e % sC;
    }
    int64_t g;
    int s;
    slab_decode(bp.c, r, &g, &s);
    double* dst = C + off_at(bp.cL, l0 + p) + g;
    const double v = alpha * Cs[p * sC + s];
    *dst = beta == 0.0 ? v : v + beta * *dst;
  }
  (void)M;
}


}  // namespace tc
