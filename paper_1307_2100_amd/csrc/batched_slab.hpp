// Slab engine for batch-dominated contractions, shared by the one-contraction
// kernel (batched.hip) and the persistent batch kernel.  See batched.hip.
#pragma once

#include "kernels.hpp"

namespace tc {

// Decode linear index r of a slab over the operand's modes (sorted by global
// stride): returns the global offset inside the slab and the LDS offset.
__device__ inline void slab_decode(const SlabDesc& d, uint32_t r, int64_t* g, int* s) {
  int64_t go = 0;
  int so = 0;
  for (int i = 0; i < d.n; ++i) {
    const uint32_t q = fdiv(r, d.div[i]);
    const int v = (int)(r - q * d.div[i].d);
    r = q;
    go += (int64_t)v * d.gstr[i];
    so += v * d.lstr[i];
  }
  *g = go;
  *s = so;
}

// Copy the slabs of np <= P batch indices starting at l0 of one operand into
// LDS (slab size d.size doubles per point).  Each thread issues 8
// independent loads before storing any, so that enough loads are in flight
// to cover the memory latency.
__device__ inline void slab_load(const double* __restrict__ X, const Offs& xl, const SlabDesc& d, int64_t l0,
                                 int np, int P, const FastDiv& P_div, double* __restrict__ lds, int tid, int nt) {
  constexpr int U = 8;
  const int total = P * d.size;
  for (int base = tid; base < total; base += nt * U) {
    double v[U];
    int dst[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * nt;
      uint32_t p, r;
      if (d.batch_fast) {  // consecutive lanes: consecutive batch indices
        r = fdiv((uint32_t)e, P_div);
        p = (uint32_t)e - r * (uint32_t)P;
      } else {             // consecutive lanes: consecutive entries of one slab
        p = fdiv((uint32_t)e, d.size_div);
        r = (uint32_t)e - p * (uint32_t)d.size;
      }
      dst[u] = -1;
      v[u] = 0.0;
      if (e < total && (int)p < np) {
        int64_t g;
        int s;
        slab_decode(d, r, &g, &s);
        dst[u] = (int)p * d.size + s;
        v[u] = X[off_at(xl, l0 + p) + g];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (dst[u] >= 0) lds[dst[u]] = v[u];
  }
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
  slab_load(A, bp.aL, bp.a, l0, np, P, bp.P_div, As, tid, blockDim.x);
  slab_load(B, bp.bL, bp.b, l0, np, P, bp.P_div, Bs, tid, blockDim.x);
  __syncthreads();
  // outputs in canonical order [p][m][n]; n fastest
  const int K = bp.K;
  for (int o = tid; o < np * sC; o += blockDim.x) {
    const uint32_t p = fdiv((uint32_t)o, bp.sC_div), mn = (uint32_t)o - p * (uint32_t)sC;
    const uint32_t m = fdiv(mn, bp.N_div), n = mn - m * (uint32_t)bp.N;
    const double* a = As + p * sA + m * K;
    const double* b = Bs + p * sB + n * K;
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc += a[k] * b[k];
    Cs[o] = acc;
  }
  __syncthreads();
  const int total = P * sC;
  for (int e = tid; e < total; e += blockDim.x) {
    uint32_t p, r;
    if (bp.c.batch_fast) {
      r = fdiv((uint32_t)e, bp.P_div);
      p = (uint32_t)e - r * (uint32_t)P;
    } else {
      p = fdiv((uint32_t)e, bp.c.size_div);
      r = (uint32_t)e - p * (uint32_t)sC;
    }
    if ((int)p >= np) continue;
    int64_t g;
    int s;
    slab_decode(bp.c, r, &g, &s);
    double* dst = C + off_at(bp.cL, l0 + p) + g;
    const double v = alpha * Cs[p * sC + s];
    *dst = beta == 0.0 ? v : v + beta * *dst;
  }
}


}  // namespace tc
