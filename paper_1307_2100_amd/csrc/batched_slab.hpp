// Slab engine for batch-dominated contractions, shared by the one-contraction
// kernel (batched.hip) and the persistent batch kernel.  See batched.hip.
#pragma once

#include "kernels.hpp"

namespace tc {

// Decode linear index r of a slab over the operand's modes (sorted by global
// stride): returns the global offset inside the slab and the LDS offset.
TC_DEV void slab_decode(const SlabDesc& d, uint32_t r, int64_t* g, int* s) {
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
// LDS (slab size d.size doubles per point): in storage order for a dense
// operand, in the canonical order otherwise.  Each thread issues 8
// independent loads before storing any, so that enough loads are in flight
// to cover the memory latency.
TC_DEV void slab_load(const double* __restrict__ X, const Offs& xl, const SlabDesc& d, int64_t l0,
                                 int np, int P, const FastDiv& P_div, double* __restrict__ lds, int tid, int nt) {
  constexpr int U = 8;
  if (d.contig) {
    // the np slabs are one contiguous run: plain streaming copy, two entries per load when aligned
    const double* __restrict__ src = X + l0 * d.size;
    const int n = np * d.size;
    typedef double d2 __attribute__((ext_vector_type(2)));
    int done = 0;
    if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
      const int n2 = n >> 1;
      for (int base = tid; base < n2; base += nt * U) {
        d2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (base + u * nt < n2) v[u] = reinterpret_cast<const d2*>(src)[base + u * nt];
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (base + u * nt < n2) {
            lds[2 * (base + u * nt)] = v[u].x;
            lds[2 * (base + u * nt) + 1] = v[u].y;
          }
      }
      done = 2 * n2;
    }
    for (int e = done + tid; e < n; e += nt) lds[e] = src[e];
    return;
  }
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
        if (d.dense) {
          g = (int64_t)r * d.s0;
          s = (int)r;
        } else {
          slab_decode(d, r, &g, &s);
        }
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
// LDS: P slabs of A, of B and of C, then the contracted offsets of A and B.
TC_DEV void batched_slab(const BatchedParams& bp, const double* __restrict__ A,
                                    const double* __restrict__ B, double* __restrict__ C, double alpha,
                                    double beta, int64_t l0, double* smem) {
  const int tid = threadIdx.x;
  const int P = bp.P;
  const int np = (int)(bp.L - l0 < P ? bp.L - l0 : P);
  const int sA = bp.a.size, sB = bp.b.size, sC = bp.c.size;
  const int K = bp.K;
  double* As = smem;
  double* Bs = As + P * sA;
  double* Cs = Bs + P * sB;
  int* kA = reinterpret_cast<int*>(Cs + P * sC);
  int* kB = kA + K;
  for (int k = tid; k < K; k += blockDim.x) {
    kA[k] = (int)off_at(bp.ak, k);
    kB[k] = (int)off_at(bp.bk, k);
  }
  slab_load(A, bp.aL, bp.a, l0, np, P, bp.P_div, As, tid, blockDim.x);
  slab_load(B, bp.bL, bp.b, l0, np, P, bp.P_div, Bs, tid, blockDim.x);
  __syncthreads();
  // one thread per output entry (p, m, n), n fastest
  for (int o = tid; o < np * sC; o += blockDim.x) {
    const uint32_t p = fdiv((uint32_t)o, bp.sC_div), mn = (uint32_t)o - p * (uint32_t)sC;
    const uint32_t m = fdiv(mn, bp.N_div), n = mn - m * (uint32_t)bp.N;
    const double* a = As + p * sA + off_at(bp.am, m);
    const double* b = Bs + p * sB + off_at(bp.bn, n);
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc += a[kA[k]] * b[kB[k]];
    Cs[p * sC + off_at(bp.cm, m) + off_at(bp.cn, n)] = acc;
  }
  __syncthreads();
  if (bp.c.contig) {
    double* __restrict__ dst = C + l0 * sC;
    for (int e = tid; e < np * sC; e += blockDim.x) {
      const double v = alpha * Cs[e];
      dst[e] = beta == 0.0 ? v : v + beta * dst[e];
    }
    return;
  }
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
    if (bp.c.dense) {
      g = (int64_t)r * bp.c.s0;
      s = (int)r;
    } else {
      slab_decode(bp.c, r, &g, &s);
    }
    double* dst = C + off_at(bp.cL, l0 + p) + g;
    const double v = alpha * Cs[p * sC + s];
    *dst = beta == 0.0 ? v : v + beta * *dst;
  }
}


}  // namespace tc
