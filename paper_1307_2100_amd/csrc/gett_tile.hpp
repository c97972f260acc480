// The FP64 MFMA tile engine shared by the one-contraction GEMM kernel and
// the persistent batch kernel: staging layouts, loaders, fragment reads and
// the per-tile main loop.  See gett_f64.hip for the design.
#pragma once

#include "kernels.hpp"

namespace tc {

typedef double d4 __attribute__((ext_vector_type(4)));

// LDS layout of one staged operand tile with R rows and BK contracted
// indices: k-contiguous when the operand is k-fast, row-contiguous otherwise.
// The k-contiguous rows are padded to an even length so that a lane can read
// four consecutive k values with two 16-byte LDS reads.
template <int R, int BK, bool KF>
struct Stage {
  static constexpr int LD = KF ? (BK + 2) : (R + 4);
  static constexpr int SIZE = KF ? R * LD : BK * LD;
  __device__ static inline int at(int k, int r) { return KF ? r * LD + k : k * LD + r; }
};

// LDS (in doubles) a GEMM tile needs, whatever the operands' fastness.
template <int BM, int BN, int BK>
__host__ __device__ constexpr int gett_lds_doubles() {
  constexpr int a = Stage<BM, BK, true>::SIZE > Stage<BM, BK, false>::SIZE ? Stage<BM, BK, true>::SIZE
                                                                           : Stage<BM, BK, false>::SIZE;
  constexpr int b = Stage<BN, BK, true>::SIZE > Stage<BN, BK, false>::SIZE ? Stage<BN, BK, true>::SIZE
                                                                           : Stage<BN, BK, false>::SIZE;
  return 2 * (a + b);
}

// Global-to-register loader for one operand tile (R rows x BK contracted)
// with NT threads.  The contracted-index offsets of a tile are looked up
// (koffs) one tile ahead of its data loads (load), so that a table lookup and
// the load that depends on it never sit back to back on the critical path.
template <int R, int BK, bool KF, int NT>
struct Loader {
  static constexpr int E = R * BK / NT;  // elements per thread
  static_assert(E >= 1 && R * BK == E * NT, "tile must split evenly over the threads");
  static_assert(KF ? (NT % BK == 0) : (NT % R == 0), "loader mapping needs whole rows per pass");
  int64_t roff[KF ? E : 1];  // row offsets (row-fast: one row per thread), -1 beyond the rows
  int64_t ko[KF ? 1 : E];    // contracted offsets of the next tile to load, -1 beyond K
  double v[E];

  __device__ inline void init(const Offs& xr, int64_t r0, int64_t rows, int tid) {
    if constexpr (KF) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int64_t r = r0 + tid / BK + (NT / BK) * e;
        roff[e] = r < rows ? off_at(xr, r) : -1;
      }
    } else {
      int64_t r = r0 + tid % R;
      roff[0] = r < rows ? off_at(xr, r) : -1;
    }
  }

  __device__ inline void koffs(const Offs& xk, int64_t k0, int64_t K, int tid) {
    if constexpr (KF) {
      int64_t k = k0 + tid % BK;
      ko[0] = k < K ? off_at(xk, k) : -1;
    } else {
      // all lanes of a wavefront share one k when R is a multiple of 64: keep it scalar
      const int kf = R % 64 == 0 ? __builtin_amdgcn_readfirstlane(tid / R) : tid / R;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int64_t k = k0 + kf + (NT / R) * e;
        ko[e] = k < K ? off_at(xk, k) : -1;
      }
    }
  }

  __device__ inline void load(const double* __restrict__ X) {
    if constexpr (KF) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = (ko[0] >= 0 && roff[e] >= 0) ? X[roff[e] + ko[0]] : 0.0;
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = (ko[e] >= 0 && roff[0] >= 0) ? X[roff[0] + ko[e]] : 0.0;
    }
  }

  __device__ inline void store(double* __restrict__ s, int tid) const {
    using S = Stage<R, BK, KF>;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if constexpr (KF) {
        s[S::at(tid % BK, tid / BK + (NT / BK) * e)] = v[e];
      } else {
        s[S::at(tid / R + (NT / R) * e, tid % R)] = v[e];
      }
    }
  }
};

// Fragment reads for one 4-deep MFMA step.  Inside a BK tile the lanes of
// quarter q (lane / 16) take contracted indices 4q .. 4q+3 of each 16-wide
// chunk, step s using index 4q + s: any bijection of k inside the tile gives
// the same sum, and this one makes a lane's four values adjacent in a
// k-contiguous stage.
template <int R, int BK, bool KF, int T>
struct Frags {
  double f[BK / 4][T];
  __device__ inline void read(const double* __restrict__ s, int row0, int fr, int fk) {
    using S = Stage<R, BK, KF>;
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
      for (int c = 0; c < BK / 16; ++c) {
        const int r = row0 + t * 16 + fr;
        const int kb = c * 16 + fk * 4;
        if constexpr (KF) {
          typedef double d2 __attribute__((ext_vector_type(2)));
          const d2 lo = *reinterpret_cast<const d2*>(s + S::at(kb, r));
          const d2 hi = *reinterpret_cast<const d2*>(s + S::at(kb + 2, r));
          f[c * 4 + 0][t] = lo.x;
          f[c * 4 + 1][t] = lo.y;
          f[c * 4 + 2][t] = hi.x;
          f[c * 4 + 3][t] = hi.y;
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) f[c * 4 + q][t] = s[S::at(kb + q, r)];
        }
      }
    }
  }
};

// One BM x BN tile of C at (m0, n0) in batch entry l, summing the contracted
// range [kb, ke).  With part == nullptr the tile is finished (alpha, beta) into
// C; otherwise its raw sums go to part[m_local * BN + n_local] (a split-K
// segment, to be reduced by gett_reduce_tile).
template <int BM, int BN, int BK, int WGM, int WGN, bool AKF, bool BKF>
TC_DEV void gett_tile(const GettParams& p, int64_t m0, int64_t n0, int64_t l, double* smem,
                                 int64_t kb, int64_t ke, double* __restrict__ part) {
  constexpr int NT = 64 * WGM * WGN;
  using SA_ = Stage<BM, BK, AKF>;
  using SB_ = Stage<BN, BK, BKF>;
  // two stages of each operand: A at smem + stage * SA_SIZE, B after both A stages
  double* const sA0 = smem;
  double* const sB0 = smem + 2 * SA_::SIZE;

  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 16, TN = WN / 16;
  static_assert(BK % 16 == 0 && TM >= 1 && TN >= 1, "tile shape");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;


  const double* __restrict__ A = p.A + off_at(p.aL, l);
  const double* __restrict__ B = p.B + off_at(p.bL, l);

  Loader<BM, BK, AKF, NT> la;
  Loader<BN, BK, BKF, NT> lb;
  la.init(p.aM, m0, p.M, tid);
  lb.init(p.bN, n0, p.N, tid);

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // Small tiles have little MFMA work per k-tile to hide a table lookup
  // followed by the load it feeds: they look the offsets up one tile ahead.
  // Large tiles keep the registers and look up just before loading.
  constexpr bool LOOK = BM * BN <= 64 * 64;
  const int64_t ktiles = ke > kb ? (ke - kb + BK - 1) / BK : 0;
  if (ktiles > 0) {
    la.koffs(p.aK, kb, ke, tid);
    lb.koffs(p.bK, kb, ke, tid);
    la.load(A);
    lb.load(B);
    if (LOOK && ktiles > 1) {
      la.koffs(p.aK, kb + BK, ke, tid);
      lb.koffs(p.bK, kb + BK, ke, tid);
    }
    la.store(sA0, tid);
    lb.store(sB0, tid);
  }
  __syncthreads();

  const int fr = lane & 15;   // row (A) / column (B) inside a 16x16 block
  const int fk = lane >> 4;   // lane quarter: which 4 contracted indices of a 16-chunk
  for (int64_t kt = 0; kt < ktiles; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < ktiles;
    if (more) {
      if constexpr (!LOOK) {
        la.koffs(p.aK, kb + (kt + 1) * BK, ke, tid);
        lb.koffs(p.bK, kb + (kt + 1) * BK, ke, tid);
      }
      la.load(A);
      lb.load(B);
      if (LOOK && kt + 2 < ktiles) {
        la.koffs(p.aK, kb + (kt + 2) * BK, ke, tid);
        lb.koffs(p.bK, kb + (kt + 2) * BK, ke, tid);
      }
    }
    Frags<BM, BK, AKF, TM> fa;
    Frags<BN, BK, BKF, TN> fb;
    fa.read(sA0 + cur * SA_::SIZE, wm * WM, fr, fk);
    fb.read(sB0 + cur * SB_::SIZE, wn * WN, fr, fk);
#pragma unroll
    for (int s = 0; s < BK / 4; ++s)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.f[s][i], fb.f[s][j], acc[i][j], 0, 0, 0);
    if (more) {
      la.store(sA0 + (cur ^ 1) * SA_::SIZE, tid);
      lb.store(sB0 + (cur ^ 1) * SB_::SIZE, tid);
    }
    __syncthreads();
  }

  // Epilogue: v_mfma_f64_16x16x4f64 leaves D[lane/16 + 4*r][lane % 16] of each
  // 16x16 block in accumulator element r (rows interleaved by four).
  if (part) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          part[(wm * WM + i * 16 + fk + 4 * r) * BN + wn * WN + j * 16 + fr] = acc[i][j][r];
    return;
  }
  double* __restrict__ C = p.C + off_at(p.cL, l);
  int64_t cn[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    int64_t n = n0 + wn * WN + j * 16 + fr;
    cn[j] = n < p.N ? off_at(p.cN, n) : -1;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int64_t m = m0 + wm * WM + i * 16 + fk + 4 * r;
      if (m >= p.M) continue;
      int64_t cm = off_at(p.cM, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        if (cn[j] < 0) continue;
        double* dst = C + cm + cn[j];
        double v = p.alpha * acc[i][j][r];
        if (p.beta != 0.0) v += p.beta * *dst;
        *dst = v;
      }
    }
  }
}

// Finishes a split-K tile: adds the S segment sums of each entry in segment
// order (a fixed order, so the result does not depend on which workgroup
// finished last) and writes alpha * sum + beta * C.
template <int BM, int BN>
TC_DEV void gett_reduce_tile(const GettParams& p, int64_t m0, int64_t n0, int64_t l,
                                        const double* __restrict__ parts, int S) {
  double* __restrict__ C = p.C + off_at(p.cL, l);
  for (int e = threadIdx.x; e < BM * BN; e += blockDim.x) {
    const int64_t m = m0 + e / BN, n = n0 + e % BN;
    if (m >= p.M || n >= p.N) continue;
    double v = 0.0;
    for (int sg = 0; sg < S; ++sg) v += parts[(int64_t)sg * BM * BN + e];
    double* dst = C + off_at(p.cM, m) + off_at(p.cN, n);
    v *= p.alpha;
    if (p.beta != 0.0) v += p.beta * *dst;
    *dst = v;
  }
}

// Entry e (row-major within the tile) of a split-K tile: the S segment sums
// added in segment order, as in gett_reduce_tile, with the loads issued eight
// at a time ahead of their (unchanged, in-order) additions.
template <int BM, int BN>
TC_DEV void gett_reduce_entry(const GettParams& p, int64_t m0, int64_t n0, int64_t l,
                              const double* __restrict__ parts, int S, int e) {
  const int64_t m = m0 + e / BN, n = n0 + e % BN;
  if (e >= BM * BN || m >= p.M || n >= p.N) return;
  double v = 0.0;
  int sg = 0;
  for (; sg + 8 <= S; sg += 8) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = parts[(int64_t)(sg + u) * BM * BN + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += x[u];
  }
  for (; sg < S; ++sg) v += parts[(int64_t)sg * BM * BN + e];
  double* dst = p.C + off_at(p.cL, l) + off_at(p.cM, m) + off_at(p.cN, n);
  v *= p.alpha;
  if (p.beta != 0.0) v += p.beta * *dst;
  *dst = v;
}

}  // namespace tc
