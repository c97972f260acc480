// FP64 MFMA GEMM over gathered tensor operands ("GETT").
//
// Computes C[m,n,l] = alpha * sum_k A[m,k,l] B[k,n,l] + beta * C[m,n,l]
// where m, n, k, l are linear indices of the four index groups (free indices
// of the kernel's A, free indices of its B, contracted, batch) and every
// operand address is the sum of per-group offsets.  This is the direct-GEMM
// recipe of the paper (Sec. 3.2, Class 3.2): instead of looping over slices
// and calling GEMM on each, all sliced indices are folded into the GEMM's own
// row, column and reduction loops, so one launch covers the whole
// contraction.  Loads gather straight from the tensors through the offset
// tables into LDS; the operand whose stride-1 mode leads the contracted
// group is staged k-contiguous, the other row-contiguous, so that consecutive
// lanes always read consecutive addresses when a stride-1 mode allows it.
//
// Workgroup: 256 threads = 4 wavefronts in a 2 x 2 arrangement; each
// wavefront owns a (BM/2) x (BN/2) block of C held in FP64 MFMA accumulators
// (v_mfma_f64_16x16x4f64: 16x16 outputs per instruction, 4 per lane).
#include "kernels.hpp"

namespace tc {
namespace {

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

// Global-to-register loader for one operand tile (R rows x BK contracted)
// with NT threads.
template <int R, int BK, bool KF, int NT>
struct Loader {
  static constexpr int E = R * BK / NT;  // elements per thread
  static_assert(E >= 1 && R * BK == E * NT, "tile must split evenly over the threads");
  static_assert(KF ? (NT % BK == 0) : (NT % R == 0), "loader mapping needs whole rows per pass");
  int64_t roff[KF ? E : 1];  // row offsets (row-fast: one row per thread)
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

  __device__ inline void load(const double* __restrict__ X, const Offs& xk, int64_t k0, int64_t K, int tid) {
    if constexpr (KF) {
      int64_t k = k0 + tid % BK;
      int64_t ko = k < K ? off_at(xk, k) : -1;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = (ko >= 0 && roff[e] >= 0) ? X[roff[e] + ko] : 0.0;
    } else {
      // all lanes of a wavefront share one k when R is a multiple of 64: keep it scalar
      const int kf = R % 64 == 0 ? __builtin_amdgcn_readfirstlane(tid / R) : tid / R;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int64_t k = k0 + kf + (NT / R) * e;
        int64_t ko = k < K ? off_at(xk, k) : -1;
        v[e] = (ko >= 0 && roff[0] >= 0) ? X[roff[0] + ko] : 0.0;
      }
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

// Bijective map of the linear workgroup id onto (batch, tile row, tile
// column): the batch index is the slowest, tiles within a batch follow the
// XCD-aware order of xcd_tile.
__device__ inline void tile_of(int64_t bid, int64_t total, int64_t tilesM, int64_t tilesN, int64_t* l,
                               int64_t* tm, int64_t* tn) {
  const int64_t per = tilesM * tilesN;
  // XCD chunks over the whole grid, then split into (batch, tile)
  const int64_t q = total / 8, r = total % 8;
  const int64_t xcd = bid % 8, loc = bid / 8;
  int64_t t = xcd < r ? xcd * (q + 1) + loc : r * (q + 1) + (xcd - r) * q + loc;
  *l = t / per;
  t -= *l * per;
  // banded order inside the batch: identity chunking (xcd_tile with one XCD)
  constexpr int64_t G = 8;
  const int64_t band = t / (G * tilesN);
  const int64_t first = band * G;
  const int64_t gs = tilesM - first < G ? tilesM - first : G;
  const int64_t w = t - band * G * tilesN;
  *tm = first + w % gs;
  *tn = w / gs;
}

template <int BM, int BN, int BK, int WGM, int WGN, bool AKF, bool BKF>
__global__ __launch_bounds__(64 * WGM * WGN) void gett_f64_kernel(GettParams p, int64_t tilesM, int64_t tilesN,
                                                                   int64_t total) {
  constexpr int NT = 64 * WGM * WGN;
  using SA_ = Stage<BM, BK, AKF>;
  using SB_ = Stage<BN, BK, BKF>;
  __shared__ __attribute__((aligned(16))) double sA[2][SA_::SIZE];
  __shared__ __attribute__((aligned(16))) double sB[2][SB_::SIZE];

  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 16, TN = WN / 16;
  static_assert(BK % 16 == 0 && TM >= 1 && TN >= 1, "tile shape");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;

  int64_t l, tm, tn;
  tile_of(blockIdx.x, total, tilesM, tilesN, &l, &tm, &tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;

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

  const int64_t ktiles = (p.K + BK - 1) / BK;
  if (ktiles > 0) {
    la.load(A, p.aK, 0, p.K, tid);
    lb.load(B, p.bK, 0, p.K, tid);
    la.store(sA[0], tid);
    lb.store(sB[0], tid);
  }
  __syncthreads();

  const int fr = lane & 15;   // row (A) / column (B) inside a 16x16 block
  const int fk = lane >> 4;   // lane quarter: which 4 contracted indices of a 16-chunk
  for (int64_t kt = 0; kt < ktiles; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < ktiles;
    if (more) {
      la.load(A, p.aK, (kt + 1) * BK, p.K, tid);
      lb.load(B, p.bK, (kt + 1) * BK, p.K, tid);
    }
    Frags<BM, BK, AKF, TM> fa;
    Frags<BN, BK, BKF, TN> fb;
    fa.read(sA[cur], wm * WM, fr, fk);
    fb.read(sB[cur], wn * WN, fr, fk);
#pragma unroll
    for (int s = 0; s < BK / 4; ++s)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.f[s][i], fb.f[s][j], acc[i][j], 0, 0, 0);
    if (more) {
      la.store(sA[cur ^ 1], tid);
      lb.store(sB[cur ^ 1], tid);
    }
    __syncthreads();
  }

  // Epilogue: v_mfma_f64_16x16x4f64 leaves D[lane/16 + 4*r][lane % 16] of each
  // 16x16 block in accumulator element r (rows interleaved by four).
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

template <int BM, int BN, int BK, int WGM, int WGN>
hipError_t launch_cfg(const GettParams& p, bool akf, bool bkf, hipStream_t s) {
  const int64_t tilesM = (p.M + BM - 1) / BM, tilesN = (p.N + BN - 1) / BN;
  const int64_t total = tilesM * tilesN * p.L;
  if (total == 0) return hipSuccess;
  if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)total), block(64 * WGM * WGN);
  if (akf && bkf)
    hipLaunchKernelGGL((gett_f64_kernel<BM, BN, BK, WGM, WGN, true, true>), grid, block, 0, s, p, tilesM, tilesN,
                       total);
  else if (akf)
    hipLaunchKernelGGL((gett_f64_kernel<BM, BN, BK, WGM, WGN, true, false>), grid, block, 0, s, p, tilesM, tilesN,
                       total);
  else if (bkf)
    hipLaunchKernelGGL((gett_f64_kernel<BM, BN, BK, WGM, WGN, false, true>), grid, block, 0, s, p, tilesM, tilesN,
                       total);
  else
    hipLaunchKernelGGL((gett_f64_kernel<BM, BN, BK, WGM, WGN, false, false>), grid, block, 0, s, p, tilesM,
                       tilesN, total);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gett_f64(const GettParams& p, int tile_id, bool a_kfast, bool b_kfast, hipStream_t s) {
  switch (tile_id) {
#define TC_TILE(id, bm, bn, bk, wgm, wgn) \
  case id: return launch_cfg<bm, bn, bk, wgm, wgn>(p, a_kfast, b_kfast, s);
    TC_GETT_TILES(TC_TILE)
#undef TC_TILE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tc
