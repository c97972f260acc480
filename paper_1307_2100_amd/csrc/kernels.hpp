// Device-side parameter blocks and launchers shared by the host runtime and
// the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tc {

constexpr int kMaxRank = 16;

// Offsets of one operand along one index group: a table of per-index
// offsets, or (tab == nullptr) an affine map idx * stride.
struct Offs {
  const int64_t* tab;
  int64_t stride;
};

__host__ __device__ inline int64_t off_at(const Offs& o, int64_t i) { return o.tab ? o.tab[i] : i * o.stride; }

// C[m,n,l] = alpha * sum_k A[m,k,l] B[k,n,l] + beta * C[m,n,l] with every
// operand address split into per-group offsets (A: M,K,L; B: N,K,L; C: M,N,L).
struct GettParams {
  const double* A;
  const double* B;
  double* C;
  Offs aM, aK, aL, bN, bK, bL, cM, cN, cL;
  int64_t M, N, K, L;
  double alpha, beta;
};

// Tile configurations of the GEMM kernel (rows x columns x contracted).
struct TileCfg {
  int bm, bn, bk;
};
constexpr TileCfg kTiles[4] = {{128, 128, 16}, {64, 64, 16}, {128, 64, 16}, {64, 128, 16}};
constexpr int kNumTiles = 4;

hipError_t launch_gett_f64(const GettParams& p, int tile_id, bool a_kfast, bool b_kfast, hipStream_t s);

// Y[sum idx_i sy_i] = X[sum idx_i sx_i] over all multi-indices.
struct PermuteParams {
  const double* X;
  double* Y;
  int rank;
  int64_t ext[kMaxRank];
  int64_t sx[kMaxRank];
  int64_t sy[kMaxRank];
};
hipError_t launch_permute(const PermuteParams& p, hipStream_t s);

// C[m,n,l] <- beta * C[m,n,l] (0 when beta == 0) over all entries.
hipError_t launch_scale(double* C, Offs cM, Offs cN, Offs cL, int64_t M, int64_t N, int64_t L, double beta,
                        hipStream_t s);

}  // namespace tc
