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
#include "gett_tile.hpp"

namespace tc {
namespace {

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

}  // namespace

namespace {

template <int BM, int BN, int BK, int WGM, int WGN, bool AKF, bool BKF>
__global__ __launch_bounds__(64 * WGM * WGN) void gett_f64_kernel(GettParams p, int64_t tilesM, int64_t tilesN,
                                                                   int64_t total) {
  __shared__ __attribute__((aligned(16))) double smem[gett_lds_doubles<BM, BN, BK>()];
  int64_t l, tm, tn;
  tile_of(blockIdx.x, total, tilesM, tilesN, &l, &tm, &tn);
  gett_tile<BM, BN, BK, WGM, WGN, AKF, BKF>(p, tm * BM, tn * BN, l, smem, 0, p.K, nullptr);
}

// Split-K: workgroup (t, s) sums segment s of the contracted range for tile t.
template <int BM, int BN, int BK, int WGM, int WGN, bool AKF, bool BKF>
__global__ __launch_bounds__(64 * WGM * WGN) void gett_f64_split_kernel(GettParams p, int64_t tilesM, int64_t tilesN,
                                                                         int S, int64_t seg_len,
                                                                         double* __restrict__ parts) {
  __shared__ __attribute__((aligned(16))) double smem[gett_lds_doubles<BM, BN, BK>()];
  const int64_t t = blockIdx.x / S, sg = blockIdx.x % S;
  const int64_t per = tilesM * tilesN, l = t / per, r = t % per;
  const int64_t kb = sg * seg_len, ke = kb + seg_len < p.K ? kb + seg_len : p.K;
  gett_tile<BM, BN, BK, WGM, WGN, AKF, BKF>(p, (r % tilesM) * BM, (r / tilesM) * BN, l, smem, kb, ke,
                                           parts + (t * S + sg) * (int64_t)(BM * BN));
}

template <int BM, int BN>
__global__ __launch_bounds__(256) void gett_reduce_kernel(GettParams p, int64_t tilesM, int64_t tilesN, int S,
                                                          const double* __restrict__ parts) {
  const int64_t t = blockIdx.x;
  const int64_t per = tilesM * tilesN, l = t / per, r = t % per;
  gett_reduce_tile<BM, BN>(p, (r % tilesM) * BM, (r / tilesM) * BN, l, parts + t * S * (int64_t)(BM * BN), S);
}

template <int BM, int BN, int BK, int WGM, int WGN>
hipError_t launch_cfg(const GettParams& p, bool akf, bool bkf, int S, int64_t seg_len, double* parts,
                      hipStream_t s) {
  const int64_t tilesM = (p.M + BM - 1) / BM, tilesN = (p.N + BN - 1) / BN;
  const int64_t total = tilesM * tilesN * p.L;
  if (total == 0) return hipSuccess;
  // a grid's total thread count must stay below 2^32
  if (total * S > 0xffffffffLL / (64 * WGM * WGN)) return hipErrorInvalidConfiguration;
  dim3 block(64 * WGM * WGN);
  if (S > 1) {
    dim3 grid((unsigned)(total * S));
#define TC_SPLIT_LAUNCH(AK, BKF_)                                                                                \
  hipLaunchKernelGGL((gett_f64_split_kernel<BM, BN, BK, WGM, WGN, AK, BKF_>), grid, block, 0, s, p, tilesM, tilesN, \
                     S, seg_len, parts)
    if (akf && bkf) TC_SPLIT_LAUNCH(true, true);
    else if (akf) TC_SPLIT_LAUNCH(true, false);
    else if (bkf) TC_SPLIT_LAUNCH(false, true);
    else TC_SPLIT_LAUNCH(false, false);
#undef TC_SPLIT_LAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gett_reduce_kernel<BM, BN>), dim3((unsigned)total), dim3(256), 0, s, p, tilesM, tilesN, S,
                       parts);
    return hipGetLastError();
  }
  dim3 grid((unsigned)total);
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

hipError_t launch_gett_f64(const GettParams& p, int tile_id, bool a_kfast, bool b_kfast, int split, int64_t seg_len,
                           double* parts, hipStream_t s) {
  switch (tile_id) {
#define TC_TILE(id, bm, bn, bk, wgm, wgn) \
  case id: return launch_cfg<bm, bn, bk, wgm, wgn>(p, a_kfast, b_kfast, split, seg_len, parts, s);
    TC_GETT_TILES(TC_TILE)
#undef TC_TILE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tc
