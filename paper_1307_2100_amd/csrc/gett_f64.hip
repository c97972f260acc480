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

// Reduction of the split-K segments: workgroup (t, c) finishes entries
// 256 c .. 256 c + 255 of tile t, one entry per thread.
template <int BM, int BN>
__global__ __launch_bounds__(256) void gett_reduce_kernel(GettParams p, int64_t tilesM, int64_t tilesN, int S,
                                                          const double* __restrict__ parts) {
  constexpr int CH = (BM * BN + 255) / 256;
  const int64_t t = blockIdx.x / CH;
  const int c = (int)(blockIdx.x % CH);
  const int64_t per = tilesM * tilesN, l = t / per, r = t % per;
  gett_reduce_entry<BM, BN>(p, (r % tilesM) * BM, (r / tilesM) * BN, l, parts + t * S * (int64_t)(BM * BN), S,
                            c * 256 + (int)threadIdx.x);
}

// The same GEMM for operands whose stride-1 mode leads their row group or
// their contracted group with an even extent, every other stride even and an
// unsliced contracted group: then two consecutive entries along the stride-1
// mode are one aligned 16-byte chunk, and the tiles are copied straight from
// global memory into LDS (global_load_lds_dwordx4: lane l of a wavefront
// lands 16 bytes at the uniform LDS base + 16 l) through a ring of NS stages,
// so NS - 1 k-tiles are in flight without holding registers.
//
// One stage holds the BM + BN rows of a 16-deep k-tile as 16-row blocks of
// 2 KB, each filled by two copies:
//   * k-fast operand, copy h: lane l takes row l%16 and k = 4(l/16) + 2h, +1,
//     so that the two 16-byte reads of lane l at +16 l and +1024 + 16 l give
//     its four contracted values (k = 4q .. 4q+3, the bijection of gett_tile);
//   * row-fast operand, copy h: lane l takes k = 8h + l/8 and rows 2(l%8),
//     +1, i.e. entry (k, r) at 1024 (k/8) + 128 (k%8) + 8 r; a fragment value
//     is one 8-byte read.
// Contracted offsets come from the digits of k over the group's modes (no
// table lookup in front of a copy).
// Rows beyond the operand load a clamped in-range row (their results are
// not stored); contracted indices beyond K load a clamped in-range index and
// the fragment values of those indices are set to zero in the last k-tile.
// Waits: a wavefront's own copies of k-tile t are complete once at most
// CPW (NS - 2) copies issued after them are outstanding (vmcnt); a bare
// s_barrier then makes every wavefront's copies visible and frees the stage
// of the previous k-tile (a __syncthreads() fence would wait for every copy
// in flight).  Copies past the last k-tile repeat it into that freed stage.
template <int BM, int BN, int WGM, int WGN, bool AKF, bool BKF, int NS>
__global__ __launch_bounds__(64 * WGM * WGN) void gett_f64_dma_kernel(GettParams p, DmaK dk, int64_t tilesM,
                                                                       int64_t tilesN, int64_t total) {
  constexpr int BK = 16;
  constexpr int NW = WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int ABLK = BM / 16, BBLK = BN / 16;
  constexpr int NCOPY = 2 * (ABLK + BBLK);  // 1 KB copies per stage
  static_assert(NCOPY % NW == 0, "whole copies per wavefront");
  constexpr int CPW = NCOPY / NW;
  static_assert(CPW * (NS - 2) <= 15, "wait count fits the vmcnt field");
  constexpr int STAGE = NCOPY * 1024;  // bytes
  extern __shared__ __attribute__((aligned(16))) unsigned char dsm[];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  int64_t l, tm, tn;
  tile_of(blockIdx.x, total, tilesM, tilesN, &l, &tm, &tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const double* __restrict__ A = p.A + off_at(p.aL, l);
  const double* __restrict__ B = p.B + off_at(p.bL, l);
  const int64_t K = p.K;
  // offset of contracted index k in the kernel's A (opb false) or B
  auto koff = [&](int64_t k, bool opb) {
    if (dk.n == 1) return k * (opb ? dk.sb[0] : dk.sa[0]);
    int64_t off = 0;
    uint32_t rem = (uint32_t)k;
#pragma unroll
    for (int i = 0; i < kDmaMaxKModes; ++i) {
      if (i >= dk.n) break;
      const uint32_t e = (uint32_t)dk.ext[i];
      const uint32_t q = i + 1 < dk.n ? rem / e : 0;
      const uint32_t d = i + 1 < dk.n ? rem - q * e : rem;
      off += (int64_t)d * (opb ? dk.sb[i] : dk.sa[i]);
      rem = q;
    }
    return off;
  };

  // this lane's part of its wavefront's copies: row offset and k position in the tile
  int64_t roff[CPW];
  int kpos[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = wave + NW * j;
    const bool opb = c >= 2 * ABLK;
    const int blk = (opb ? c - 2 * ABLK : c) >> 1, h = c & 1;
    const bool kf = opb ? BKF : AKF;
    const int64_t rows = opb ? p.N : p.M;
    const int64_t r0 = (opb ? n0 : m0) + 16 * blk;
    int64_t r = kf ? r0 + (lane & 15) : r0 + 2 * (lane & 7);
    const int64_t rmax = kf ? rows - 1 : rows - 2;  // row-fast operands have an even row count
    r = r < rmax ? r : rmax;
    roff[j] = off_at(opb ? p.bN : p.aM, r);
    kpos[j] = kf ? 4 * (lane >> 4) + 2 * h : 8 * h + (lane >> 3);
  }
  // when the first contracted mode spans whole k-tiles, a tile's k digits
  // above the first are the same for every lane: one (scalar) decomposition
  // per tile and operand, plus this lane's position along the first mode
  const bool whole = dk.ext[0] % BK == 0;
  auto issue = [&](int64_t kt, int stage) {
    const int64_t kb = kt * BK;
    const int64_t ba = whole ? koff(kb, false) : 0, bb = whole ? koff(kb, true) : 0;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int c = wave + NW * j;
      const bool opb = c >= 2 * ABLK;
      const bool kf = opb ? BKF : AKF;
      int64_t k = kb + kpos[j];
      const int64_t kmax = kf ? K - 2 : K - 1;  // k-fast operands have an even K
      int64_t ko;
      if (whole && k <= kmax) {
        ko = (opb ? bb : ba) + kpos[j] * (opb ? dk.sb[0] : dk.sa[0]);
      } else {
        k = k < kmax ? k : kmax;
        ko = koff(k, opb);
      }
      const double* src = (opb ? B : A) + roff[j] + ko;
      __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)src,
                                       (void __attribute__((address_space(3)))*)(dsm + stage * STAGE + c * 1024),
                                       16, 0, 0);
    }
  };

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int fr = lane & 15, fk = lane >> 4;
  const int64_t ktiles = (K + BK - 1) / BK, last = ktiles - 1;
#pragma unroll
  for (int st = 0; st < NS - 1; ++st) issue(st < last ? st : last, st);
  for (int64_t kt = 0; kt < ktiles; ++kt) {
    __builtin_amdgcn_s_waitcnt((CPW * (NS - 2)) | (7 << 4) | (15 << 8));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    const int64_t nk = kt + NS - 1;
    issue(nk < last ? nk : last, (int)(nk % NS));
    const unsigned char* st = dsm + (kt % NS) * STAGE;
    double fa[4][TM], fb[4][TN];
    typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const unsigned char* blk = st + (wm * WM / 16 + i) * 2048;
      if constexpr (AKF) {
        const d2 lo = *(const d2*)(blk + lane * 16), hi = *(const d2*)(blk + 1024 + lane * 16);
        fa[0][i] = lo.x;
        fa[1][i] = lo.y;
        fa[2][i] = hi.x;
        fa[3][i] = hi.y;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = 4 * fk + s;
          fa[s][i] = *(const double*)(blk + (k >> 3) * 1024 + (k & 7) * 128 + fr * 8);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const unsigned char* blk = st + (2 * ABLK + 2 * (wn * WN / 16 + j)) * 1024;
      if constexpr (BKF) {
        const d2 lo = *(const d2*)(blk + lane * 16), hi = *(const d2*)(blk + 1024 + lane * 16);
        fb[0][j] = lo.x;
        fb[1][j] = lo.y;
        fb[2][j] = hi.x;
        fb[3][j] = hi.y;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = 4 * fk + s;
          fb[s][j] = *(const double*)(blk + (k >> 3) * 1024 + (k & 7) * 128 + fr * 8);
        }
      }
    }
    if (kt == last && (K & (BK - 1))) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (kt * BK + 4 * fk + s < K) continue;
#pragma unroll
        for (int i = 0; i < TM; ++i) fa[s][i] = 0.0;
#pragma unroll
        for (int j = 0; j < TN; ++j) fb[s][j] = 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][i], fb[s][j], acc[i][j], 0, 0, 0);
  }
  // the repeated copies of the tail must land before the workgroup's LDS is released
  __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));

  // epilogue: accumulator element r of a 16x16 block holds D[lane/16 + 4r][lane%16]
  double* __restrict__ C = p.C + off_at(p.cL, l);
  int64_t cn[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int64_t n = n0 + wn * WN + j * 16 + fr;
    cn[j] = n < p.N ? off_at(p.cN, n) : -1;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + wm * WM + i * 16 + fk + 4 * r;
      if (m >= p.M) continue;
      const int64_t cm = off_at(p.cM, m);
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

template <int BM, int BN, int WGM, int WGN, bool AKF, bool BKF, int NS>
hipError_t launch_dma_one(const GettParams& p, const DmaK& dk, int64_t tilesM, int64_t tilesN, int64_t total,
                          hipStream_t s) {
  constexpr int bytes = NS * 2 * (BM / 16 + BN / 16) * 1024;
  static std::atomic<uint64_t> allowed{0};
  const hipError_t e =
      allow_dynamic_lds((const void*)gett_f64_dma_kernel<BM, BN, WGM, WGN, AKF, BKF, NS>, bytes, allowed);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((gett_f64_dma_kernel<BM, BN, WGM, WGN, AKF, BKF, NS>), dim3((unsigned)total),
                     dim3(64 * WGM * WGN), bytes, s, p, dk, tilesM, tilesN, total);
  return hipGetLastError();
}

template <int BM, int BN, int WGM, int WGN>
hipError_t launch_dma(const GettParams& p, const DmaK& dk, bool akf, bool bkf, hipStream_t s) {
  const int64_t tilesM = (p.M + BM - 1) / BM, tilesN = (p.N + BN - 1) / BN;
  const int64_t total = tilesM * tilesN * p.L;
  if (total == 0) return hipSuccess;
  if (total > 0xffffffffLL / (64 * WGM * WGN)) return hipErrorInvalidConfiguration;
  if (dk.n < 1 || dk.n > kDmaMaxKModes || p.K > 0x7fffffffLL) return hipErrorInvalidValue;
  constexpr int NS = 3;
  if (akf && bkf) return launch_dma_one<BM, BN, WGM, WGN, true, true, NS>(p, dk, tilesM, tilesN, total, s);
  if (akf) return launch_dma_one<BM, BN, WGM, WGN, true, false, NS>(p, dk, tilesM, tilesN, total, s);
  if (bkf) return launch_dma_one<BM, BN, WGM, WGN, false, true, NS>(p, dk, tilesM, tilesN, total, s);
  return launch_dma_one<BM, BN, WGM, WGN, false, false, NS>(p, dk, tilesM, tilesN, total, s);
}

template <int BM, int BN, int BK, int WGM, int WGN>
hipError_t launch_cfg(const GettParams& p, bool akf, bool bkf, int S, int64_t seg_len, double* parts,
                      hipStream_t s) {
  const int64_t tilesM = (p.M + BM - 1) / BM, tilesN = (p.N + BN - 1) / BN;
  const int64_t total = tilesM * tilesN * p.L;
  if (total == 0) return hipSuccess;
  // a grid's total thread count must stay below 2^32
  if (total * S > 0xffffffffLL / (64 * WGM * WGN)) return hipErrorInvalidConfiguration;
  if (S > 1 && total * ((BM * BN + 255) / 256) > 0xffffffffLL / 256) return hipErrorInvalidConfiguration;
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
    constexpr int CH = (BM * BN + 255) / 256;
    hipLaunchKernelGGL((gett_reduce_kernel<BM, BN>), dim3((unsigned)(total * CH)), dim3(256), 0, s, p, tilesM,
                       tilesN, S, parts);
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
                           double* parts, hipStream_t s, const DmaK* dma) {
  if (dma && split == 1 && tile_id == kDmaTile) {
    // same 256 x 128 x 16 tile, as 8 wavefronts of 64 x 64 (the copies hold no
    // registers, so each wavefront can keep a larger block of C)
    static_assert(kTiles[kDmaTile].bm == 256 && kTiles[kDmaTile].bn == 128 && kTiles[kDmaTile].bk == 16,
                  "the copy-fed kernel is instantiated for this tile");
    return launch_dma<256, 128, 4, 2>(p, *dma, a_kfast, b_kfast, s);
  }
  switch (tile_id) {
#define TC_TILE(id, bm, bn, bk, wgm, wgn) \
  case id: return launch_cfg<bm, bn, bk, wgm, wgn>(p, a_kfast, b_kfast, split, seg_len, parts, s);
    TC_GETT_TILES(TC_TILE)
#undef TC_TILE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tc
