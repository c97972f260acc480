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
// lands 16 bytes at the uniform LDS base + 16 l) through a ring of three
// stages, without holding registers.
//
// One stage holds the BM + BN rows of a 16-deep k-tile as 16-row blocks of
// 2 KB, each filled by two copies:
//   * k-fast operand, copy h: lane l takes row l%16 and k = 4(l/16) + 2h, +1,
//     so that the 16-byte chunks of lane l at +16 l and +1024 + 16 l hold its
//     four contracted values (k = 4q .. 4q+3, the bijection of gett_tile);
//   * row-fast operand, copy h: lane l takes k = 8h + l/8 and rows 2(l%8),
//     +1, i.e. entry (k, r) at 1024 (k/8) + 128 (k%8) + 8 r.
// MFMA step s of a k-tile (s = 0..3) takes contracted index 4q + s from lane
// group q; its fragments are one 8-byte LDS read per 16-row block.
//
// Schedule.  Tile t sits in stage t mod 3.  Each wavefront double-buffers the
// fragments of one step: the MFMAs of step s run while the reads of step s+1
// are issued between them, so LDS latency hides behind the matrix cores.  The
// barrier of a k-tile sits between its steps 1 and 2: before it every
// wavefront waits for its own copies of tile t+1 (vmcnt(0): the only vector
// memory operations in flight), after it tile t+1 is visible to all and every
// wavefront is done with stage (t-1) mod 3, which the copies of tile t+2 --
// spread between the MFMAs of step 2 -- then refill.  Copies cost two 64-bit
// adds each: a per-lane base address fixed per workgroup plus the tile's
// contracted offset, a uniform value (digits of k over the contracted modes,
// valid while the first contracted extent is a multiple of 16).  Tiles whose
// copies need per-lane contracted digits (a first contracted extent not a
// multiple of 16, or the clamped last tile of a ragged range) go through a
// plain loop.  Rows beyond the operand load a clamped in-range row (their
// results are not stored); contracted indices beyond K load a clamped index
// and the fragment values of those indices are zeroed in the last k-tile.
template <int BM, int BN, int WGM, int WGN, bool AKF, bool BKF>
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
  static_assert(CPW <= 15, "wait count fits the vmcnt field");
  constexpr int STAGE = NCOPY * 1024;  // bytes
  constexpr int NM = TM * TN;          // MFMAs per step
  constexpr int NR = TM + TN;          // fragment reads per step
  extern __shared__ __attribute__((aligned(16))) unsigned char dsm[];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  int64_t l, tm, tn;
  tile_of(blockIdx.x, total, tilesM, tilesN, &l, &tm, &tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const double* const A = p.A + off_at(p.aL, l);
  const double* const B = p.B + off_at(p.bL, l);
  const int64_t K = p.K;
  // the wavefront index as a uniform value: a copy's LDS address (M0) is then
  // scalar arithmetic
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  const int64_t sa0 = dk.sa[0], sb0 = dk.sb[0];
  // offset of contracted index k in the kernel's A (koff_a) or B (koff_b)
  auto koff_a = [&](int64_t k) -> int64_t {
    if (dk.n == 1) return k * sa0;
    int64_t off = 0;
    uint32_t rem = (uint32_t)k;
#pragma unroll
    for (int i = 0; i < kDmaMaxKModes; ++i) {
      if (i >= dk.n) break;
      const uint32_t e = (uint32_t)dk.ext[i];
      const uint32_t q = i + 1 < dk.n ? rem / e : 0;
      off += (int64_t)(i + 1 < dk.n ? rem - q * e : rem) * dk.sa[i];
      rem = q;
    }
    return off;
  };
  auto koff_b = [&](int64_t k) -> int64_t {
    if (dk.n == 1) return k * sb0;
    int64_t off = 0;
    uint32_t rem = (uint32_t)k;
#pragma unroll
    for (int i = 0; i < kDmaMaxKModes; ++i) {
      if (i >= dk.n) break;
      const uint32_t e = (uint32_t)dk.ext[i];
      const uint32_t q = i + 1 < dk.n ? rem / e : 0;
      off += (int64_t)(i + 1 < dk.n ? rem - q * e : rem) * dk.sb[i];
      rem = q;
    }
    return off;
  };

  // copy j of this wavefront is copy c = wave + NW j of the stage: operand,
  // 16-row block and half h; base[j] = its source address at k-tile 0
  const double* base[CPW];
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
    const int kp = kf ? 4 * (lane >> 4) + 2 * h : 8 * h + (lane >> 3);
    if (opb)
      base[j] = B + off_at(p.bN, r) + kp * sb0;
    else
      base[j] = A + off_at(p.aM, r) + kp * sa0;
  }
  const int64_t ktiles = (K + BK - 1) / BK, last = ktiles - 1;
  const bool whole = dk.ext[0] % BK == 0;
  // copy j of tile t, uniform contracted offsets (whole first mode, tile in range)
  auto copy_fast = [&](int j, int64_t ta, int64_t tb, int stage) {
    const int c = wave_u + NW * j;
    const bool opb = c >= 2 * ABLK;
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)(base[j] + (opb ? tb : ta)),
                                     (void __attribute__((address_space(3)))*)(dsm + stage * STAGE + c * 1024), 16,
                                     0, 0);
  };
  // copy j of tile t with this lane's own contracted digits (clamped to K)
  auto copy_slow = [&](int j, int64_t t, int stage) {
    const int c = wave_u + NW * j;
    const bool opb = c >= 2 * ABLK;
    const int h = c & 1;
    const bool kf = opb ? BKF : AKF;
    const int kp = kf ? 4 * (lane >> 4) + 2 * h : 8 * h + (lane >> 3);
    int64_t k = t * BK + kp;
    const int64_t kmax = kf ? K - 2 : K - 1;  // k-fast operands have an even K
    k = k < kmax ? k : kmax;
    const double* src = opb ? base[j] - kp * sb0 + koff_b(k) : base[j] - kp * sa0 + koff_a(k);
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)src,
                                     (void __attribute__((address_space(3)))*)(dsm + stage * STAGE + c * 1024), 16,
                                     0, 0);
  };
  auto issue_all = [&](int64_t t, int stage) {
    if (whole && (t < last || K % BK == 0)) {
      const int64_t ta = koff_a(t * BK), tb = koff_b(t * BK);
#pragma unroll
      for (int j = 0; j < CPW; ++j) copy_fast(j, ta, tb, stage);
    } else {
#pragma unroll
      for (int j = 0; j < CPW; ++j) copy_slow(j, t, stage);
    }
  };

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int fr = lane & 15, fk = lane >> 4;
  // LDS byte offset of this lane's fragment of step 0 in the first block of
  // its rows (k-fast: k = 4 fk at +16 lane; row-fast: (k, r) = (4 fk, fr));
  // step s adds (s / 2) 1024 + (s % 2) 8, resp. 128 s
  const int nf_lane = (fk >> 1) * 1024 + (fk & 1) * 512 + fr * 8;
  const int a_lds = (wm * WM / 16) * 2048 + (AKF ? lane * 16 : nf_lane);
  const int b_lds = (2 * ABLK + 2 * (wn * WN / 16)) * 1024 + (BKF ? lane * 16 : nf_lane);
  auto rd1 = [&](int stage, int s, int q, double (&fa)[TM], double (&fb)[TN]) {
    if (q < TM) {
      const int so = AKF ? (s >> 1) * 1024 + (s & 1) * 8 : s * 128;
      fa[q] = *(const double*)(dsm + stage * STAGE + a_lds + q * 2048 + so);
    } else {
      const int so = BKF ? (s >> 1) * 1024 + (s & 1) * 8 : s * 128;
      fb[q - TM] = *(const double*)(dsm + stage * STAGE + b_lds + (q - TM) * 2048 + so);
    }
  };
  auto rd_all = [&](int stage, int s, double (&fa)[TM], double (&fb)[TN]) {
#pragma unroll
    for (int q = 0; q < NR; ++q) rd1(stage, s, q, fa, fb);
  };
  auto mfma1 = [&](const double (&fa)[TM], const double (&fb)[TN], int q) {
    acc[q / TN][q % TN] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[q / TN], fb[q % TN], acc[q / TN][q % TN], 0, 0, 0);
  };
  auto mm = [&](const double (&fa)[TM], const double (&fb)[TN]) {
#pragma unroll
    for (int q = 0; q < NM; ++q) mfma1(fa, fb, q);
  };
  // the MFMAs of one step (fa, fb) with the reads of step (stage, s) into
  // (ga, gb) spread over its first two thirds and, when CP, the fast copies
  // of a k-tile spread over all of it (the scheduler keeps this order)
  auto mm_rd = [&](bool cp, const double (&fa)[TM], const double (&fb)[TN], int stage, int s, double (&ga)[TM],
                   double (&gb)[TN], int64_t ta, int64_t tb, int cstage) {
    constexpr int SPAN = (2 * NM) / 3;
#pragma unroll
    for (int q = 0; q < NM; ++q) {
      mfma1(fa, fb, q);
      if (q < SPAN && q * NR / SPAN != (q + 1) * NR / SPAN) {
        __builtin_amdgcn_sched_barrier(0);
        rd1(stage, s, q * NR / SPAN, ga, gb);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (cp && q * CPW / NM != (q + 1) * CPW / NM) {
        __builtin_amdgcn_sched_barrier(0);
        copy_fast(q * CPW / NM, ta, tb, cstage);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };
  // wait for this wavefront's copies in flight, then for every wavefront
  auto sync = [&]() {
    __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));  // vmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

  issue_all(0, 0);
  issue_all(last < 1 ? last : 1, 1);
  __builtin_amdgcn_s_waitcnt(CPW | (7 << 4) | (15 << 8));  // this wavefront's copies of tile 0
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
  double f0a[TM], f0b[TN], f1a[TM], f1b[TN];
  rd_all(0, 0, f0a, f0b);
  int scur = 0, snext = 1, sfree = 2;
  int64_t kt = 0;
  // tiles whose copies of tile kt + 2 take the uniform offsets (kt + 2 < last)
  const int64_t fast_end = whole && last > 2 ? last - 2 : 0;
  // contracted offsets (ta, tb) and digits of tile kt + 2, advanced by 16
  // per tile (the first extent is a multiple of 16, so a carry leaves the
  // first digit at 0)
  int64_t ta = 0, tb = 0;
  uint32_t dig[kDmaMaxKModes] = {0u, 0u, 0u, 0u};
  if (fast_end > 0) {
    uint32_t rem = 2u * BK;
    for (int i = 0; i < dk.n; ++i) {
      const uint32_t e = (uint32_t)dk.ext[i];
      dig[i] = i + 1 < dk.n ? rem % e : rem;
      rem = i + 1 < dk.n ? rem / e : 0u;
      ta += (int64_t)dig[i] * dk.sa[i];
      tb += (int64_t)dig[i] * dk.sb[i];
    }
  }
  for (; kt < fast_end; ++kt) {
    __builtin_amdgcn_sched_barrier(0);
    mm_rd(false, f0a, f0b, scur, 1, f1a, f1b, 0, 0, 0);        // step 0, reads step 1
    __builtin_amdgcn_sched_barrier(0);
    mm_rd(false, f1a, f1b, scur, 2, f0a, f0b, 0, 0, 0);        // step 1, reads step 2
    __builtin_amdgcn_sched_barrier(0);
    sync();
    __builtin_amdgcn_sched_barrier(0);
    mm_rd(true, f0a, f0b, scur, 3, f1a, f1b, ta, tb, sfree);    // step 2, reads step 3, copies
    __builtin_amdgcn_sched_barrier(0);
    mm_rd(false, f1a, f1b, snext, 0, f0a, f0b, 0, 0, 0);       // step 3, reads step 0 of tile kt + 1
    __builtin_amdgcn_sched_barrier(0);
    const int t = scur;
    scur = snext;
    snext = sfree;
    sfree = t;
    dig[0] += BK;
    ta += BK * sa0;
    tb += BK * sb0;
    for (int i = 0; i + 1 < dk.n && dig[i] >= (uint32_t)dk.ext[i]; ++i) {
      dig[i] = 0u;
      ta += dk.sa[i + 1] - dk.ext[i] * dk.sa[i];
      tb += dk.sb[i + 1] - dk.ext[i] * dk.sb[i];
      ++dig[i + 1];
    }
  }
  for (; kt < last; ++kt) {
    mm_rd(false, f0a, f0b, scur, 1, f1a, f1b, 0, 0, 0);
    mm_rd(false, f1a, f1b, scur, 2, f0a, f0b, 0, 0, 0);
    sync();
    if (kt + 2 <= last) issue_all(kt + 2, sfree);
    mm_rd(false, f0a, f0b, scur, 3, f1a, f1b, 0, 0, 0);
    mm_rd(false, f1a, f1b, snext, 0, f0a, f0b, 0, 0, 0);
    const int t = scur;
    scur = snext;
    snext = sfree;
    sfree = t;
  }
  // the last k-tile, with the steps past K zeroed
  const bool ragged = (K & (BK - 1)) != 0;
  auto zero = [&](int s, double (&fa)[TM], double (&fb)[TN]) {
    if (ragged && last * BK + 4 * fk + s >= K) {
#pragma unroll
      for (int i = 0; i < TM; ++i) fa[i] = 0.0;
#pragma unroll
      for (int j = 0; j < TN; ++j) fb[j] = 0.0;
    }
  };
  rd_all(scur, 1, f1a, f1b);
  zero(0, f0a, f0b);
  zero(1, f1a, f1b);
  mm(f0a, f0b);
  rd_all(scur, 2, f0a, f0b);
  mm(f1a, f1b);
  rd_all(scur, 3, f1a, f1b);
  zero(2, f0a, f0b);
  zero(3, f1a, f1b);
  mm(f0a, f0b);
  mm(f1a, f1b);
  // with a single k-tile the prologue's second copy of it may still be in
  // flight: it must land before the workgroup's LDS is released
  __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));

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

template <int BM, int BN, int WGM, int WGN, bool AKF, bool BKF>
hipError_t launch_dma_one(const GettParams& p, const DmaK& dk, int64_t tilesM, int64_t tilesN, int64_t total,
                          hipStream_t s) {
  constexpr int bytes = 3 * 2 * (BM / 16 + BN / 16) * 1024;
  static std::atomic<uint64_t> allowed{0};
  const hipError_t e =
      allow_dynamic_lds((const void*)gett_f64_dma_kernel<BM, BN, WGM, WGN, AKF, BKF>, bytes, allowed);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((gett_f64_dma_kernel<BM, BN, WGM, WGN, AKF, BKF>), dim3((unsigned)total), dim3(64 * WGM * WGN),
                     bytes, s, p, dk, tilesM, tilesN, total);
  return hipGetLastError();
}

template <int BM, int BN, int WGM, int WGN>
hipError_t launch_dma(const GettParams& p, const DmaK& dk, bool akf, bool bkf, hipStream_t s) {
  const int64_t tilesM = (p.M + BM - 1) / BM, tilesN = (p.N + BN - 1) / BN;
  const int64_t total = tilesM * tilesN * p.L;
  if (total == 0) return hipSuccess;
  if (total > 0xffffffffLL / (64 * WGM * WGN)) return hipErrorInvalidConfiguration;
  if (dk.n < 1 || dk.n > kDmaMaxKModes || p.K > 0x7fffffffLL) return hipErrorInvalidValue;
  if (akf && bkf) return launch_dma_one<BM, BN, WGM, WGN, true, true>(p, dk, tilesM, tilesN, total, s);
  if (akf) return launch_dma_one<BM, BN, WGM, WGN, true, false>(p, dk, tilesM, tilesN, total, s);
  if (bkf) return launch_dma_one<BM, BN, WGM, WGN, false, true>(p, dk, tilesM, tilesN, total, s);
  return launch_dma_one<BM, BN, WGM, WGN, false, false>(p, dk, tilesM, tilesN, total, s);
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
  if (dma && split == 1 && (tile_id == kDmaTile || tile_id == kDmaTileWide)) {
    // 8 wavefronts of 64 x 64 (256 x 128, 128 x 256) or 96 x 48 (192 x 192):
    // the copies hold no registers, so each wavefront keeps a large block of C
    static_assert(kTiles[kDmaTile].bm == 256 && kTiles[kDmaTile].bn == 128 && kTiles[kDmaTileWide].bm == 128 &&
                      kTiles[kDmaTileWide].bn == 256,
                  "the copy-fed kernel stands in for these tiles");
    switch (dma->shape) {
      case kDma256x128: return launch_dma<256, 128, 4, 2>(p, *dma, a_kfast, b_kfast, s);
      case kDma128x256: return launch_dma<128, 256, 2, 4>(p, *dma, a_kfast, b_kfast, s);
      case kDma192x192: return launch_dma<192, 192, 2, 4>(p, *dma, a_kfast, b_kfast, s);
      default: return hipErrorInvalidValue;
    }
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
