// Device-side parameter blocks and launchers shared by the host runtime and
// the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "../../include/tc.h"

// Raises a kernel's dynamic LDS limit to `bytes` once per device (`done`
// holds one bit per device id; concurrent first calls repeat the same
// idempotent request).
inline hipError_t allow_dynamic_lds(const void* fn, int bytes, std::atomic<uint64_t>& done) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const uint64_t bit = dev < 64 ? (uint64_t)1 << dev : 0;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_release);
  return e;
}

// Grid-stride kernels launch at most this many workgroups (a grid's total
// thread count must stay below 2^32).
constexpr int64_t kMaxGridBlocks = 1 << 20;

// Device helpers are always inlined: a real call would cost the calling
// kernel its register budget (the callee cannot share the caller's).
#define TC_DEV __device__ __attribute__((always_inline)) inline

namespace tc {

constexpr int kMaxRank = 16;

// Records `msg` as the calling thread's tc_last_error() text and returns s
// (for entry points defined outside the main ABI source).
tc_status set_error(tc_status s, const char* msg);

// Offsets of one operand along one index group: a table of per-index
// offsets, or (tab == nullptr) an affine map idx * stride.
// Division by a divisor fixed at plan time, for 0 <= n < 2^31: multiply by
// ceil(2^p / d) and shift (p = 31 + ceil(log2 d)); d = 1 divides trivially.
struct FastDiv {
  uint32_t d, mul, shift;
};
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{d, 0u, 0u};
  if (d <= 1) return f;
  int l = 0;
  while ((1u << l) < d) ++l;
  const uint64_t p = 31 + (uint64_t)l;
  f.mul = (uint32_t)(((1ull << p) + d - 1) / d);
  f.shift = (uint32_t)(p - 32);
  return f;
}
TC_DEV uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return f.d == 1 ? n : (__umulhi(n, f.mul) >> f.shift);
}

// Offsets of one operand along one index group: a table of per-index
// offsets, or (tab == nullptr) an affine map idx * stride.
struct Offs {
  const int64_t* tab;
  int64_t stride;
};

__host__ __device__ inline int64_t off_at(const Offs& o, int64_t i) { return o.tab ? o.tab[i] : i * o.stride; }

// Bijective map of a linear workgroup id onto (tile row, tile column).
// Workgroups are dealt round-robin to the 8 XCDs; consecutive tiles are
// gathered on one XCD (sharing its L2), and within an XCD tiles are walked in
// bands of 8 tile rows so that neighbours reuse the same rows and columns.
TC_DEV void xcd_tile(int64_t bid, int64_t total, int64_t tilesM, int64_t tilesN, int64_t* tm,
                                int64_t* tn) {
  const int64_t q = total / 8, r = total % 8;
  const int64_t xcd = bid % 8, loc = bid / 8;
  int64_t t = xcd < r ? xcd * (q + 1) + loc : r * (q + 1) + (xcd - r) * q + loc;
  constexpr int64_t G = 8;
  const int64_t band = t / (G * tilesN);
  const int64_t first = band * G;
  const int64_t gs = tilesM - first < G ? tilesM - first : G;
  const int64_t w = t - band * G * tilesN;
  *tm = first + w % gs;
  *tn = w / gs;
}

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

// Tile configurations of the GEMM kernel: (id, rows, columns, contracted
// depth, wavefronts along rows, wavefronts along columns).
#define TC_GETT_TILES(X)      \
  X(0, 128, 128, 16, 2, 2)    \
  X(1, 64, 64, 16, 2, 2)      \
  X(2, 128, 64, 16, 2, 2)     \
  X(3, 64, 128, 16, 2, 2)     \
  X(4, 64, 64, 32, 2, 2)      \
  X(5, 128, 128, 16, 2, 4)    \
  X(6, 128, 64, 32, 2, 2)     \
  X(7, 64, 128, 32, 2, 2)     \
  X(8, 32, 32, 16, 2, 2)      \
  X(9, 128, 128, 32, 4, 4)    \
  X(10, 128, 128, 16, 4, 4)   \
  X(11, 256, 128, 16, 4, 4)   \
  X(12, 128, 256, 16, 4, 4)   \
  X(13, 128, 128, 32, 2, 4)   \
  X(14, 32, 32, 64, 2, 2)     \
  X(15, 64, 64, 32, 2, 2)     \
  X(16, 32, 32, 128, 2, 2)    \
  X(17, 64, 64, 64, 2, 2)      \
  X(18, 128, 32, 16, 4, 1)     \
  X(19, 32, 128, 16, 1, 4)
struct TileCfg {
  int id, bm, bn, bk, wgm, wgn;
};
#define TC_TILE_ENTRY(id, bm, bn, bk, wgm, wgn) {id, bm, bn, bk, wgm, wgn},
constexpr TileCfg kTiles[] = {TC_GETT_TILES(TC_TILE_ENTRY)};
#undef TC_TILE_ENTRY
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

// The large tiles (256 x 128 and 128 x 256) whose layout-eligible launches
// (see Analysis::dma_ok) run the copy-fed kernel.
constexpr int kDmaTile = 11;
constexpr int kDmaTileWide = 12;
// Output tiles of the copy-fed kernel, all 8 wavefronts over a 144 KB LDS
// ring: 256 x 128, 128 x 256 and 192 x 192.
enum { kDma256x128 = 0, kDma128x256 = 1, kDma192x192 = 2, kDmaShapes = 3 };
constexpr int kDmaShapeBM[kDmaShapes] = {256, 128, 192};
constexpr int kDmaShapeBN[kDmaShapes] = {128, 256, 192};
// Compute units of the target (MI355X): one copy-fed workgroup runs per unit.
constexpr int kDmaComputeUnits = 256;
// Copy-fed shape for an (M, N, L) output: the one among the three whose
// workgroups, dealt out in rounds of one per compute unit, leave the least
// output area in flight (rounds x tile area); ties keep the lower index.
inline int dma_shape(int64_t M, int64_t N, int64_t L) {
  int best = 0;
  double cost = 0.0;
  for (int s = 0; s < kDmaShapes; ++s) {
    const int64_t tiles = ((M + kDmaShapeBM[s] - 1) / kDmaShapeBM[s]) * ((N + kDmaShapeBN[s] - 1) / kDmaShapeBN[s]) * L;
    const double c = (double)((tiles + kDmaComputeUnits - 1) / kDmaComputeUnits) * kDmaShapeBM[s] * kDmaShapeBN[s];
    if (s == 0 || c < cost) {
      best = s;
      cost = c;
    }
  }
  return best;
}
// Contracted group of the copy-fed kernel as modes (first fastest): the
// offset of k is computed from its digits, so no table lookup (a dependent
// load) sits in front of a copy.
constexpr int kDmaMaxKModes = 4;
struct DmaK {
  int n;
  int shape;                  // kDma256x128, kDma128x256 or kDma192x192
  int64_t ext[kDmaMaxKModes];
  int64_t sa[kDmaMaxKModes];  // strides in the kernel's A
  int64_t sb[kDmaMaxKModes];  // strides in the kernel's B
};
// split > 1: the contracted range is cut into `split` segments of seg_len
// (a multiple of the tile depth); parts holds tiles * split * BM * BN doubles.
// dma: the operands qualify for the copy-fed kernel (used for the large
// tiles without split); it runs in dma->shape.
hipError_t launch_gett_f64(const GettParams& p, int tile_id, bool a_kfast, bool b_kfast, int split, int64_t seg_len,
                           double* parts, hipStream_t s, const DmaK* dma = nullptr);
// Split-K choice for `tiles` output tiles of depth-`bk` steps over K.
inline void choose_split(int64_t tiles, int64_t K, int bk, int* split, int64_t* seg_len) {
  *split = 1;
  *seg_len = K;
  if (tiles >= 128 || K < 2048) return;
  int64_t S = (512 + tiles - 1) / tiles;
  const int64_t cap = K / 256;  // at least 256 contracted indices per segment
  if (S > cap) S = cap;
  if (S > 256) S = 256;
  if (S <= 1) return;
  int64_t len = (K + S - 1) / S;
  len = (len + bk - 1) / bk * bk;
  *split = (int)((K + len - 1) / len);
  *seg_len = len;
}

// GEMV / GER family: one thread per output entry walking the contracted
// index (consecutive lanes along n when n_fastest, else along m).
// seg > 1: the contracted range is cut into seg segments whose partial sums
// go to part (outputs * seg doubles) and are added in segment order.
hipError_t launch_lanes_over_outputs(const GettParams& p, bool n_fastest, int64_t seg, double* part, hipStream_t s);
// Contracted segments for lanes-over-outputs: enough workgroups to cover the
// chip when outputs are few, segments of at least 256 indices.
int64_t out_segments(int64_t outputs, int64_t K);
// GEMV-T / DOT family: one wavefront per (output entry, contracted segment);
// seg > 1 needs part[] of M*N*L*seg doubles and adds a second pass.
hipError_t launch_lanes_over_k(const GettParams& p, int64_t seg, double* part, hipStream_t s);
// Number of contracted segments the DOT family uses for this many outputs.
int64_t k_segments(int64_t outputs, int64_t K);

// Split precision: the two inputs are cut into `slices` BF16 or FP8 digit
// planes (dense, k-contiguous, rows padded to Mp / Np, k padded to Kp) plus
// per-row power-of-two scales, then multiplied on the matrix cores.
struct SplitParams {
  const double* A;
  const double* B;
  double* C;
  Offs aM, aK, bN, bK, cM, cN;
  int64_t M, N, K, Mp, Np, Kp;
  bool a_rfast, a_kfast, b_rfast, b_kfast;
  int slices;    // digits per input, or moduli (crt)
  bool fp8;
  bool crt;      // integer residues modulo `slices` coprime moduli
  int bits;      // crt: inputs are rounded to integers of this many bits below the row scale
  int crt_tile;  // crt: residue GEMM configuration (kCrtTiles)
  bool c_nfast;  // crt: C's stride-1 mode is in the N group (rebuild lanes run along n)
  void* planesA;
  void* planesB;
  void* zres;    // crt: residues of the product, slices * Mp * Np bytes
  double* sigA;
  double* sigB;
  double* part;  // max over both inputs of row_max_segments(R, K) * R doubles of scratch
  double alpha, beta;
};
// Contracted segments of the row-maximum pass when rows are stride-1.
inline int64_t row_max_segments(int64_t R, int64_t K) {
  int64_t seg = R > 0 ? (1048576 + R - 1) / R : 1;
  const int64_t cap = K / 64 > 1 ? K / 64 : 1;
  return seg < 1 ? 1 : (seg > cap ? cap : seg);
}
constexpr int kSplitMaxBf16 = 7;
constexpr int kSplitMaxFp8 = 8;
constexpr int kSplitDefaultBf16 = 5;
constexpr int kSplitDefaultFp8 = 8;
struct SplitTile {
  int bm, bn, bk;
};
// Tile of the split GEMM for a digit type and slice count (the LDS holds every
// slice of a k-step twice over, so more slices need smaller tiles).
inline constexpr SplitTile split_tile(bool fp8, int slices) {
  return fp8 ? SplitTile{32, 32, 128} : (slices <= 5 ? SplitTile{128, 64, 32} : SplitTile{64, 64, 32});
}
hipError_t launch_split_contraction(const SplitParams& sp, hipStream_t s);

// Residue arithmetic (crt): pairwise coprime moduli, largest first.  Residues
// lie in [-floor(p/2), ceil(p/2) - 1], so they fit in int8, and a product of
// two is at most 2^14 in magnitude.
constexpr int kCrtMaxModuli = 14;
// Default precision: the fewest moduli that keep at least this many bits per
// input for the contraction's K (at most about 6e-12 componentwise error on
// inputs whose slices span six decades, over 15 times below the 1e-10 the
// form is tested to; 38 bits measured up to 1.7e-11 on short contractions).
constexpr int kCrtDefaultBits = 40;
constexpr int kCrtModuli[kCrtMaxModuli] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199};
// Tile configurations of the residue GEMM: (id, rows, columns, wavefronts
// along rows, wavefronts along columns, pipeline depth).  Depth 1 or 2: k-steps
// of global loads in flight through registers; 3 or more: stages of an LDS
// ring filled by direct global-to-LDS copies.  The contracted depth of a
// k-step is 64 (one INT8 matrix-core step).
#define TC_CRT_TILES(X)        \
  X(0, 128, 128, 2, 2, 1)      \
  X(1, 128, 128, 2, 2, 2)      \
  X(2, 256, 128, 4, 2, 2)      \
  X(3, 128, 256, 2, 4, 2)      \
  X(4, 256, 256, 2, 4, 2)      \
  X(5, 256, 256, 4, 4, 2)       \
  X(6, 256, 256, 4, 4, 1)       \
  X(7, 256, 256, 4, 4, 3)       \
  X(8, 256, 256, 4, 4, 4)       \
  X(9, 256, 128, 4, 2, 4)       \
  X(10, 256, 256, 2, 4, 4)      \
  X(11, 256, 256, 4, 2, 4)
struct CrtTileCfg {
  int bm, bn, wgm, wgn, pf;
};
#define TC_CRT_ROW(id, bm, bn, wgm, wgn, pf) {bm, bn, wgm, wgn, pf},
constexpr CrtTileCfg kCrtTiles[] = {TC_CRT_TILES(TC_CRT_ROW)};
#undef TC_CRT_ROW
constexpr int kCrtNumTiles = sizeof(kCrtTiles) / sizeof(kCrtTiles[0]);
static_assert(kCrtNumTiles == TC_CRT_NUM_TILES, "tile table and header agree");
constexpr int kCrtDefaultTile = 11;
constexpr int kCrtBK = 64;
// Largest b <= 48 such that n moduli represent every sum of K products of
// integers |a|, |b| <= 2^b without ambiguity: 2 K 4^b < P, P the product of
// the moduli.  0 when no b >= 1 fits.  (Up to 2^48 the FP64 quotient y / p of
// the residue pass rounds to the nearest integer exactly.)
constexpr int kCrtMaxBits = 48;
inline int crt_bits(int n, int64_t K) {
  unsigned __int128 P = 1;
  for (int i = 0; i < n; ++i) P *= (unsigned)kCrtModuli[i];
  const unsigned __int128 k = (unsigned __int128)(K > 0 ? K : 1);
  for (int b = kCrtMaxBits; b >= 1; --b)
    if (k <= ((P - 1) >> (2 * b + 1))) return b;
  return 0;
}
// The default number of moduli for contracted extent K.
inline int crt_default_moduli(int64_t K) {
  for (int n = 2; n < kCrtMaxModuli; ++n)
    if (crt_bits(n, K) >= kCrtDefaultBits) return n;
  return kCrtMaxModuli;
}

// Batch-dominated contractions: per-point slabs staged through LDS.
struct SlabDesc {
  int n;                 // modes of the operand inside one slab
  int size;              // entries per slab
  int batch_fast;        // the batch index varies fastest in memory
  int dense;             // the slab's modes are dense in their storage order: entry r at r * s0
  int contig;            // dense, s0 = 1 and consecutive batch indices' slabs follow each other
  int64_t s0;            // global stride of the slab's storage order (dense only)
  FastDiv size_div;      // division by size
  FastDiv div[kMaxRank];   // extents, sorted by global stride
  int64_t gstr[kMaxRank];  // global strides
  int lstr[kMaxRank];    // strides in the canonical LDS slab (operands that are not dense)
};
struct BatchedParams {
  const double* A;
  const double* B;
  double* C;
  Offs aL, bL, cL;
  SlabDesc a, b, c;
  // LDS offsets of the group indices inside one point's slab: the storage
  // order for dense operands, the canonical [m][k] / [n][k] / [m][n] otherwise
  Offs am, ak, bn, bk, cm, cn;
  int M, N, K;           // per-point group sizes
  int P;                 // batch indices per workgroup
  FastDiv P_div, N_div, sC_div;
  int64_t L;
  double alpha, beta;
};
constexpr int kBatchedLdsDoubles = 2048;  // 16 KB of LDS per workgroup: several workgroups per CU
// LDS budget of the standalone slab kernel's batch points per workgroup
#ifndef TC_SLAB_LDS_DOUBLES
#define TC_SLAB_LDS_DOUBLES 2048
#endif
constexpr int kBatchedSlabLdsDoubles = TC_SLAB_LDS_DOUBLES;
// Points per workgroup for per-point slabs of `per` doubles and K contracted
// indices (the contracted offsets of A and B are staged in LDS as well).
inline int slab_points(int per, int K, int lds_doubles) {
  const int P = (lds_doubles - K) / per;
  return P > 64 ? 64 : P;
}
hipError_t launch_batched_small(const BatchedParams& bp, hipStream_t s);

// Persistent batches.  Tile configurations of the batch kernel (id, rows,
// columns, contracted depth; 2 x 2 wavefronts each).
#define TC_BATCH_TILES(X) \
  X(0, 64, 64, 16)        \
  X(1, 32, 32, 16)        \
  X(2, 32, 32, 64)        \
  X(3, 64, 64, 32)        \
  X(4, 32, 32, 128)       \
  X(5, 64, 64, 64)
constexpr int kNumBatchTiles = 6;
constexpr int kBatchTileBM[kNumBatchTiles] = {64, 32, 32, 64, 32, 64};
constexpr int kBatchTileBN[kNumBatchTiles] = {64, 32, 32, 64, 32, 64};
constexpr int kBatchSlabLdsDoubles = 2048;     // slab LDS of batch tasks: at least 16 KB ...
constexpr int kBatchSlabLdsMaxDoubles = 8192;  // ... and at most 64 KB, whatever the kernel's occupancy leaves
// Task kinds of the batch kernel.
enum BatchKind {
  kBatchGemm = 0,        // one GEMM tile (or one contracted segment of it)
  kBatchSlab = 1,        // the slabs of P batch indices
  kBatchLanesK = 2,      // 4 (output, segment) units, one wavefront each, lanes along the contracted index
  kBatchLanesOut = 3     // 256 outputs along lanes, each walking one contracted segment
};
constexpr int kLanesKOutputs = 4;      // (output, segment) units per lanes-over-k task (one per wavefront)
constexpr int kLanesOutOutputs = 256;  // outputs per lanes-over-outputs task (one per thread)
struct BatchItem {       // one contraction of a batch (layout only)
  GettParams g;          // kinds 0, 2, 3
  BatchedParams b;       // kind 1: slabs of batch indices
  int kind;
  int akf, bkf, swapped;
  int64_t tilesM, tilesN;
  int ksplit;            // contracted segments per task group (1 = none)
  int n_fastest;         // kind 3: consecutive lanes along n (else along m)
  int64_t seg_len;       // contracted indices per segment (kind 2 with kblk: blocks)
  int64_t part_off;      // first partial sum of this item (in doubles)
  int64_t cnt_off;       // first completion counter of this item
  // Kind 2 over a contracted group of several modes: its entries in blocks
  // of at most 64, lane l taking entry (l % kbp) of mode p and (l / kbp) of
  // mode q of a block.  g.aK / g.bK hold each block's base offset in A and
  // B, klim its extents along p and q (bits 0-7 and 8-15).
  int kblk;              // 1: blocked addressing
  int kbp;               // block extent along mode p
  int64_t nblk;          // blocks
  int64_t ksa_p, ksa_q, ksb_p, ksb_q;  // strides of modes p and q in A and B
  Offs klim;
};
struct BatchPtrs {       // per execution
  const double* A;
  const double* B;
  double* C;
  double alpha, beta;
};
struct BatchTask {
  int item;
  int seg;               // contracted segment (ksplit > 1)
  int64_t idx;           // tile (kind 0), slab (1) or output group (2, 3) index
};
// Engines of a batch: each runs as its own persistent launch over its own
// task list (GEMM tiles; inner products and matrix-vector groups; slabs).
enum { kBatchEngineGemm = 0, kBatchEngineLanes = 1, kBatchEngineSlab = 2, kBatchEngines = 3 };
inline int batch_engine_of(int kind) {
  return kind == kBatchGemm ? kBatchEngineGemm : (kind == kBatchSlab ? kBatchEngineSlab : kBatchEngineLanes);
}
struct BatchLaunch {
  const BatchItem* items;
  const BatchPtrs* ptrs;
  const BatchTask* tasks;
  int64_t ntasks;
  const int64_t* chunks[kBatchEngines];  // engine e's chunk c holds tasks [chunks[e][c], chunks[e][c+1])
  int64_t nchunks[kBatchEngines];
  unsigned long long* counter;           // kBatchEngines chunk counters
  double* parts;                         // partial sums of split items
  unsigned* tile_cnt;                    // segments finished per split tile or output group
  int64_t n_cnt;
  int config;
  int slab_lds_doubles;
  int num_cus;
  // slab items large enough to fill the chip on their own: one launch each,
  // a workgroup per P batch indices (host arrays: item index, workgroups)
  const int* direct_items;
  const int64_t* direct_blocks;
  int ndirect;
  const BatchItem* host_items;  // host copy of the items (layouts of the direct launches)
};
// Slab items with at least this many workgroups per CU run as launches of
// their own instead of tasks of the persistent slab engine.
constexpr int kBatchDirectSlabBlocksPerCu = 16;
// Workgroups of the slab engine one CU holds at once with this much LDS per
// workgroup (doubles), or 0 on error.
int batch_slab_blocks_per_cu(int slab_lds_doubles);
hipError_t launch_batch(const BatchLaunch& bl, hipStream_t s);

// The picker's MLP (n_in -> hidden -> hidden -> n_out, ReLU, FP32).
struct MlpDims {
  int n_in, hidden, n_out;
  int64_t num_params() const {
    return (int64_t)n_in * hidden + hidden + (int64_t)hidden * hidden + hidden + (int64_t)hidden * n_out + n_out;
  }
};
struct MlpScratch {  // activations and their gradients for one batch
  float *H1, *H2, *Y, *dY, *dH2, *dH1;
};
hipError_t mlp_forward(const MlpDims& d, const float* params, const float* X, float* H1, float* H2, float* Y, int B,
                       hipStream_t s);
// After mlp_forward into w.H1/w.H2/w.Y: gradients of the masked mean-squared
// error into grads (same layout as params); sums[0] receives the loss.
hipError_t mlp_backward(const MlpDims& d, const float* params, const float* X, const float* T, const float* M,
                        const MlpScratch& w, float* grads, float* sums, int B, hipStream_t s);
hipError_t mlp_adam(float* params, const float* grads, float* m, float* v, int64_t n, float lr, int step,
                    hipStream_t s);

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
