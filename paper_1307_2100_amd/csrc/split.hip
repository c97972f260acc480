// Split-precision contraction: FP64 accuracy from BF16 (or FP8) matrix cores.
//
// Scheme (error-free splitting in the manner of Ozaki, Ogita, Oishi and Rump,
// 2012; written from the mathematics, not from any code):
//   * each row r of the gathered A (and each column of B) gets a power-of-two
//     scale sigma_r >= max_k |X[r,k]|, so every x / sigma_r lies in (-1, 1);
//   * that ratio is cut into S integer digits: q_0 = rint(2^b x/sigma), then
//     each remainder (at most 1/2 in magnitude) is multiplied by 2^(b+1) and
//     rounded again, so |q_s| <= 2^b and x = sigma * sum_s q_s 2^(-b-(b+1)s)
//     up to the last remainder.  b = 8 for BF16 (integers up to 256 are exact
//     there) and b = 4 for FP8 E4M3 (integers up to 16);
//   * C = sum over digit pairs (s, t) with s + t < S of the digit products.
//     Products of one "level" g = s + t carry the same power of two.  Every
//     digit product is an integer below 2^(2b), so sums of a few hundred of
//     them are exact in FP32: the sums of levels 0, 1 and 2 are kept in their
//     own FP32 accumulators and moved to FP64 before they could round (level
//     g after 256 / (g + 1) contracted indices), which keeps them exact; the
//     deeper levels (2^-27 and below) share one FP32 accumulator, moved every
//     64 indices, whose rounding is far below the target accuracy.
//   * BF16 planes are stored pre-scaled by 2^(-9(s-1)), so that every product
//     of planes s and t carries the same factor 2^(-34) sigma_m tau_n; the FP8
//     planes keep the raw digits and pass the per-plane powers of two as the
//     matrix-core block scales.
// The digits are written densely, k-contiguous and digit-interleaved per
// k-step ([row][k-step][s][k]); gathering the tensor through its strides
// happens once, in the split pass.
#include <cmath>

#include "kernels.hpp"

namespace tc {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef unsigned short u16;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline int fq_of(int lane) { return lane >> 4; }

// ---------------------------------------------------------------- scales
// sigma[r] = 2^e with max_k |X[r,k]| < 2^e (0 for an all-zero row or padding).
__device__ inline double pow2_above(double mx) {
  if (mx == 0.0) return 0.0;
  int e;
  (void)frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1)
  return ldexp(1.0, e);
}

// Rows stride-1 in memory: one thread per row walks one segment of k and
// writes a partial maximum; a second pass takes the maximum over segments.
__global__ __launch_bounds__(256) void row_max_rows_kernel(const double* __restrict__ X, Offs xr, Offs xk,
                                                           int64_t R, int64_t K, int64_t seg_len,
                                                           double* __restrict__ part) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t sgi = blockIdx.y;
  if (r >= R) return;
  const double* row = X + off_at(xr, r);
  const int64_t k0 = sgi * seg_len, k1 = k0 + seg_len < K ? k0 + seg_len : K;
  // four independent maxima so that four loads are in flight per thread
  double m4[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t k = k0;
  for (; k + 4 <= k1; k += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) m4[u] = fmax(m4[u], fabs(row[off_at(xk, k + u)]));
  }
  for (; k < k1; ++k) m4[0] = fmax(m4[0], fabs(row[off_at(xk, k)]));
  part[sgi * R + r] = fmax(fmax(m4[0], m4[1]), fmax(m4[2], m4[3]));
}

__global__ __launch_bounds__(256) void row_scale_from_parts_kernel(const double* __restrict__ part, int64_t R,
                                                                   int64_t nseg, int64_t Rp,
                                                                   double* __restrict__ sigma) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= Rp) return;
  double mx = 0.0;
  if (r < R)
    for (int64_t g = 0; g < nseg; ++g) mx = fmax(mx, part[g * R + r]);
  sigma[r] = pow2_above(mx);
}

// One wavefront per row, lanes along k (k stride-1 in memory).
__global__ __launch_bounds__(256) void row_scale_wave_kernel(const double* __restrict__ X, Offs xr, Offs xk,
                                                             int64_t R, int64_t K, int64_t Rp,
                                                             double* __restrict__ sigma) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= Rp) return;
  double mx = 0.0;
  if (r < R) {
    const double* row = X + off_at(xr, r);
    for (int64_t k = lane; k < K; k += 64) mx = fmax(mx, fabs(row[off_at(xk, k)]));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) sigma[r] = pow2_above(mx);
}

// ---------------------------------------------------------------- digits
__device__ inline u16 bf16_bits_of_small_int(double v, int scale_exp) {
  // v is an integer with |v| <= 256; v * 2^scale_exp is exact in BF16
  float f = ldexpf((float)v, scale_exp);
  unsigned u = __float_as_uint(f);
  return (u16)(u >> 16);  // exact: the low 16 bits are zero
}

// E4M3 (OCP) bits of an integer v with |v| <= 16.
__device__ inline unsigned char e4m3_of_small_int(int v) {
  if (v == 0) return 0;
  unsigned char s = v < 0 ? 0x80 : 0;
  int a = v < 0 ? -v : v;
  int e = 31 - __clz(a);                  // a in [2^e, 2^(e+1))
  int m = ((a - (1 << e)) << 3) >> e;     // 3 mantissa bits, exact for a <= 16
  return s | (unsigned char)(((e + 7) << 3) | m);
}

// Digits of a 64 x 64 tile of X staged in LDS; rows beyond R and columns
// beyond K are written as zero digits.
// Stage the 64 x 64 tile of X at (r0, k0) in LDS, lanes along whichever of
// r and k is stride-1 in memory (zeros beyond R and K).  256 threads.  The
// offsets of a thread's 16 entries are formed first (one branch on table or
// stride for the whole tile) and the 16 loads are unconditional (out-of-range
// entries read X[0] and are replaced by zero), so all of them are in flight
// together instead of one per basic block.
TC_DEV void gather_tile64(const double* __restrict__ X, const Offs& xr, const Offs& xk, int64_t R, int64_t K,
                          int64_t r0, int64_t k0, int rfast, double (*tile)[65]) {
  const int tid = threadIdx.x;
  const int lane64 = tid & 63, q = tid >> 6;
  double v[16];
  if (R <= 0 || K <= 0) {
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = 0.0;
  } else {
    // the fixed index (one per thread) and the 16 varying ones
    const Offs& fixo = rfast ? xr : xk;
    const Offs& varo = rfast ? xk : xr;
    const int64_t fix = (rfast ? r0 : k0) + lane64, fixn = rfast ? R : K;
    const int64_t var0 = rfast ? k0 : r0, varn = rfast ? K : R;
    const int64_t fo = fix < fixn ? off_at(fixo, fix) : 0;
    int64_t vo[16];
    if (varo.tab) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t j = var0 + q + 4 * i;
        vo[i] = varo.tab[j < varn ? j : 0];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) vo[i] = (var0 + q + 4 * i) * varo.stride;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const bool ok = fix < fixn && var0 + q + 4 * i < varn;
      const double x = X[ok ? fo + vo[i] : 0];
      v[i] = ok ? x : 0.0;
    }
  }
  if (rfast) {
#pragma unroll
    for (int i = 0; i < 16; ++i) tile[lane64][q + 4 * i] = v[i];
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) tile[q + 4 * i][lane64] = v[i];
  }
}

template <int S, bool FP8>
__global__ __launch_bounds__(256) void split_planes_kernel(const double* __restrict__ X, Offs xr, Offs xk,
                                                           int64_t R, int64_t K, int64_t Rp, int64_t Kp,
                                                           const double* __restrict__ sigma, int rfast,
                                                           void* __restrict__ planes) {
  __shared__ double tile[64][65];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * 64, k0 = (int64_t)blockIdx.x * 64;
  gather_tile64(X, xr, xk, R, K, r0, k0, rfast, tile);
  __syncthreads();
  constexpr double first = FP8 ? 16.0 : 256.0;   // 2^b
  constexpr double next = FP8 ? 32.0 : 512.0;    // 2^(b+1)
  // digit-interleaved layout [r][k / KB][s][k % KB]: one k-step of a row
  // holds all S digits contiguously (whole cache lines per load).  A thread
  // takes V consecutive k of one row and writes each digit plane's V entries
  // as one 16-byte store.
  constexpr int KB = FP8 ? 128 : 32;
  constexpr int V = FP8 ? 16 : 8;             // entries per 16 bytes
  constexpr int GROUPS = 64 / V;              // k groups per tile row
  for (int item = tid; item < 64 * GROUPS; item += 256) {
    const int rr = item / GROUPS, kk0 = (item % GROUPS) * V;
    const int64_t r = r0 + rr, k = k0 + kk0;
    if (r >= Rp || k >= Kp) continue;  // Kp is a multiple of KB, so all V entries are in range
    const double sg = sigma[r];
    double rem[V];
    // exact: sg is a power of two, and so is its reciprocal unless sg is subnormal
    if (sg >= 0x1p-1022) {
      const double inv = 1.0 / sg;
#pragma unroll
      for (int v = 0; v < V; ++v) rem[v] = tile[rr][kk0 + v] * inv;
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) rem[v] = sg > 0.0 ? tile[rr][kk0 + v] / sg : 0.0;
    }
    const int64_t base = r * Kp * S + (k / KB) * (S * KB) + (k % KB);
#pragma unroll
    for (int s_ = 0; s_ < S; ++s_) {
      u32x4 word = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double y = rem[v] * (s_ == 0 ? first : next);
        const double q = rint(y);
        rem[v] = y - q;  // exact
        unsigned bits;
        int shift;
        if constexpr (FP8) {
          bits = e4m3_of_small_int((int)q);
          shift = 8 * (v & 3);
        } else {
          bits = bf16_bits_of_small_int(q, -9 * (s_ - 1));
          shift = 16 * (v & 1);
        }
        word[v / (V / 4)] |= bits << shift;
      }
      if constexpr (FP8) {
        *reinterpret_cast<u32x4*>((unsigned char*)planes + base + s_ * KB) = word;
      } else {
        *reinterpret_cast<u32x4*>((u16*)planes + base + s_ * KB) = word;
      }
    }
  }
}

// ---------------------------------------------------------------- GEMM
struct SplitGemmArgs {
  const void* pa;        // digits of the kernel's A: [Mp][Kp/KB][S][KB]
  const void* pb;        // digits of the kernel's B: [Np][Kp/KB][S][KB]
  const double* sa;      // sigma of A rows (Mp)
  const double* sb;      // sigma of B rows (Np)
  double* C;
  Offs cM, cN;
  int64_t M, N, Mp, Np, Kp;
  double alpha, beta;
  double unit;           // power of two turning the accumulated digit sums into values
};

// Register stage of one k-step: each thread moves CPT 16-byte chunks from
// global memory (row pointers fixed per tile, advanced by the k offset) to
// precomputed LDS offsets.  Kept in a struct with constant-indexed arrays so
// that the chunks stay in registers while the MFMAs of the current k-step run.
template <typename T, int CPT, int CHUNKS, int NT>
struct Stager {
  u32x4 v[CPT];
  int dst[CPT];
  __device__ inline void load(const T* const (&row)[CPT], int64_t koff, int tid) {
#pragma unroll
    for (int i = 0; i < CPT; ++i)
      if (CHUNKS % NT == 0 || tid + i * NT < CHUNKS) v[i] = *(const u32x4*)(row[i] + koff);
  }
  __device__ inline void store(T* st, int tid) const {
#pragma unroll
    for (int i = 0; i < CPT; ++i)
      if (CHUNKS % NT == 0 || tid + i * NT < CHUNKS) *(u32x4*)(st + dst[i]) = v[i];
  }
};

// BF16 digits: v_mfma_f32_16x16x32_bf16.  Operand lane layout (measured):
// lane l holds A[l%16][8(l/16) .. 8(l/16)+7] and B[8(l/16) ..][l%16]; the
// accumulator element r holds D[4(l/16) + r][l%16].
template <int BM, int BN, int WGM, int WGN, int S>
__global__ __launch_bounds__(64 * WGM * WGN) void split_gemm_bf16_kernel(SplitGemmArgs p) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int BK = 32;                  // one MFMA depth per k-step
  constexpr int ROW = S * BK;             // bf16 per staged row: all S digits of one k-step
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int CPR = S * 4;                            // 16-byte chunks per staged row
  constexpr int CHUNKS = (BM + BN) * CPR;
  constexpr int CPT = (CHUNKS + NT - 1) / NT;           // chunks per thread
  __shared__ __attribute__((aligned(16))) u16 sm[2][(BM + BN) * ROW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  int64_t tm, tn;
  xcd_tile(blockIdx.x, (p.Mp / BM) * (p.Np / BN), p.Mp / BM, p.Np / BN, &tm, &tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;

  const u16* __restrict__ PA = (const u16*)p.pa;
  const u16* __restrict__ PB = (const u16*)p.pb;
  const int64_t rowlen = p.Kp * S;  // digits per row of the dense digit matrix

  // Staged row r keeps its 16-byte chunk q of digit s at slot q ^ ((r >> 2) & 3):
  // the 16 rows one fragment read touches then fall in 16 distinct bank groups.
  auto lds_off = [](int r, int s_, int q) { return r * ROW + s_ * BK + ((q ^ ((r >> 2) & 3)) << 3); };
  Stager<u16, CPT, CHUNKS, NT> stg;
  const u16* srow[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int c = tid + i * NT;
    const int row = (c < CHUNKS ? c : 0) / CPR, sub = (c < CHUNKS ? c : 0) % CPR;
    srow[i] = (row < BM ? PA + (m0 + row) * rowlen : PB + (n0 + row - BM) * rowlen) + sub * 8;
    stg.dst[i] = lds_off(row, sub >> 2, sub & 3);
  }

  // Level g (digit pair s + t = g) sums: levels 0, 1, 2 exact in their own
  // accumulators over 64 contracted indices (at most 3 * 64 * 2^16 < 2^24 digit
  // units), deeper levels together.
  constexpr int NACC = S < 4 ? S : 4;
  f4 acc[NACC][TM][TN];
  double acc64[TM][TN][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
#pragma unroll
      for (int g = 0; g < NACC; ++g) acc[g][i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
    }

  const int64_t ksteps = p.Kp / BK;
  stg.load(srow, 0, tid);
  stg.store(sm[0], tid);
  __syncthreads();
  const int fr = lane & 15, fq = lane >> 4;
  for (int64_t ks = 0; ks < ksteps; ++ks) {
    const int cur = ks & 1;
    if (ks + 1 < ksteps) stg.load(srow, (ks + 1) * ROW, tid);
    const u16* st = sm[cur];
    bf8 af[S][TM];
#pragma unroll
    for (int s_ = 0; s_ < S; ++s_)
#pragma unroll
      for (int i = 0; i < TM; ++i) af[s_][i] = *(const bf8*)(st + lds_off(wm * WM + i * 16 + fr, s_, fq));
#pragma unroll
    for (int t = 0; t < S; ++t) {
      bf8 bfr[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) bfr[j] = *(const bf8*)(st + lds_off(BM + wn * WN + j * 16 + fr, t, fq));
#pragma unroll
      for (int s_ = 0; s_ + t < S; ++s_) {
        const int g = s_ + t < NACC ? s_ + t : NACC - 1;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[g][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[s_][i], bfr[j], acc[g][i][j], 0, 0, 0);
      }
    }
    // Move FP32 level sums to FP64 before they could round: level g adds
    // g + 1 digit products below 2^16 per contracted index, so it stays exact
    // for 256 / (g + 1) indices: level 0 every 256 (8 k-steps), level 1 every
    // 128, level 2 every 64; the shared deeper levels every 64 as well.
    const bool last_step = ks + 1 == ksteps;
#pragma unroll
    for (int g = 0; g < NACC; ++g) {
      const int every = g == 0 ? 8 : (g == 1 ? 4 : 2);
      if (((ks + 1) % every) != 0 && !last_step) continue;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[g][i][j][r];
          acc[g][i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    if (ks + 1 < ksteps) stg.store(sm[cur ^ 1], tid);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + wm * WM + i * 16 + fq * 4 + r;
      if (m >= p.M) continue;
      const double sm_ = p.sa[m] * p.unit * p.alpha;
      const int64_t cm = off_at(p.cM, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + wn * WN + j * 16 + fr;
        if (n >= p.N) continue;
        double* dst = p.C + cm + off_at(p.cN, n);
        double v = sm_ * p.sb[n] * acc64[i][j][r];
        if (p.beta != 0.0) v += p.beta * *dst;
        *dst = v;
      }
    }
  }
}

// BF16 digits, fed by direct global-to-LDS copies through two stages.  A
// stage holds one k-step (32 contracted indices) of all S digits of the
// tile's BM + BN rows, row after row (S x 64 bytes each, the digits' 16-byte
// chunks swizzled within each digit), filled by global_load_lds_dwordx4
// copies of 1 KB each.
// Schedule of a k-step ks: the MFMAs go in phases t = 0 .. S-1 (digit t of B
// against digits s < S - t of A).  The reads of B's remaining digits are
// spread over phases 0 and 1; then each wavefront waits for its own copies
// (vmcnt(0): those of k-step ks + 1, the only vector memory operations in
// flight) and reads (lgkmcnt(0)), and the workgroup meets at a barrier.
// After it, k-step ks + 1 is visible in the other stage and nothing reads
// this one any more, so the copies of k-step ks + 2 into this stage and the
// reads of k-step ks + 1's first fragments (A's digits, B's digit 0, into a
// second register set) are spread over the remaining phases: a copy has one
// whole k-step to land.  The last k-step is peeled off.
template <int BM, int BN, int WGM, int WGN, int S>
__global__ __launch_bounds__(64 * WGM * WGN) void split_gemm_bf16_dma_kernel(SplitGemmArgs p) {
  constexpr int NW = WGM * WGN;
  constexpr int KB = 32;                   // contracted indices per k-step (one MFMA depth)
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int AG = BM / 16, BG = BN / 16;
  constexpr int NCOPY = (AG + BG) * S;     // 1 KB blocks per stage
  constexpr int CPW = (NCOPY + NW - 1) / NW;
  constexpr int STAGE = NCOPY * 1024;
  constexpr int BP = S >= 3 ? 1 : 0;       // the barrier follows this phase
  extern __shared__ __attribute__((aligned(16))) signed char dsm[];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  int64_t tm, tn;
  xcd_tile(blockIdx.x, (p.Mp / BM) * (p.Np / BN), p.Mp / BM, p.Np / BN, &tm, &tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const u16* const PA = (const u16*)p.pa;
  const u16* const PB = (const u16*)p.pb;
  const int64_t rowlen = p.Kp * S;         // bf16 per row of the dense digit matrix
  // Copy j of this wavefront fills 1 KB block c = wave + NW j of the stage
  // (when c < NCOPY): its lane l lands 16 bytes at slot P = 64 c + l, and
  // fetches the chunk stored there -- staged row r = P / (4 S), digit d, and
  // contracted-index chunk q ^ ((r >> 2) & 3) for slot q of the digit's four.
  // A copy thus reads whole runs of each row's S x 64 contiguous bytes.  The
  // first AG S blocks are A's rows, a whole number per wavefront, so copy j
  // reads A for j < AG S / NW and B after.  Its address is a uniform base (the
  // tile's first row of that operand, advanced per k-step) plus a 32-bit
  // per-lane byte offset (the launch keeps BM rows of digits below 2^31
  // bytes), and its LDS address is uniform: no vector arithmetic per copy.
  static_assert((AG * S) % NW == 0, "A's blocks must split evenly over the wavefronts");
  constexpr int CPA = AG * S / NW;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  uint32_t voff[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = wave + NW * j < NCOPY ? wave + NW * j : 0;
    const int P = 64 * c + lane, r = P / (4 * S), w = P % (4 * S);
    const int dig = w >> 2, q = (w & 3) ^ ((r >> 2) & 3);
    const int rr = j < CPA ? r : r - BM;
    voff[j] = (uint32_t)(((int64_t)rr * rowlen + dig * KB + q * 8) * 2);
  }
  const char* const tileA = (const char*)(PA + m0 * rowlen);
  const char* const tileB = (const char*)(PB + n0 * rowlen);
  auto copy1 = [&](int j, int64_t ks, int stage) {
    const int c = wave_u + NW * j;
    if (c < NCOPY) {
      const char* g = (j < CPA ? tileA : tileB) + ks * (S * KB * 2);
      __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)(g + voff[j]),
                                       (void __attribute__((address_space(3)))*)(dsm + stage * STAGE + c * 1024), 16,
                                       0, 0);
    }
  };
  // A fragment: rows 16 g .. 16 g + 15, lane l reading row l%16's chunk l/16
  // of one digit; for odd S the swizzle puts the 16 rows' chunks in 16
  // distinct 16-byte bank groups of the LDS's 64 banks (S = 2 and 4 leave 2-
  // and 4-way conflicts).
  const int lanepart = (lane & 15) * (S * 64) + (((lane >> 4) ^ ((lane >> 2) & 3)) << 4);
  auto afrag = [&](int stage, int dig, int i) {
    return *(const bf8*)(dsm + stage * STAGE + (wm * TM + i) * (16 * S * 64) + dig * 64 + lanepart);
  };
  auto bfrag = [&](int stage, int dig, int j) {
    return *(const bf8*)(dsm + stage * STAGE + (AG + wn * TN + j) * (16 * S * 64) + dig * 64 + lanepart);
  };

  // Level g (digit pair s + t = g) sums: levels 0, 1, 2 exact in their own
  // FP32 accumulators for the intervals below, deeper levels together.
  constexpr int NACC = S < 4 ? S : 4;
  f4 acc[NACC][TM][TN];
  double acc64[TM][TN][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
#pragma unroll
      for (int g = 0; g < NACC; ++g) acc[g][i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
    }
  // FP32 level sums to FP64 before they could round: level g adds g + 1
  // digit products below 2^16 per contracted index, so it stays exact for
  // 256 / (g + 1) indices: level 0 every 8 k-steps, level 1 every 4, level 2
  // and the shared deeper levels every 2.
  auto flush = [&](int64_t ks, bool last_step) {
#pragma unroll
    for (int g = 0; g < NACC; ++g) {
      const int every = g == 0 ? 8 : (g == 1 ? 4 : 2);
      if (((ks + 1) % every) != 0 && !last_step) continue;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[g][i][j][r];
          acc[g][i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
  };
  // MFMAs of phase t (A digits s < S - t against B digit t)
  auto phase_mfma = [&](int t, const bf8 (&af)[S][TM], const bf8 (&bt)[TN], int q0, int q1) {
    // products numbered q = (s, i, j) in this phase; only those in [q0, q1)
    int q = 0;
#pragma unroll
    for (int s_ = 0; s_ + t < S; ++s_) {
      const int g = s_ + t < NACC ? s_ + t : NACC - 1;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j, ++q)
          if (q >= q0 && q < q1)
            acc[g][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[s_][i], bt[j], acc[g][i][j], 0, 0, 0);
    }
  };
  // number of MFMAs of phase t
  auto nmfma = [](int t) { return (S - t) * TM * TN; };

  bf8 a0[S][TM], a1[S][TM];
  bf8 b[S][TN];
  const int64_t ksteps = p.Kp / KB, last = ksteps - 1;
#pragma unroll
  for (int j = 0; j < CPW; ++j) copy1(j, 0, 0);
#pragma unroll
  for (int j = 0; j < CPW; ++j) copy1(j, last > 0 ? 1 : 0, 1);
  __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int i = 0; i < TM; ++i) a0[d][i] = afrag(0, d, i);
#pragma unroll
  for (int j = 0; j < TN; ++j) b[0][j] = bfrag(0, 0, j);

  // one k-step with a next one: reads of stage cur, then copies into stage
  // cur (of k-step ks + 2, or of the last one again: a stage nobody reads
  // after the barrier) and reads of stage cur ^ 1; (af) holds this k-step's A
  // digits, (an) receives the next
  auto kstep = [&](int64_t ks, const bf8 (&af)[S][TM], bf8 (&an)[S][TM]) {
    const int cur = (int)(ks & 1), nxt = cur ^ 1;
    const int64_t kc = ks + 2 <= last ? ks + 2 : last;
    // phases 0 .. BP: reads of B digits 1 .. S-1
    constexpr int NB = (S - 1) * TN;          // B fragments still to read
#pragma unroll
    for (int t = 0; t <= BP; ++t) {
      const int n = nmfma(t);
#pragma unroll
      for (int q = 0; q < n; ++q) {
        __builtin_amdgcn_sched_barrier(0);
        phase_mfma(t, af, b[t], q, q + 1);
        __builtin_amdgcn_sched_barrier(0);
        // B reads: those numbered [before NB / span, (before + 1) NB / span)
        // after the MFMA numbered (before) of phases 0 .. BP
        const int before = (t == 0 ? 0 : nmfma(0)) + q;
        const int span = BP == 0 ? nmfma(0) : nmfma(0) + nmfma(1);
#pragma unroll
        for (int x = before * NB / span; x < (before + 1) * NB / span; ++x)
          b[1 + x / TN][x % TN] = bfrag(cur, 1 + x / TN, x % TN);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    // this wavefront's copies of the next k-step, and its reads of this one
    // (so no read of a stage is in flight when the copies into it start)
    __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (0 << 8));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    // phases BP+1 .. S-1: copies into this stage and reads of the next
    // k-step's fragments spread over them
    constexpr int NR = S * TM + TN;
    int span = 0;
#pragma unroll
    for (int t = BP + 1; t < S; ++t) span += nmfma(t);
    int before = 0;
#pragma unroll
    for (int t = BP + 1; t < S; ++t) {
      const int n = nmfma(t);
#pragma unroll
      for (int q = 0; q < n; ++q, ++before) {
        __builtin_amdgcn_sched_barrier(0);
        phase_mfma(t, af, b[t], q, q + 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = before * CPW / span; j < (before + 1) * CPW / span; ++j) copy1(j, kc, cur);
#pragma unroll
        for (int x = before * NR / span; x < (before + 1) * NR / span; ++x) {
          if (x < S * TM)
            an[x / TM][x % TM] = afrag(nxt, x / TM, x % TM);
          else
            b[0][x - S * TM] = bfrag(nxt, 0, x - S * TM);
        }
      }
    }
    if (span == 0) {  // no phase after the barrier (S = 1): copy and read here
#pragma unroll
      for (int j = 0; j < CPW; ++j) copy1(j, kc, cur);
#pragma unroll
      for (int d = 0; d < S; ++d)
#pragma unroll
        for (int i = 0; i < TM; ++i) an[d][i] = afrag(nxt, d, i);
#pragma unroll
      for (int j = 0; j < TN; ++j) b[0][j] = bfrag(nxt, 0, j);
    }
    __builtin_amdgcn_sched_barrier(0);
    flush(ks, false);
  };
  int64_t ks = 0;
  for (; ks + 1 < last; ks += 2) {
    kstep(ks, a0, a1);
    kstep(ks + 1, a1, a0);
  }
  if (ks < last) {
    kstep(ks, a0, a1);
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
      for (int i = 0; i < TM; ++i) a0[d][i] = a1[d][i];
    ++ks;
  }
  // the last k-step: read B's remaining digits, then every phase
  {
    const int cur = (int)(ks & 1);
#pragma unroll
    for (int t = 1; t < S; ++t)
#pragma unroll
      for (int j = 0; j < TN; ++j) b[t][j] = bfrag(cur, t, j);
#pragma unroll
    for (int t = 0; t < S; ++t) phase_mfma(t, a0, b[t], 0, nmfma(t));
    flush(ks, true);
  }
  // the copies issued during the k-step before (of the last k-step again)
  // land before the workgroup's LDS can be handed to another
  __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));

#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + wm * WM + i * 16 + (lane >> 4) * 4 + r;
      if (m >= p.M) continue;
      const double sm_ = p.sa[m] * p.unit * p.alpha;
      const int64_t cm = off_at(p.cM, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + wn * WN + j * 16 + (lane & 15);
        if (n >= p.N) continue;
        double* dst = p.C + cm + off_at(p.cN, n);
        double v = sm_ * p.sb[n] * acc64[i][j][r];
        if (p.beta != 0.0) v += p.beta * *dst;
        *dst = v;
      }
    }
  }
}

// FP8 E4M3 digits: v_mfma_scale_f32_16x16x128_f8f6f4 with the per-plane powers
// of two as E8M0 block scales.  Lane l holds A[l%16][32(l/16) .. +31]; the
// accumulator element r holds D[4(l/16) + r][l%16].
template <int BM, int BN, int WGM, int WGN, int S>
__global__ __launch_bounds__(64 * WGM * WGN) void split_gemm_fp8_kernel(SplitGemmArgs p) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int BK = 128;                        // one MFMA depth per k-step (bytes = digits)
  constexpr int ROW = S * BK + (S % 2 ? 0 : BK);  // bytes per staged row (odd multiple of 128)
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int CPR = S * 8;
  constexpr int CHUNKS = (BM + BN) * CPR;
  constexpr int CPT = (CHUNKS + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) unsigned char sm[2][(BM + BN) * ROW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  int64_t tm, tn;
  xcd_tile(blockIdx.x, (p.Mp / BM) * (p.Np / BN), p.Mp / BM, p.Np / BN, &tm, &tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const unsigned char* __restrict__ PA = (const unsigned char*)p.pa;
  const unsigned char* __restrict__ PB = (const unsigned char*)p.pb;
  const int64_t rowlen = p.Kp * S;

  // chunk q of digit s of staged row r sits at slot q ^ ((r >> 1) & 7)
  auto lds_off = [](int r, int s_, int q) { return r * ROW + s_ * BK + ((q ^ ((r >> 1) & 7)) << 4); };
  Stager<unsigned char, CPT, CHUNKS, NT> stg;
  const unsigned char* srow[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int c = tid + i * NT;
    const int row = (c < CHUNKS ? c : 0) / CPR, sub = (c < CHUNKS ? c : 0) % CPR;
    srow[i] = (row < BM ? PA + (m0 + row) * rowlen : PB + (n0 + row - BM) * rowlen) + sub * 16;
    stg.dst[i] = lds_off(row, sub >> 3, sub & 7);
  }
  auto frag = [&](const unsigned char* st, int row, int s_) -> i8v {
    const u32x4 lo = *(const u32x4*)(st + lds_off(row, s_, 2 * fq_of(lane)));
    const u32x4 hi = *(const u32x4*)(st + lds_off(row, s_, 2 * fq_of(lane) + 1));
    return i8v{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
  };

  // Every FP8 digit product is an integer below 2^8 times the block scales
  // (which put each level at its true relative weight 2^(-5g)).  Levels 0 to 4
  // keep their own FP32 accumulators, exact for 4096 contracted indices
  // ((g+1) 4096 2^8 < 2^24); deeper levels (2^-25 and below) share one.
  // Flushed to FP64 every 4096.
  constexpr int NACC = S < 6 ? S : 6;
  f4 acc[NACC][TM][TN];
  double acc64[TM][TN][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
#pragma unroll
      for (int g = 0; g < NACC; ++g) acc[g][i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
    }
  const int64_t ksteps = p.Kp / BK;
  stg.load(srow, 0, tid);
  stg.store(sm[0], tid);
  __syncthreads();
  const int fr = lane & 15, fq = lane >> 4;
  for (int64_t ks = 0; ks < ksteps; ++ks) {
    const int cur = ks & 1;
    if (ks + 1 < ksteps) stg.load(srow, (ks + 1) * (S * BK), tid);
    const unsigned char* st = sm[cur];
    i8v af[S][TM];
#pragma unroll
    for (int s_ = 0; s_ < S; ++s_)
#pragma unroll
      for (int i = 0; i < TM; ++i) af[s_][i] = frag(st, wm * WM + i * 16 + fr, s_);
#pragma unroll
    for (int t = 0; t < S; ++t) {
      i8v bfr[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) bfr[j] = frag(st, BM + wn * WN + j * 16 + fr, t);
#pragma unroll
      for (int s_ = 0; s_ + t < S; ++s_) {
        // digit plane s carries 2^(-5s): E8M0 scale 127 - 5s (127 = 2^0)
        const int g = s_ + t < NACC ? s_ + t : NACC - 1;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[g][i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(af[s_][i], bfr[j], acc[g][i][j], 0, 0, 0,
                                                                          127 - 5 * s_, 0, 127 - 5 * t);
      }
    }
    if ((ks & 31) == 31 || ks + 1 == ksteps) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double v = 0.0;
#pragma unroll
            for (int g = NACC - 1; g >= 0; --g) v += (double)acc[g][i][j][r];
            acc64[i][j][r] += v;
          }
#pragma unroll
          for (int g = 0; g < NACC; ++g) acc[g][i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    if (ks + 1 < ksteps) stg.store(sm[cur ^ 1], tid);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + wm * WM + i * 16 + fq * 4 + r;
      if (m >= p.M) continue;
      const double sm_ = p.sa[m] * p.unit * p.alpha;
      const int64_t cm = off_at(p.cM, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + wn * WN + j * 16 + fr;
        if (n >= p.N) continue;
        double* dst = p.C + cm + off_at(p.cN, n);
        double v = sm_ * p.sb[n] * acc64[i][j][r];
        if (p.beta != 0.0) v += p.beta * *dst;
        *dst = v;
      }
    }
  }
}

// ---------------------------------------------------------------- residues
// Moduli as FP64 for the residue pass (exact integers and rounded reciprocals).
struct CrtModuli {
  int n;
  double p[kCrtMaxModuli];
  double inv[kCrtMaxModuli];
};

// Integers y = rint(2^bits X[r,k] / sigma_r) (|y| <= 2^bits <= 2^48, exact in
// FP64) of one 64 x 64 tile, written as residues modulo each p_i into the
// int8 planes [i][Kp/64][Rp][64]: one k-step of 64 contracted indices of all
// rows is contiguous, so the tile lands as one 4 KB block per modulus and a
// k-step of a GEMM tile is one contiguous run of its rows.  Workgroup b
// covers row block b % (Rp / 64) and k block b / (Rp / 64).
//
// For |y| <= 2^48 the product of y and the rounded reciprocal of p is within
// 1/(16p) of y/p, closer than any half-integer is for odd p, so
// q = rint(y / p) is the nearest integer and r = y - q p (one exact FMA) lies
// in [-(p-1)/2, (p-1)/2].  For p = 256 the product is exact and r may be 128,
// whose byte 0x80 reads back as -128: the same residue.
__global__ __launch_bounds__(256) void crt_planes_kernel(const double* __restrict__ X, Offs xr, Offs xk, int64_t R,
                                                         int64_t K, int64_t Rp, int64_t Kp,
                                                         const double* __restrict__ sigma, int rfast, double lift,
                                                         CrtModuli md, signed char* __restrict__ planes) {
  __shared__ double tile[64][65];
  const int tid = threadIdx.x;
  const int64_t rblocks = Rp / 64;
  const int64_t kb = (int64_t)blockIdx.x / rblocks;
  const int64_t r0 = ((int64_t)blockIdx.x - kb * rblocks) * 64, k0 = kb * 64;
  gather_tile64(X, xr, xk, R, K, r0, k0, rfast, tile);
  __syncthreads();
  // a thread takes 16 consecutive k of one row: one 16-byte store per modulus
  const int rr = tid >> 2, kk0 = (tid & 3) * 16;
  const int64_t r = r0 + rr;
  const double sg = sigma[r];
  double y[16];
  // exact scaling by powers of two: one factor 2^bits / sg unless it would overflow
  if (sg >= 0x1p-969) {
    const double f = lift / sg;
#pragma unroll
    for (int v = 0; v < 16; ++v) y[v] = rint(tile[rr][kk0 + v] * f);
  } else {
#pragma unroll
    for (int v = 0; v < 16; ++v) y[v] = sg > 0.0 ? rint(tile[rr][kk0 + v] / sg * lift) : 0.0;
  }
  signed char* dst = planes + k0 * Rp + r * 64 + kk0;  // k0 is a multiple of 64
  const int64_t plane = Rp * Kp;
  for (int i = 0; i < md.n; ++i) {
    const double p = md.p[i], inv = md.inv[i];
    u32x4 word = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const double q = rint(y[v] * inv);
      const int rm = (int)fma(-q, p, y[v]);
      word[v >> 2] |= ((unsigned)rm & 255u) << (8 * (v & 3));
    }
    *reinterpret_cast<u32x4*>(dst + i * plane) = word;
  }
}

typedef int i4 __attribute__((ext_vector_type(4)));

// Register stage of one k-step of the residue planes: each thread moves CPT
// 16-byte chunks.  The first ACH chunks of the tile belong to A; with ACH a
// multiple of NT, chunk i of every thread comes from the same operand, so the
// k-step base of each operand is one uniform pointer and a chunk needs only
// its 32-bit offset.
template <int CPT, int CHUNKS, int NT, int ACH>
struct KStager {
  static_assert(ACH % NT == 0, "each chunk slot from one operand");
  u32x4 v[CPT];
  int dst[CPT];
  __device__ inline void load(const signed char* a, const signed char* b, const int (&off)[CPT], int tid) {
#pragma unroll
    for (int i = 0; i < CPT; ++i)
      if (CHUNKS % NT == 0 || tid + i * NT < CHUNKS) v[i] = *(const u32x4*)((i * NT < ACH ? a : b) + off[i]);
  }
  __device__ inline void store(signed char* st, int tid) const {
#pragma unroll
    for (int i = 0; i < CPT; ++i)
      if (CHUNKS % NT == 0 || tid + i * NT < CHUNKS) *(u32x4*)(st + dst[i]) = v[i];
  }
};

struct CrtGemmArgs {
  const signed char* pa;   // residues of the kernel's A: [n][Kp/64][Mp][64]
  const signed char* pb;   // residues of the kernel's B: [n][Kp/64][Np][64]
  unsigned char* z;        // residues of the product in [0, p): [n][Np][Mp], or [n][Mp][Np] when zt
  int64_t Mp, Np, Kp;
  int n;
  int zt;                  // 1: rows of z along m (n contiguous), to match an output stride-1 along n
  int p[kCrtMaxModuli];
};

// LDS slot of 16-byte chunk q (of 4) of staged row r (64 bytes) in the
// register-staged kernels is q ^ crt_swizzle(r): the 16 rows of one fragment
// read fall in 16 distinct 16-byte bank groups.
TC_DEV int crt_swizzle(int r) { return (r >> 2) & 3; }

// Product residues z = Z mod p in [0, p) of one wavefront's TM x TN
// fragments (rows from mw, columns from nw), one byte per output.
template <int TM, int TN, int WM, int WN>
TC_DEV void crt_store_residues(const CrtGemmArgs& g, const i4 (&acc)[TM][TN], int mod, int p, int64_t mw, int64_t nw,
                               int lane) {
  const int fr = lane & 15, fq = lane >> 4;
  unsigned char* __restrict__ Z = g.z + (int64_t)mod * g.Mp * g.Np;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t m = mw + i * 16 + fq * 4;
      const int64_t n = nw + j * 16 + fr;
      unsigned word = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int v = acc[i][j][r] % p;
        v += v < 0 ? p : 0;
        word |= (unsigned)v << (8 * r);
      }
      if (g.zt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Z[(m + r) * g.Np + n] = (unsigned char)(word >> (8 * r));
      } else {
        *reinterpret_cast<unsigned*>(Z + n * g.Mp + m) = word;
      }
    }
}

// Tile of the residue GEMM for workgroup bid: modulus, first row, first column.
TC_DEV void crt_tile_of(const CrtGemmArgs& g, int BM, int BN, int* mod, int* p, int64_t* m0, int64_t* n0) {
  const int64_t tilesM = g.Mp / BM, tilesN = g.Np / BN;
  int64_t tmx, tn;
  xcd_tile(blockIdx.x, tilesM * g.n * tilesN, tilesM * g.n, tilesN, &tmx, &tn);
  *mod = (int)(tmx / tilesM);
  *m0 = (tmx - (int64_t)*mod * tilesM) * BM;
  *n0 = tn * BN;
  int q = g.p[0];
#pragma unroll
  for (int i = 1; i < kCrtMaxModuli; ++i) q = *mod == i ? g.p[i] : q;  // no dynamic index into the arguments
  *p = q;
}

// One residue product per workgroup tile and modulus: Z_i = A_i B_i exactly in
// INT32 (v_mfma_i32_16x16x64_i8), stored reduced modulo p_i.  Lane l supplies
// 16 int8 of row l%16 of A and of column l%16 of B from the same 16
// contracted positions (chunk l/16 of the 64), so any order the matrix core
// gives those positions pairs A and B alike; accumulator element r holds
// D[4(l/16) + r][l%16].  The tiles of all moduli are one sequence of row
// blocks for the XCD-aware walk (modulus-major), so concurrent workgroups share
// residue planes.  PF k-steps of global loads are in flight (register
// stages) while the matrix cores work on the k-step staged in LDS.
template <int BM, int BN, int WGM, int WGN, int PF>
__global__ __launch_bounds__(64 * WGM * WGN) void crt_gemm_kernel(CrtGemmArgs g) {
  static_assert(PF == 1 || PF == 2, "one or two k-steps in flight");
  constexpr int BK = kCrtBK;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int CPR = BK / 16;  // 16-byte chunks per staged row
  constexpr int CHUNKS = (BM + BN) * CPR;
  constexpr int CPT = (CHUNKS + NT - 1) / NT;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 16, TN = WN / 16;
  __shared__ __attribute__((aligned(16))) signed char sm[2][(BM + BN) * BK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  int mod, p;
  int64_t m0, n0;
  crt_tile_of(g, BM, BN, &mod, &p, &m0, &n0);

  const signed char* __restrict__ PA = g.pa + (int64_t)mod * g.Mp * g.Kp;
  const signed char* __restrict__ PB = g.pb + (int64_t)mod * g.Np * g.Kp;
  auto lds_off = [](int r, int q) { return r * BK + ((q ^ crt_swizzle(r)) << 4); };
  KStager<CPT, CHUNKS, NT, BM * CPR> stg[PF];
  int soff[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int c = tid + i * NT;
    const int row = (c < CHUNKS ? c : 0) / CPR, sub = (c < CHUNKS ? c : 0) % CPR;
    soff[i] = (row < BM ? row : row - BM) * BK + sub * 16;
#pragma unroll
    for (int f = 0; f < PF; ++f) stg[f].dst[i] = lds_off(row, sub);
  }
  // k-step ks of this tile's rows: one contiguous run per operand
  const signed char* const PA0 = PA + m0 * BK;
  const signed char* const PB0 = PB + n0 * BK;
  const int64_t kstepA = g.Mp * BK, kstepB = g.Np * BK;
  auto load = [&](KStager<CPT, CHUNKS, NT, BM * CPR>& st, int64_t ks) {
    st.load(PA0 + ks * kstepA, PB0 + ks * kstepB, soff, tid);
  };
  i4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = i4{0, 0, 0, 0};

  // every residue product is at most 2^14 in magnitude: reducing the sums
  // modulo p every 2^16 contracted indices keeps them below 2^31
  constexpr int64_t kReduce = 65536 / BK;
  const int64_t ksteps = g.Kp / BK, last = ksteps - 1;
  const int fr = lane & 15, fq = lane >> 4;
  auto compute = [&](const signed char* st, int64_t ks) {
    i4 af[TM], bfr[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) af[i] = *(const i4*)(st + lds_off(wm * WM + i * 16 + fr, fq));
#pragma unroll
    for (int j = 0; j < TN; ++j) bfr[j] = *(const i4*)(st + lds_off(BM + wn * WN + j * 16 + fr, fq));
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[i], bfr[j], acc[i][j], 0, 0, 0);
    if ((ks + 1) % kReduce == 0) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j][r] %= p;
    }
  };
  if constexpr (PF == 1) {
    load(stg[0], 0);
    stg[0].store(sm[0], tid);
    __syncthreads();
    for (int64_t ks = 0; ks < ksteps; ++ks) {
      const int cur = ks & 1;
      if (ks + 1 < ksteps) load(stg[0], ks + 1);
      compute(sm[cur], ks);
      if (ks + 1 < ksteps) stg[0].store(sm[cur ^ 1], tid);
      __syncthreads();
    }
  } else {
    // Two register sets, each k-step loaded two steps ahead; the loop is
    // unrolled by two so that each half names its sets statically.  Loads past
    // the end repeat the last k-step (in bounds; staged into a buffer that is
    // not read again), so every half has the same shape.
    load(stg[0], 0);
    load(stg[PF - 1], last < 1 ? last : 1);
    stg[0].store(sm[0], tid);
    __syncthreads();
    for (int64_t ks = 0; ks < ksteps; ks += 2) {
      load(stg[0], ks + 2 < last ? ks + 2 : last);
      compute(sm[0], ks);
      stg[PF - 1].store(sm[1], tid);  // k-step ks + 1
      __syncthreads();
      if (ks + 1 >= ksteps) break;
      load(stg[PF - 1], ks + 3 < last ? ks + 3 : last);
      compute(sm[1], ks + 1);
      stg[0].store(sm[0], tid);       // k-step ks + 2
      __syncthreads();
    }
  }
  crt_store_residues<TM, TN, WM, WN>(g, acc, mod, p, m0 + wm * WM, n0 + wn * WN, lane);
}

// The same product with the k-steps copied straight from global memory into
// LDS (global_load_lds_dwordx4: lane l of a wavefront lands 16 bytes at the
// uniform LDS base + 16 l), NS stages deep, so NS - 1 k-steps are in flight
// without holding registers.  One stage is the tile's BM + BN rows of one
// k-step, stored in fragment order: the 16 rows of group g take 1 KB at
// 1024 g, chunk q (of 4) of row 16 g + j at 256 q + 16 j.  A fragment read
// (lane l: row l%16 of the group, chunk l/16) is then one contiguous 1 KB, free
// of bank conflicts however the LDS groups lanes, and a wavefront's copy of
// group g (lane l fetching that same row and chunk) is one instruction.
// Waits: a wavefront's own copies of k-step ks are complete once at most the
// CPW (NS - 2) copies issued after them are outstanding (vmcnt), and the barrier
// that follows makes every wavefront's copies visible and frees the stage
// computed in the previous step.  Copies past the last k-step repeat it into
// that freed stage, which is not read again, so every step has the same shape.
template <int BM, int BN, int WGM, int WGN, int NS>
__global__ __launch_bounds__(64 * WGM * WGN) void crt_gemm_dma_kernel(CrtGemmArgs g) {
  constexpr int BK = kCrtBK;
  constexpr int NW = WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int STAGE = (BM + BN) * BK;          // bytes per stage
  constexpr int CH = (BM + BN) / 16;             // 1 KB copies per stage
  static_assert(CH % NW == 0 && BM % 16 == 0, "whole copies per wavefront, none straddling A and B");
  constexpr int CPW = CH / NW;                   // copies per wavefront per k-step
  static_assert(CPW * (NS - 2) <= 15, "wait count fits the vmcnt field");
  extern __shared__ __attribute__((aligned(16))) signed char dsm[];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  int mod, p;
  int64_t m0, n0;
  crt_tile_of(g, BM, BN, &mod, &p, &m0, &n0);
  const signed char* __restrict__ PA = g.pa + (int64_t)mod * g.Mp * g.Kp + m0 * BK;
  const signed char* __restrict__ PB = g.pb + (int64_t)mod * g.Np * g.Kp + n0 * BK;
  const int64_t kstepA = g.Mp * BK, kstepB = g.Np * BK;
  // fragment-order offset of (row group base b, lane l): 64 b + 16 l
  auto frag_off = [](int b, int l) { return b * BK + l * 16; };
  // this lane's source offset within each of its copies (rows 16c .. 16c+15)
  int src[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = wave + NW * j;
    const int r = 16 * c + (lane & 15);
    const int q = lane >> 4;
    src[j] = (r < BM ? r : r - BM) * BK + q * 16;
  }
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);  // uniform: LDS addresses in scalar arithmetic
  auto issue = [&](int64_t ks, int stage) {
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int c = wave_u + NW * j;
      const signed char* base = 16 * c < BM ? PA + ks * kstepA : PB + ks * kstepB;
      __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)(base + src[j]),
                                       (void __attribute__((address_space(3)))*)(dsm + stage * STAGE + c * 1024),
                                       16, 0, 0);
    }
  };
  i4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = i4{0, 0, 0, 0};
  constexpr int64_t kReduce = 65536 / BK;
  const int64_t ksteps = g.Kp / BK, last = ksteps - 1;
#pragma unroll
  for (int s = 0; s < NS - 1; ++s) issue(s < last ? s : last, s);
  for (int64_t ks = 0; ks < ksteps; ++ks) {
    // vmcnt <= CPW (NS - 2): simm16 = vmcnt[3:0] | expcnt 7 << 4 | lgkmcnt 15 << 8.
    // A bare s_barrier, not __syncthreads(): its workgroup fence would wait for
    // every copy in flight.  The empty asm keeps the compiler from moving LDS
    // reads above the barrier.
    __builtin_amdgcn_s_waitcnt((CPW * (NS - 2)) | (7 << 4) | (15 << 8));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    const int64_t nk = ks + NS - 1;
    issue(nk < last ? nk : last, (int)(nk % NS));
    const signed char* st = dsm + (ks % NS) * STAGE;
    i4 af[TM], bfr[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) af[i] = *(const i4*)(st + frag_off(wm * WM + i * 16, lane));
#pragma unroll
    for (int j = 0; j < TN; ++j) bfr[j] = *(const i4*)(st + frag_off(BM + wn * WN + j * 16, lane));
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[i], bfr[j], acc[i][j], 0, 0, 0);
    if ((ks + 1) % kReduce == 0) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j][r] %= p;
    }
  }
  // the repeated copies of the tail must land before the workgroup's LDS is released
  __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
  crt_store_residues<TM, TN, WM, WN>(g, acc, mod, p, m0 + wm * WM, n0 + wn * WN, lane);
}

// The copy-fed residue product for 8 wavefronts (each 64 x 128 or 128 x 64
// of the tile) with the schedule pipelined: the fragments of k-step ks + 1
// are read from LDS between the MFMAs of k-step ks (two register sets
// alternating), and the copies of k-step ks + NS - 1 are spread between them
// too, so the matrix cores are not left idle while reads and copies issue.
// One barrier per k-step, before its MFMAs: after it k-step ks + 1 is visible
// to every wavefront (each first waits for its own copies of it: at most the
// CPW (NS - 3) copies issued after them outstanding) and the stage of k-step
// ks - 1 -- whose fragments were all read during k-step ks - 2 and consumed
// by the MFMAs of k-step ks - 1 -- is free for the copies issued after it.
// Copies past the last k-step repeat it into that freed stage.
template <int BM, int BN, int WGM, int WGN, int NS>
__global__ __launch_bounds__(64 * WGM * WGN) void crt_gemm_pipe_kernel(CrtGemmArgs g) {
  constexpr int BK = kCrtBK;
  constexpr int NW = WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int STAGE = (BM + BN) * BK;          // bytes per stage
  constexpr int CH = (BM + BN) / 16;             // 1 KB copies per stage
  static_assert(CH % NW == 0 && BM % 16 == 0, "whole copies per wavefront, none straddling A and B");
  constexpr int CPW = CH / NW;                   // copies per wavefront per k-step
  static_assert(NS >= 3 && CPW * (NS - 2) <= 15, "ring of three or more stages; wait count fits the vmcnt field");
  constexpr int NM = TM * TN, NR = TM + TN;
  extern __shared__ __attribute__((aligned(16))) signed char dsm[];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  int mod, p;
  int64_t m0, n0;
  crt_tile_of(g, BM, BN, &mod, &p, &m0, &n0);
  const signed char* const PA = g.pa + (int64_t)mod * g.Mp * g.Kp + m0 * BK;
  const signed char* const PB = g.pb + (int64_t)mod * g.Np * g.Kp + n0 * BK;
  const int64_t kstepA = g.Mp * BK, kstepB = g.Np * BK;
  // Copy j of this wavefront fills 1 KB block c = wave + NW j (rows 16c ..
  // 16c+15, chunk lane/16); the first BM / 16 blocks are A's, a whole number
  // per wavefront, so copy j reads A for j < BM / (16 NW).  Its address is a
  // uniform base (the operand's k-step) plus this lane's 32-bit offset, and
  // its LDS address is uniform: no vector arithmetic per copy.
  static_assert((BM / 16) % NW == 0, "A's copies must split evenly over the wavefronts");
  constexpr int CPA = BM / 16 / NW;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  uint32_t voff[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int r = 16 * (wave + NW * j) + (lane & 15);
    voff[j] = (uint32_t)((j < CPA ? r : r - BM) * BK + (lane >> 4) * 16);
  }
  auto copy1 = [&](int j, int64_t ks, int stage) {
    const int c = wave_u + NW * j;
    const signed char* base = j < CPA ? PA + ks * kstepA : PB + ks * kstepB;
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)(base + voff[j]),
                                     (void __attribute__((address_space(3)))*)(dsm + stage * STAGE + c * 1024), 16,
                                     0, 0);
  };
  // fragment-order offsets: row group base b, lane l at 64 b + 16 l
  const int a_lds = (wm * WM) * BK + lane * 16, b_lds = (BM + wn * WN) * BK + lane * 16;
  i4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = i4{0, 0, 0, 0};
  // every residue product is at most 2^14 in magnitude: reducing the sums
  // modulo p every 2^16 contracted indices keeps them below 2^31
  constexpr int64_t kReduce = 65536 / BK;
  static_assert(kReduce % 2 == 0, "the loop takes k-steps in pairs");
  const int64_t ksteps = g.Kp / BK, last = ksteps - 1;
#pragma unroll
  for (int s = 0; s < NS - 1; ++s)
#pragma unroll
    for (int j = 0; j < CPW; ++j) copy1(j, s < last ? s : last, s);
  __builtin_amdgcn_s_waitcnt((CPW * (NS - 2)) | (7 << 4) | (15 << 8));  // this wavefront's copies of k-step 0
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
  i4 fa0[TM], fb0[TN], fa1[TM], fb1[TN];
#pragma unroll
  for (int q = 0; q < TM; ++q) fa0[q] = *(const i4*)(dsm + a_lds + q * 16 * BK);
#pragma unroll
  for (int q = 0; q < TN; ++q) fb0[q] = *(const i4*)(dsm + b_lds + q * 16 * BK);
  int st = 0;  // stage of k-step ks
  // k-step ks on (fa, fb); reads k-step ks + 1 into (ga, gb)
  auto body = [&](int64_t ks, const i4 (&fa)[TM], const i4 (&fb)[TN], i4 (&ga)[TM], i4 (&gb)[TN]) {
    __builtin_amdgcn_s_waitcnt((CPW * (NS - 3)) | (7 << 4) | (15 << 8));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    const int64_t nk = ks + NS - 1;
    const int cs = (st + NS - 1) % NS, rs = (st + 1) % NS;
    const signed char* nx = dsm + rs * STAGE;
    constexpr int SPAN = (2 * NM) / 3;  // reads in the first two thirds of the MFMAs
#pragma unroll
    for (int q = 0; q < NM; ++q) {
      acc[q / TN][q % TN] =
          __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[q / TN], fb[q % TN], acc[q / TN][q % TN], 0, 0, 0);
      const bool r = q < SPAN && q * NR / SPAN != (q + 1) * NR / SPAN;
      const bool c = q * CPW / NM != (q + 1) * CPW / NM;
      if (r || c) __builtin_amdgcn_sched_barrier(0);
      if (r) {
        const int x = q * NR / SPAN;
        if (x < TM)
          ga[x] = *(const i4*)(nx + a_lds + x * 16 * BK);
        else
          gb[x - TM] = *(const i4*)(nx + b_lds + (x - TM) * 16 * BK);
      }
      if (c) copy1(q * CPW / NM, nk < last ? nk : last, cs);
      if (r || c) __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_sched_barrier(0);
    st = rs;
  };
  int64_t ks = 0;
  for (; ks + 1 < last; ks += 2) {
    body(ks, fa0, fb0, fa1, fb1);
    body(ks + 1, fa1, fb1, fa0, fb0);
    if ((ks + 2) % kReduce == 0) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j][r] %= p;
    }
  }
  if (ks < last) {  // one k-step left before the last
    body(ks, fa0, fb0, fa1, fb1);
#pragma unroll
    for (int q = 0; q < TM; ++q) fa0[q] = fa1[q];
#pragma unroll
    for (int q = 0; q < TN; ++q) fb0[q] = fb1[q];
  }
#pragma unroll
  for (int q = 0; q < NM; ++q)
    acc[q / TN][q % TN] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa0[q / TN], fb0[q % TN], acc[q / TN][q % TN], 0, 0, 0);
  // the repeated copies of the tail must land before the workgroup's LDS is released
  __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
  crt_store_residues<TM, TN, WM, WN>(g, acc, mod, p, m0 + wm * WM, n0 + wn * WN, lane);
}

// Chinese-remainder rebuild: with M_i = P / p_i and w_i = M_i (M_i^-1 mod p_i)
// (each below P), Z = sum_i z_i w_i mod P, taken in (-P/2, P/2].  P < 2^111,
// so the sum of at most 14 terms below 2^8 P fits in 128 bits.
struct CrtRebuild {
  int n;
  unsigned long long w[kCrtMaxModuli][2];  // (low, high) 64-bit words
  unsigned long long P[2];
  double inv_P;
};

// One thread takes four consecutive entries along the output's stride-1
// group (m, or n when zt) at one index of the other (one 4-byte load per
// modulus); C[m,n] = alpha sigma_m tau_n 2^(-2 bits) Z + beta C[m,n].
__global__ __launch_bounds__(256) void crt_rebuild_kernel(const unsigned char* __restrict__ z, int64_t Mp, int64_t Np,
                                                          int zt, const double* __restrict__ sa,
                                                          const double* __restrict__ sb, double* __restrict__ C,
                                                          Offs cM, Offs cN, int64_t M, int64_t N, double unit,
                                                          double alpha, double beta, CrtRebuild cr) {
  typedef unsigned __int128 u128;
  typedef __int128 s128;
  const u128 P = ((u128)cr.P[1] << 64) | cr.P[0];
  // fast group: padded length (a multiple of 4) and true length; slow group: true length
  const int64_t fp = zt ? Np : Mp, fl = zt ? N : M, sl = zt ? M : N;
  const int64_t quads = fp / 4, units = quads * sl, plane = Mp * Np;
  for (int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x; u < units; u += (int64_t)gridDim.x * 256) {
    const int64_t so = u / quads, f4 = (u - so * quads) * 4;
    if (f4 >= fl) continue;
    // sum per 32-bit limb of the weights (each term below 2^40, 14 terms
    // below 2^44), then one carry-propagating 128-bit sum per output
    unsigned long long limb[4][4] = {};
    for (int i = 0; i < cr.n; ++i) {
      const unsigned word = *reinterpret_cast<const unsigned*>(z + i * plane + so * fp + f4);
      const unsigned w0 = (unsigned)cr.w[i][0], w1 = (unsigned)(cr.w[i][0] >> 32);
      const unsigned w2 = (unsigned)cr.w[i][1], w3 = (unsigned)(cr.w[i][1] >> 32);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const unsigned long long zr = (word >> (8 * r)) & 255u;
        limb[r][0] += zr * w0;
        limb[r][1] += zr * w1;
        limb[r][2] += zr * w2;
        limb[r][3] += zr * w3;
      }
    }
    u128 S[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
      S[r] = (u128)limb[r][0] + ((u128)limb[r][1] << 32) + ((u128)limb[r][2] << 64) + ((u128)limb[r][3] << 96);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (f4 + r >= fl) break;
      const int64_t m = zt ? so : f4 + r, n = zt ? f4 + r : so;
      // quotient from FP64 (S / P < 2^12, so the estimate is at most one off)
      const double sd = (double)(unsigned long long)(S[r] >> 64) * 0x1p64 + (double)(unsigned long long)S[r];
      const unsigned long long q = (unsigned long long)floor(sd * cr.inv_P);
      s128 R = (s128)(S[r] - (u128)q * P);
      if (R < 0)
        R += (s128)P;
      else if (R >= (s128)P)
        R -= (s128)P;
      if (2 * R > (s128)P) R -= (s128)P;
      const bool neg = R < 0;
      const u128 U = neg ? (u128)(-R) : (u128)R;
      double v = (double)(unsigned long long)(U >> 64) * 0x1p64 + (double)(unsigned long long)U;
      v = neg ? -v : v;
      double* dst = C + off_at(cM, m) + off_at(cN, n);
      double out = alpha * (sa[m] * (sb[n] * unit) * v);
      if (beta != 0.0) out += beta * *dst;
      *dst = out;
    }
  }
}

// Residue GEMM launch: register-staged (pf 1 or 2 k-steps in flight) or
// copied straight into an LDS ring of pf stages (dynamic LDS beyond 64 KB,
// allowed once per kernel and device).
template <int BM, int BN, int WGM, int WGN, int PF>
hipError_t launch_crt_gemm(const CrtGemmArgs& g, unsigned blocks, hipStream_t s) {
  if constexpr (PF <= 2) {
    hipLaunchKernelGGL((crt_gemm_kernel<BM, BN, WGM, WGN, PF>), dim3(blocks), dim3(64 * WGM * WGN), 0, s, g);
  } else {
    constexpr int bytes = PF * (BM + BN) * kCrtBK;
    static std::atomic<uint64_t> allowed{0};
    if constexpr (WGM * WGN == 8) {  // registers for two fragment sets: the pipelined schedule
      const hipError_t e =
          allow_dynamic_lds((const void*)crt_gemm_pipe_kernel<BM, BN, WGM, WGN, PF>, bytes, allowed);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((crt_gemm_pipe_kernel<BM, BN, WGM, WGN, PF>), dim3(blocks), dim3(64 * WGM * WGN), bytes, s,
                         g);
    } else {
      const hipError_t e = allow_dynamic_lds((const void*)crt_gemm_dma_kernel<BM, BN, WGM, WGN, PF>, bytes, allowed);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((crt_gemm_dma_kernel<BM, BN, WGM, WGN, PF>), dim3(blocks), dim3(64 * WGM * WGN), bytes, s,
                         g);
    }
  }
  return hipGetLastError();
}

// Row scales of one input: one wavefront per row when k is stride-1 (and
// rows are not), else per-segment maxima and a fixed-order second pass.
hipError_t launch_row_scales(const double* X, Offs xr, Offs xk, int64_t R, int64_t K, int64_t Rp, double* sigma,
                             double* part, bool rfast, bool kfast, hipStream_t s) {
  if (kfast && !rfast) {
    hipLaunchKernelGGL(row_scale_wave_kernel, dim3((unsigned)((Rp + 3) / 4)), dim3(256), 0, s, X, xr, xk, R, K, Rp,
                       sigma);
  } else {
    const int64_t nseg = row_max_segments(R, K);
    const int64_t seg_len = (K + nseg - 1) / nseg;
    if (R > 0)
      hipLaunchKernelGGL(row_max_rows_kernel, dim3((unsigned)((R + 255) / 256), (unsigned)nseg), dim3(256), 0, s, X,
                         xr, xk, R, K, seg_len, part);
    hipLaunchKernelGGL(row_scale_from_parts_kernel, dim3((unsigned)((Rp + 255) / 256)), dim3(256), 0, s, part, R,
                       nseg, Rp, sigma);
  }
  return hipGetLastError();
}

hipError_t launch_crt(const SplitParams& sp, hipStream_t s) {
  const int n = sp.slices;
  if (n < 2 || n > kCrtMaxModuli || sp.bits < 1 || sp.bits > kCrtMaxBits) return hipErrorInvalidValue;
  if (sp.crt_tile < 0 || sp.crt_tile >= kCrtNumTiles) return hipErrorInvalidValue;
  const CrtTileCfg t = kCrtTiles[sp.crt_tile];
  if (sp.Mp % t.bm || sp.Np % t.bn || sp.Kp % kCrtBK) return hipErrorInvalidValue;
  CrtModuli md{};
  md.n = n;
  for (int i = 0; i < n; ++i) {
    md.p[i] = kCrtModuli[i];
    md.inv[i] = 1.0 / kCrtModuli[i];
  }
  const double lift = std::ldexp(1.0, sp.bits);
  constexpr int64_t kMaxBlocks = 0xffffffffLL / 256;
  hipError_t e;
  for (int op = 0; op < 2; ++op) {
    const double* X = op ? sp.B : sp.A;
    const Offs xr = op ? sp.bN : sp.aM, xk = op ? sp.bK : sp.aK;
    const int64_t R = op ? sp.N : sp.M, Rp = op ? sp.Np : sp.Mp;
    double* sig = op ? sp.sigB : sp.sigA;
    e = launch_row_scales(X, xr, xk, R, sp.K, Rp, sig, sp.part, op ? sp.b_rfast : sp.a_rfast,
                          op ? sp.b_kfast : sp.a_kfast, s);
    if (e != hipSuccess) return e;
    const int64_t blocks = (Rp / 64) * (sp.Kp / 64);
    if (blocks > kMaxBlocks) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(crt_planes_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, xr, xk, R, sp.K, Rp, sp.Kp, sig,
                       (op ? sp.b_rfast : sp.a_rfast) ? 1 : 0, lift, md,
                       (signed char*)(op ? sp.planesB : sp.planesA));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  CrtGemmArgs g{};
  g.pa = (const signed char*)sp.planesA;
  g.pb = (const signed char*)sp.planesB;
  g.z = (unsigned char*)sp.zres;
  g.Mp = sp.Mp;
  g.Np = sp.Np;
  g.Kp = sp.Kp;
  g.n = n;
  g.zt = sp.c_nfast ? 1 : 0;
  for (int i = 0; i < kCrtMaxModuli; ++i) g.p[i] = kCrtModuli[i];
  const int64_t gblocks = (sp.Mp / t.bm) * (sp.Np / t.bn) * n;
  if (gblocks > kMaxBlocks) return hipErrorInvalidConfiguration;
  switch (sp.crt_tile) {
#define TC_CRT_LAUNCH(id, bm, bn, wgm, wgn, pf)                         \
  case id:                                                            \
    e = launch_crt_gemm<bm, bn, wgm, wgn, pf>(g, (unsigned)gblocks, s); \
    break;
    TC_CRT_TILES(TC_CRT_LAUNCH)
#undef TC_CRT_LAUNCH
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // weights: M_i as the product of the other moduli (no 128-bit division)
  typedef unsigned __int128 u128;
  CrtRebuild cr{};
  cr.n = n;
  u128 P = 1;
  double Pd = 1.0;
  for (int i = 0; i < n; ++i) {
    P *= (unsigned)kCrtModuli[i];
    Pd *= kCrtModuli[i];
  }
  for (int i = 0; i < n; ++i) {
    const unsigned pi = (unsigned)kCrtModuli[i];
    u128 Mi = 1;
    unsigned mi = 1;  // M_i mod p_i
    for (int j = 0; j < n; ++j)
      if (j != i) {
        Mi *= (unsigned)kCrtModuli[j];
        mi = (unsigned)((unsigned long long)mi * (unsigned)kCrtModuli[j] % pi);
      }
    unsigned inv = 0;
    for (unsigned x = 1; x < pi; ++x)
      if ((unsigned long long)mi * x % pi == 1) {
        inv = x;
        break;
      }
    if (inv == 0) return hipErrorInvalidValue;  // moduli not coprime
    const u128 w = Mi * inv;
    cr.w[i][0] = (unsigned long long)w;
    cr.w[i][1] = (unsigned long long)(w >> 64);
  }
  cr.P[0] = (unsigned long long)P;
  cr.P[1] = (unsigned long long)(P >> 64);
  cr.inv_P = 1.0 / Pd;
  const int64_t units = sp.c_nfast ? (sp.Np / 4) * sp.M : (sp.Mp / 4) * sp.N;
  if (units > 0) {
    const int64_t want = (units + 255) / 256;
    const unsigned blocks = (unsigned)(want < kMaxGridBlocks ? want : kMaxGridBlocks);
    hipLaunchKernelGGL(crt_rebuild_kernel, dim3(blocks), dim3(256), 0, s, (const unsigned char*)sp.zres, sp.Mp, sp.Np,
                       sp.c_nfast ? 1 : 0, sp.sigA, sp.sigB, sp.C, sp.cM, sp.cN, sp.M, sp.N, std::ldexp(1.0, -2 * sp.bits), sp.alpha,
                       sp.beta, cr);
  }
  return hipGetLastError();
}

template <int S>
hipError_t launch_planes(const double* X, Offs xr, Offs xk, int64_t R, int64_t K, int64_t Rp, int64_t Kp,
                         double* sigma, double* part, bool rfast, bool kfast, bool fp8, void* planes,
                         hipStream_t s) {
  hipError_t e = launch_row_scales(X, xr, xk, R, K, Rp, sigma, part, rfast, kfast, s);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((Kp + 63) / 64), (unsigned)((Rp + 63) / 64));
  if (fp8)
    hipLaunchKernelGGL((split_planes_kernel<S, true>), grid, dim3(256), 0, s, X, xr, xk, R, K, Rp, Kp, sigma,
                       rfast ? 1 : 0, planes);
  else
    hipLaunchKernelGGL((split_planes_kernel<S, false>), grid, dim3(256), 0, s, X, xr, xk, R, K, Rp, Kp, sigma,
                       rfast ? 1 : 0, planes);
  return hipGetLastError();
}

template <int S>
hipError_t launch_split_gemm(const SplitGemmArgs& a, bool fp8, hipStream_t s) {
  const SplitTile t = split_tile(fp8, S);
  const dim3 grid((unsigned)((a.Mp / t.bm) * (a.Np / t.bn)));
  if (fp8) {
    if constexpr (S <= kSplitMaxFp8)
      hipLaunchKernelGGL((split_gemm_fp8_kernel<32, 32, 2, 2, S>), grid, dim3(256), 0, s, a);
    else
      return hipErrorInvalidValue;
  } else if constexpr (S <= 5) {
    // the copy-fed kernel addresses a tile's rows by 32-bit byte offsets
    if ((double)a.Kp * S * 2.0 * 128.0 >= 2147483648.0) {
      hipLaunchKernelGGL((split_gemm_bf16_kernel<128, 64, 4, 2, S>), grid, dim3(512), 0, s, a);
      return hipGetLastError();
    }
    constexpr int bytes = 2 * (128 / 16 + 64 / 16) * S * 1024;
    static std::atomic<uint64_t> allowed{0};
    const hipError_t e = allow_dynamic_lds((const void*)split_gemm_bf16_dma_kernel<128, 64, 4, 2, S>, bytes, allowed);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((split_gemm_bf16_dma_kernel<128, 64, 4, 2, S>), grid, dim3(512), bytes, s, a);
  } else if constexpr (S <= kSplitMaxBf16) {
    hipLaunchKernelGGL((split_gemm_bf16_kernel<64, 64, 2, 2, S>), grid, dim3(256), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_split_contraction(const SplitParams& sp, hipStream_t s) {
  if (sp.crt) return launch_crt(sp, s);
  const int S = sp.slices;
  const bool fp8 = sp.fp8;
  hipError_t e = hipSuccess;
#define TC_SPLIT_CASE(NS)                                                                                        \
  case NS:                                                                                                       \
    e = launch_planes<NS>(sp.A, sp.aM, sp.aK, sp.M, sp.K, sp.Mp, sp.Kp, sp.sigA, sp.part, sp.a_rfast, sp.a_kfast, \
                          fp8, sp.planesA, s);                                                                   \
    if (e != hipSuccess) return e;                                                                               \
    e = launch_planes<NS>(sp.B, sp.bN, sp.bK, sp.N, sp.K, sp.Np, sp.Kp, sp.sigB, sp.part, sp.b_rfast, sp.b_kfast, \
                          fp8, sp.planesB, s);                                                                   \
    if (e != hipSuccess) return e;                                                                               \
    {                                                                                                            \
      SplitGemmArgs a{sp.planesA, sp.planesB, sp.sigA, sp.sigB, sp.C,  sp.cM, sp.cN,     sp.M,                   \
                      sp.N,       sp.Mp,      sp.Np,   sp.Kp,   sp.alpha, sp.beta, fp8 ? 0x1p-8 : 0x1p-34};      \
      return launch_split_gemm<NS>(a, fp8, s);                                                                   \
    }
  switch (S) {
    TC_SPLIT_CASE(1)
    TC_SPLIT_CASE(2)
    TC_SPLIT_CASE(3)
    TC_SPLIT_CASE(4)
    TC_SPLIT_CASE(5)
    TC_SPLIT_CASE(6)
    TC_SPLIT_CASE(7)
    TC_SPLIT_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef TC_SPLIT_CASE
}

}  // namespace tc
