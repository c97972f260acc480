// Persistent batch kernel: many independent contractions of any shapes in one
// launch.
//
// The host turns every contraction of the batch into tasks -- GEMM tiles for
// contractions run by the FP64 MFMA tile engine, groups of batch indices for
// batch-dominated ones run by the slab engine, groups of outputs for the
// memory-bound matrix-vector and inner-product shapes (lanes along the
// contracted index or along the outputs, long contracted ranges cut into
// segments whose partial sums the last segment adds in a fixed order) -- and
// orders all tasks by
// estimated cost, largest first (longest-processing-time order), then cut
// into consecutive chunks of about equal cost.  The grid is sized to the
// number of workgroups the chip holds at once; each workgroup repeatedly takes
// the next chunk index from a global counter (atomic add) and runs its tasks,
// until the counter passes the chunk count.  Every workgroup
// reaches that exit, so the grid always drains.  Pointers and scalars of the
// contractions are read from a small device array written before each launch,
// so one captured graph serves every execution of the batch.
#include "batched_slab.hpp"
#include "gett_tile.hpp"
#include "lanes.hpp"

namespace tc {
namespace {

// Values the whole workgroup shares, made wavefront-uniform so that the
// compiler keeps them (and what is loaded through them) in scalar registers.
TC_DEV int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
TC_DEV int64_t uni64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

TC_DEV double batch_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Completion of one contracted segment of a split task group: returns true in
// the workgroup that finished the last segment (all partial sums visible).
TC_DEV bool batch_last_segment(unsigned* cnt, int S, int* last) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) *last = atomicAdd(cnt, 1u) == (unsigned)(S - 1);
  __syncthreads();
  if (*last) __threadfence();
  return *last;
}

// C entry of output o = m + M (n + N l) (kinds 2 and 3 when n is not fastest).
TC_DEV void batch_store(const GettParams& p, int64_t m, int64_t n, int64_t l, double v) {
  double* dst = p.C + off_at(p.cL, l) + off_at(p.cM, m) + off_at(p.cN, n);
  *dst = p.beta == 0.0 ? p.alpha * v : p.alpha * v + p.beta * *dst;
}

// Lanes over k: the (output, contracted segment) units of the item are
// numbered u = o * S + s, and wavefront w of the workgroup takes unit
// 4 idx + w (so the four wavefronts share an output's segments when outputs
// are few).  Lanes stride along k.  With S > 1 each wavefront stores its
// partial sum and counts its output's finished segments; the wavefront that
// finishes the last one adds the S partial sums in a fixed order.
TC_DEV void batch_lanes_k(const BatchItem& it, const GettParams& p, const BatchTask& task,
                          double* __restrict__ parts, unsigned* __restrict__ tile_cnt) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t outputs = p.M * p.N * p.L;
  const int S = it.ksplit;
  const int64_t u = task.idx * kLanesKOutputs + wave;
  if (u >= outputs * S) return;  // uniform per wavefront; no workgroup barrier follows
  const int64_t o = u / S;
  const int s = (int)(u - o * S);
  const int64_t m = o % p.M;
  const int64_t r = o / p.M;
  const int64_t n = r % p.N;
  const int64_t l = r / p.N;
  const double* __restrict__ A = p.A + off_at(p.aL, l) + off_at(p.aM, m);
  const double* __restrict__ B = p.B + off_at(p.bL, l) + off_at(p.bN, n);
  const int64_t kend = it.kblk ? it.nblk : p.K;
  const int64_t k0 = (int64_t)s * it.seg_len;
  const int64_t k1 = k0 + it.seg_len < kend ? k0 + it.seg_len : kend;
  double v;
  if (it.kblk) {
    const int lp = lane % it.kbp, lq = lane / it.kbp;
    v = batch_wave_sum(lanes_k_blocks<8>(A, B, p.aK.tab, p.bK.tab, it.klim.tab, k0, k1, lp * it.ksa_p + lq * it.ksa_q,
                                         lp * it.ksb_p + lq * it.ksb_q, lp, lq));
  } else {
    v = batch_wave_sum(lanes_k_dot_flat<8>(A, B, p.aK, p.bK, k0, k1, lane));
  }
  if (S == 1) {
    if (lane == 0) batch_store(p, m, n, l, v);
    return;
  }
  if (lane == 0) parts[it.part_off + o * S + s] = v;
  __threadfence();
  int last = 0;
  if (lane == 0) last = atomicAdd(&tile_cnt[it.cnt_off + o], 1u) == (unsigned)(S - 1);
  last = __shfl(last, 0, 64);
  if (!last) return;
  __threadfence();
  // segments in a fixed order: lane-strided, then the fixed reduction tree
  double acc = 0.0;
  for (int sg = lane; sg < S; sg += 64) acc += parts[it.part_off + o * S + sg];
  acc = batch_wave_sum(acc);
  if (lane == 0) batch_store(p, m, n, l, acc);
}

// Lanes over outputs: thread t takes output 256 idx + t (n or m fastest
// along lanes) and walks contracted segment seg.
TC_DEV void batch_lanes_out(const BatchItem& it, const GettParams& p, const BatchTask& task,
                                       double* __restrict__ parts, unsigned* __restrict__ tile_cnt, int* last) {
  const int64_t outputs = p.M * p.N * p.L;
  const int64_t o = task.idx * kLanesOutOutputs + threadIdx.x;
  const int S = it.ksplit;
  int64_t m = 0, n = 0, l = 0;
  double v = 0.0;
  if (o < outputs) {
    if (it.n_fastest) {
      n = o % p.N;
      const int64_t r = o / p.N;
      m = r % p.M;
      l = r / p.M;
    } else {
      m = o % p.M;
      const int64_t r = o / p.M;
      n = r % p.N;
      l = r / p.N;
    }
    const double* __restrict__ A = p.A + off_at(p.aL, l) + off_at(p.aM, m);
    const double* __restrict__ B = p.B + off_at(p.bL, l) + off_at(p.bN, n);
    const int64_t k0 = (int64_t)task.seg * it.seg_len;
    const int64_t k1 = k0 + it.seg_len < p.K ? k0 + it.seg_len : p.K;
    v = lanes_out_dot_flat(A, B, p.aK, p.bK, k0, k1);
  }
  if (S == 1) {
    if (o < outputs) batch_store(p, m, n, l, v);
    return;
  }
  if (o < outputs) parts[it.part_off + (int64_t)task.seg * outputs + o] = v;
  if (!batch_last_segment(&tile_cnt[it.cnt_off + task.idx], S, last)) return;
  if (o < outputs) {
    double acc = 0.0;
    for (int sg = 0; sg < S; ++sg) acc += parts[it.part_off + (int64_t)sg * outputs + o];
    batch_store(p, m, n, l, acc);
  }
}

// ENG selects the engine this launch runs (kBatchEngineGemm, kBatchEngineLanes
// or kBatchEngineSlab): its task list holds tasks of that engine only, and the
// instance carries only that engine's code, so the memory-bound engines are
// not held to the occupancy the GEMM tiles' registers and LDS allow.
template <int BM, int BN, int BK, int ENG>
__global__ __launch_bounds__(256) void batch_kernel(const BatchItem* __restrict__ items,
                                                    const BatchPtrs* __restrict__ ptrs,
                                                    const BatchTask* __restrict__ tasks,
                                                    const int64_t* __restrict__ chunks, int64_t nchunks,
                                                    unsigned long long* counter, double* __restrict__ parts,
                                                    unsigned* __restrict__ tile_cnt) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  __shared__ int64_t next;
  __shared__ int last;
  int64_t t = 0, t_end = 0;
  for (;;) {
    __syncthreads();  // the previous task is done with LDS and with `next`
    if (t >= t_end) {
      // take the next chunk of tasks (one atomic per chunk, not per task)
      if (threadIdx.x == 0) next = (int64_t)atomicAdd(counter, 1ull);
      __syncthreads();
      const int64_t c = uni64(next);
      if (c >= nchunks) break;
      t = uni64(chunks[c]);
      t_end = uni64(chunks[c + 1]);
      if (t >= t_end) continue;
    }
    BatchTask task = tasks[t++];
    task.item = uni(task.item);
    task.seg = uni(task.seg);
    task.idx = uni64(task.idx);
    const BatchItem& it = items[task.item];
    const BatchPtrs pt = ptrs[task.item];
    if (ENG == kBatchEngineLanes) {
      GettParams p = it.g;
      p.A = it.swapped ? pt.B : pt.A;
      p.B = it.swapped ? pt.A : pt.B;
      p.C = pt.C;
      p.alpha = pt.alpha;
      p.beta = pt.beta;
      if (it.kind == kBatchLanesK)
        batch_lanes_k(it, p, task, parts, tile_cnt);
      else
        batch_lanes_out(it, p, task, parts, tile_cnt, &last);
    } else if (ENG == kBatchEngineGemm) {
      GettParams p = it.g;
      p.A = it.swapped ? pt.B : pt.A;
      p.B = it.swapped ? pt.A : pt.B;
      p.C = pt.C;
      p.alpha = pt.alpha;
      p.beta = pt.beta;
      const int64_t per = it.tilesM * it.tilesN;
      const int64_t l = task.idx / per, r = task.idx % per;
      const int64_t m0 = (r % it.tilesM) * BM, n0 = (r / it.tilesM) * BN;
      const int S = it.ksplit;
      const int64_t kb = S > 1 ? task.seg * it.seg_len : 0;
      const int64_t ke = S > 1 ? (kb + it.seg_len < p.K ? kb + it.seg_len : p.K) : p.K;
      double* part = S > 1 ? parts + it.part_off + (task.idx * S + task.seg) * (int64_t)(BM * BN) : nullptr;
      switch (it.akf * 2 + it.bkf) {
        case 0: gett_tile<BM, BN, BK, 2, 2, false, false>(p, m0, n0, l, smem, kb, ke, part); break;
        case 1: gett_tile<BM, BN, BK, 2, 2, false, true>(p, m0, n0, l, smem, kb, ke, part); break;
        case 2: gett_tile<BM, BN, BK, 2, 2, true, false>(p, m0, n0, l, smem, kb, ke, part); break;
        default: gett_tile<BM, BN, BK, 2, 2, true, true>(p, m0, n0, l, smem, kb, ke, part); break;
      }
      if (S > 1) {
        // the workgroup that completes the last segment of this tile adds the
        // segments in order and writes C
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) last = atomicAdd(&tile_cnt[it.cnt_off + task.idx], 1u) == (unsigned)(S - 1);
        __syncthreads();
        if (last) {
          __threadfence();
          gett_reduce_tile<BM, BN>(p, m0, n0, l, parts + it.part_off + task.idx * S * (int64_t)(BM * BN), S);
        }
      }
    } else {
      batched_slab(it.b, it.swapped ? pt.B : pt.A, it.swapped ? pt.A : pt.B, pt.C, pt.alpha, pt.beta,
                   task.idx * it.b.P, smem);
    }
  }
}

// One large slab item on its own: workgroup b takes its batch indices
// b P .. b P + P - 1.  The layout comes by value; the pointers and scalars
// of this execution from the staged pointer array.
__global__ __launch_bounds__(256) void batch_slab_direct_kernel(BatchedParams bp, const BatchPtrs* __restrict__ ptrs,
                                                                int item, int swapped) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const BatchPtrs pt = ptrs[item];
  batched_slab(bp, swapped ? pt.B : pt.A, swapped ? pt.A : pt.B, pt.C, pt.alpha, pt.beta, (int64_t)blockIdx.x * bp.P,
               smem);
}

__global__ void batch_reset_kernel(unsigned long long* counter, unsigned* tile_cnt, int64_t n_cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kBatchEngines) counter[i] = 0ull;
  if (i < n_cnt) tile_cnt[i] = 0u;
}

// LDS (bytes) of an engine's launch
size_t engine_lds_bytes(int eng, int gemm_doubles, int slab_lds_doubles) {
  if (eng == kBatchEngineGemm) return (size_t)gemm_doubles * sizeof(double);
  if (eng == kBatchEngineSlab) return (size_t)slab_lds_doubles * sizeof(double);
  return 0;
}

template <int BM, int BN, int BK, int ENG>
hipError_t launch_engine(const BatchLaunch& bl, hipStream_t s) {
  if (bl.nchunks[ENG] == 0) return hipSuccess;
  const size_t lds = engine_lds_bytes(ENG, gett_lds_doubles<BM, BN, BK>(), bl.slab_lds_doubles);
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<BM, BN, BK, ENG>, 256, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  int64_t grid = (int64_t)bl.num_cus * per_cu;
  if (grid > bl.nchunks[ENG]) grid = bl.nchunks[ENG];
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((batch_kernel<BM, BN, BK, ENG>), dim3((unsigned)grid), dim3(256), lds, s, bl.items, bl.ptrs,
                     bl.tasks, bl.chunks[ENG], bl.nchunks[ENG], bl.counter + ENG, bl.parts, bl.tile_cnt);
  return hipGetLastError();
}

template <int BM, int BN, int BK>
hipError_t launch_cfg(const BatchLaunch& bl, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3((unsigned)((bl.n_cnt + 255) / 256 + 1)), dim3(256), 0, s, bl.counter,
                     bl.tile_cnt, bl.n_cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the engines one after the other: GEMM tiles, then the memory-bound
  // inner products and matrix-vector groups, then the slabs
  if ((e = launch_engine<BM, BN, BK, kBatchEngineGemm>(bl, s)) != hipSuccess) return e;
  if ((e = launch_engine<BM, BN, BK, kBatchEngineLanes>(bl, s)) != hipSuccess) return e;
  if ((e = launch_engine<BM, BN, BK, kBatchEngineSlab>(bl, s)) != hipSuccess) return e;
  for (int d = 0; d < bl.ndirect; ++d) {
    const BatchItem& it = bl.host_items[bl.direct_items[d]];
    hipLaunchKernelGGL(batch_slab_direct_kernel, dim3((unsigned)bl.direct_blocks[d]), dim3(256),
                       (size_t)bl.slab_lds_doubles * sizeof(double), s, it.b, bl.ptrs, bl.direct_items[d], it.swapped);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

int batch_slab_blocks_per_cu(int slab_lds_doubles) {
  int n = 0;
  // the slab engine's code is the same in every tile configuration
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &n, batch_kernel<64, 64, 16, kBatchEngineSlab>, 256, (size_t)slab_lds_doubles * sizeof(double));
  return e == hipSuccess ? n : 0;
}

hipError_t launch_batch(const BatchLaunch& bl, hipStream_t s) {
  if (bl.ntasks == 0 && bl.ndirect == 0) return hipSuccess;
  switch (bl.config) {
#define TC_BCFG(id, bm, bn, bk) \
  case id: return launch_cfg<bm, bn, bk>(bl, s);
    TC_BATCH_TILES(TC_BCFG)
#undef TC_BCFG
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tc
