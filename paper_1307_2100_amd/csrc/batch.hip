// Persistent batch kernel: many independent contractions of any shapes in one
// launch.
//
// The host turns every contraction of the batch into tasks -- GEMM tiles for
// contractions run by the FP64 MFMA tile engine, groups of batch indices for
// batch-dominated ones run by the slab engine -- and orders all tasks by
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

namespace tc {
namespace {

template <int BM, int BN, int BK>
__global__ __launch_bounds__(256) void batch_kernel(const BatchItem* __restrict__ items,
                                                    const BatchPtrs* __restrict__ ptrs,
                                                    const BatchTask* __restrict__ tasks,
                                                    const int64_t* __restrict__ chunks, int64_t nchunks,
                                                    unsigned long long* counter, double* __restrict__ parts,
                                                    unsigned* __restrict__ tile_cnt) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  __shared__ int64_t next;
  __shared__ int last;
  // slab layout of the current item, staged in LDS: the per-element decode
  // loops read it many times
  __shared__ BatchedParams sbp;
  int sbp_item = -1;
  int64_t t = 0, t_end = 0;
  for (;;) {
    __syncthreads();  // the previous task is done with LDS and with `next`
    if (t >= t_end) {
      // take the next chunk of tasks (one atomic per chunk, not per task)
      if (threadIdx.x == 0) next = (int64_t)atomicAdd(counter, 1ull);
      __syncthreads();
      const int64_t c = next;
      if (c >= nchunks) break;
      t = chunks[c];
      t_end = chunks[c + 1];
      if (t >= t_end) continue;
    }
    const BatchTask task = tasks[t++];
    const BatchItem& it = items[task.item];
    const BatchPtrs pt = ptrs[task.item];
    if (it.kind == 0) {
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
      double* part = S > 1 ? parts + (it.part_off + task.idx * S + task.seg) * (int64_t)(BM * BN) : nullptr;
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
          gett_reduce_tile<BM, BN>(p, m0, n0, l, parts + (it.part_off + task.idx * S) * (int64_t)(BM * BN), S);
        }
      }
    } else {
      if (task.item != sbp_item) {
        constexpr int W = (int)(sizeof(BatchedParams) / sizeof(uint32_t));
        static_assert(sizeof(BatchedParams) % sizeof(uint32_t) == 0, "word copy");
        for (int w = threadIdx.x; w < W; w += blockDim.x)
          reinterpret_cast<uint32_t*>(&sbp)[w] = reinterpret_cast<const uint32_t*>(&it.b)[w];
        sbp_item = task.item;
        __syncthreads();
      }
      batched_slab(sbp, it.swapped ? pt.B : pt.A, it.swapped ? pt.A : pt.B, pt.C, pt.alpha, pt.beta,
                   task.idx * sbp.P, smem);
    }
  }
}

__global__ void batch_reset_kernel(unsigned long long* counter, unsigned* tile_cnt, int64_t n_cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *counter = 0ull;
  if (i < n_cnt) tile_cnt[i] = 0u;
}

template <int BM, int BN, int BK>
hipError_t launch_cfg(const BatchLaunch& bl, hipStream_t s) {
  const size_t lds = batch_lds_bytes(bl.config, bl.slab_lds_doubles);
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<BM, BN, BK>, 256, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  int64_t grid = (int64_t)bl.num_cus * per_cu;
  if (grid > bl.nchunks) grid = bl.nchunks;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(batch_reset_kernel, dim3((unsigned)((bl.n_cnt + 255) / 256 + 1)), dim3(256), 0, s, bl.counter,
                     bl.tile_cnt, bl.n_cnt);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((batch_kernel<BM, BN, BK>), dim3((unsigned)grid), dim3(256), lds, s, bl.items, bl.ptrs,
                     bl.tasks, bl.chunks, bl.nchunks, bl.counter, bl.parts, bl.tile_cnt);
  return hipGetLastError();
}

}  // namespace

size_t batch_lds_bytes(int config, int slab_lds_doubles) {
  int g = 0;
  switch (config) {
#define TC_BCFG(id, bm, bn, bk) \
  case id: g = gett_lds_doubles<bm, bn, bk>(); break;
    TC_BATCH_TILES(TC_BCFG)
#undef TC_BCFG
    default: g = 0;
  }
  return (size_t)(g > slab_lds_doubles ? g : slab_lds_doubles) * sizeof(double);
}

hipError_t launch_batch(const BatchLaunch& bl, hipStream_t s) {
  if (bl.ntasks == 0) return hipSuccess;
  switch (bl.config) {
#define TC_BCFG(id, bm, bn, bk) \
  case id: return launch_cfg<bm, bn, bk>(bl, s);
    TC_BATCH_TILES(TC_BCFG)
#undef TC_BCFG
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tc
