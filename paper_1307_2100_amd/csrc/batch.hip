// Persistent batch kernel: many independent contractions of any shapes in one
// launch.
//
// The host turns every contraction of the batch into tasks -- GEMM tiles for
// contractions run by the FP64 MFMA tile engine, groups of batch indices for
// batch-dominated ones run by the slab engine -- and orders all tasks by
// estimated cost, largest first (longest-processing-time order).  The grid is
// sized to the number of workgroups the chip holds at once; each workgroup
// repeatedly takes the next task index from a global counter (atomic add)
// and runs it, until the counter passes the task count.  Every workgroup
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
                                                    const BatchTask* __restrict__ tasks, int64_t ntasks,
                                                    unsigned long long* counter) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  __shared__ int64_t next;
  for (;;) {
    __syncthreads();  // the previous task is done with LDS and with `next`
    if (threadIdx.x == 0) next = (int64_t)atomicAdd(counter, 1ull);
    __syncthreads();
    const int64_t t = next;
    if (t >= ntasks) break;
    const BatchTask task = tasks[t];
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
      switch (it.akf * 2 + it.bkf) {
        case 0: gett_tile<BM, BN, BK, 2, 2, false, false>(p, m0, n0, l, smem); break;
        case 1: gett_tile<BM, BN, BK, 2, 2, false, true>(p, m0, n0, l, smem); break;
        case 2: gett_tile<BM, BN, BK, 2, 2, true, false>(p, m0, n0, l, smem); break;
        default: gett_tile<BM, BN, BK, 2, 2, true, true>(p, m0, n0, l, smem); break;
      }
    } else {
      batched_slab(it.b, it.swapped ? pt.B : pt.A, it.swapped ? pt.A : pt.B, pt.C, pt.alpha, pt.beta,
                   task.idx * it.b.P, smem);
    }
  }
}

__global__ void batch_reset_kernel(unsigned long long* counter) { *counter = 0ull; }

template <int BM, int BN, int BK>
hipError_t launch_cfg(const BatchLaunch& bl, hipStream_t s) {
  const size_t lds = batch_lds_bytes(bl.config, bl.slab_lds_doubles);
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<BM, BN, BK>, 256, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  int64_t grid = (int64_t)bl.num_cus * per_cu;
  if (grid > bl.ntasks) grid = bl.ntasks;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, s, bl.counter);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((batch_kernel<BM, BN, BK>), dim3((unsigned)grid), dim3(256), lds, s, bl.items, bl.ptrs,
                     bl.tasks, bl.ntasks, bl.counter);
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
