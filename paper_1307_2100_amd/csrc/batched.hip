// Batch-dominated contractions: many independent tiny contractions that
// share one layout, such as the per-grid-point tensor algebra of the paper's
// general-relativity example (Sec. 4.2: contracted extent 4 on a lattice).
//
// A workgroup takes P consecutive batch indices.  For each operand it copies
// the P per-point slabs into LDS, walking each slab in the operand's own
// storage order so that consecutive lanes read consecutive addresses (whether
// the batch index is the slowest mode, "array of structures", or the fastest,
// "structure of arrays").  A slab that is dense in its storage order is copied
// as it is stored -- when consecutive points' slabs also follow each other the
// copy is a plain stream -- and the compute reads it through small tables of
// per-index LDS offsets; other slabs are decoded mode by mode into a canonical
// order ([p][m][k] for A, [p][n][k] for B, [p][m][n] for C).  Each thread then
// computes whole output entries from LDS, and C is written back in its
// storage order.
#include "batched_slab.hpp"

namespace tc {
namespace {

__global__ __launch_bounds__(256) void batched_small_kernel(BatchedParams bp) {
  extern __shared__ double smem[];
  batched_slab(bp, bp.A, bp.B, bp.C, bp.alpha, bp.beta, (int64_t)blockIdx.x * bp.P, smem);
}

}  // namespace

hipError_t launch_batched_small(const BatchedParams& bp, hipStream_t s) {
  if (bp.L == 0) return hipSuccess;
  const int64_t blocks = (bp.L + bp.P - 1) / bp.P;
  if (blocks > 0xffffffffLL / 256) return hipErrorInvalidConfiguration;  // total threads below 2^32
  const size_t lds = (size_t)bp.P * (bp.a.size + bp.b.size + bp.c.size) * sizeof(double) + 2 * sizeof(int) * bp.K;
  hipLaunchKernelGGL(batched_small_kernel, dim3((unsigned)blocks), dim3(256), lds, s, bp);
  return hipGetLastError();
}

}  // namespace tc
