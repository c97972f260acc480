// Inner loops of the memory-bound recipes (GEMV, DOT, fused GER sums),
// shared by their own kernels and by the persistent batch kernel.
//
// A contracted group of several modes is addressed through offset tables, so
// each element costs a table lookup before its load.  Both loops look up the
// offsets of their next step while the loads of the current step are in
// flight, so a step waits on one memory latency, not two in a row.
#pragma once

#include "kernels.hpp"

namespace tc {

// Lanes along k: this lane's share of sum_k A[aK(k)] B[bK(k)] over
// k = k0 + lane, k0 + lane + 64, ... below k1.  U strided elements of each
// operand are in flight per step (U independent sums); kernels with registers
// to spare take U = 8.
template <int U = 4>
TC_DEV double lanes_k_dot(const double* __restrict__ A, const double* __restrict__ B, const Offs& aK,
                          const Offs& bK, int64_t k0, int64_t k1, int lane) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  typedef double d2 __attribute__((ext_vector_type(2)));
  const bool unit = !aK.tab && !bK.tab && aK.stride == 1 && bK.stride == 1;
  if (unit && ((reinterpret_cast<uintptr_t>(A + k0) | reinterpret_cast<uintptr_t>(B + k0)) & 15) == 0) {
    // both operands contiguous along k: 16-byte loads, lane l takes pairs
    // k0 + 2l + 128j (four pairs in flight per step)
    const d2* __restrict__ A2 = reinterpret_cast<const d2*>(A + k0);
    const d2* __restrict__ B2 = reinterpret_cast<const d2*>(B + k0);
    const int64_t pairs = (k1 - k0) >> 1;
    int64_t q = lane;
    for (; q + 192 < pairs; q += 256) {
      d2 a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = A2[q + 64 * u];
        b[u] = B2[q + 64 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += a[u].x * b[u].x + a[u].y * b[u].y;
    }
    for (; q < pairs; q += 64) {
      const d2 a = A2[q], b = B2[q];
      acc[0] += a.x * b.x + a.y * b.y;
    }
    if (((k1 - k0) & 1) && lane == 0) acc[1] += A[k1 - 1] * B[k1 - 1];
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
  double accu[U];
  int64_t oa[U], ob[U];
  int64_t k = k0 + lane;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    accu[u] = 0.0;
    const int64_t kk = k + 64 * u;
    oa[u] = kk < k1 ? off_at(aK, kk) : -1;
    ob[u] = kk < k1 ? off_at(bK, kk) : -1;
  }
  for (; k < k1; k += 64 * U) {
    double a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] = oa[u] >= 0 ? A[oa[u]] : 0.0;
      b[u] = ob[u] >= 0 ? B[ob[u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t kk = k + 64 * U + 64 * u;
      oa[u] = kk < k1 ? off_at(aK, kk) : -1;
      ob[u] = kk < k1 ? off_at(bK, kk) : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) accu[u] += a[u] * b[u];
  }
  // pairwise in a fixed order
#pragma unroll
  for (int w = U / 2; w >= 1; w /= 2)
#pragma unroll
    for (int u = 0; u < w; ++u) accu[u] += accu[u + w];
  return accu[0];
}

// One output per thread: sum_k A[aK(k)] B[bK(k)] over k in [k0, k1) in order
// of four interleaved sums (all lanes of a wavefront walk the same k).
TC_DEV double lanes_out_dot(const double* __restrict__ A, const double* __restrict__ B, const Offs& aK,
                            const Offs& bK, int64_t k0, int64_t k1) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t oa[4], ob[4];
  int64_t k = k0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    oa[u] = k + u < k1 ? off_at(aK, k + u) : -1;
    ob[u] = k + u < k1 ? off_at(bK, k + u) : -1;
  }
  for (; k < k1; k += 4) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = oa[u] >= 0 ? A[oa[u]] : 0.0;
      b[u] = ob[u] >= 0 ? B[ob[u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t kk = k + 4 + u;
      oa[u] = kk < k1 ? off_at(aK, kk) : -1;
      ob[u] = kk < k1 ? off_at(bK, kk) : -1;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += a[u] * b[u];
  }
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Branch-free forms of the generic (offset-table) loops for the persistent
// batch kernel: whether each operand goes through a table or a stride is
// decided once, outside the loop (TA, TB), and steps past the end read
// offset index k0 and are masked out of the sums instead of skipping their
// loads, so every load of a step is in flight together.  The sums are the
// same, in the same order, as in the loops above.
template <int U, bool TA, bool TB>
TC_DEV double lanes_k_steps(const double* __restrict__ A, const double* __restrict__ B, const Offs& aK,
                            const Offs& bK, int64_t k0, int64_t k1, int lane) {
  auto offa = [&](int64_t kk) { return TA ? aK.tab[kk] : kk * aK.stride; };
  auto offb = [&](int64_t kk) { return TB ? bK.tab[kk] : kk * bK.stride; };
  double accu[U];
  int64_t oa[U], ob[U];
  int64_t k = k0 + lane;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    accu[u] = 0.0;
    const int64_t kk = k + 64 * u < k1 ? k + 64 * u : k0;
    oa[u] = offa(kk);
    ob[u] = offb(kk);
  }
  for (; k < k1; k += 64 * U) {
    double a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] = A[oa[u]];
      b[u] = B[ob[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t kn = k + 64 * U + 64 * u;
      const int64_t kk = kn < k1 ? kn : k0;
      oa[u] = offa(kk);
      ob[u] = offb(kk);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) accu[u] += k + 64 * u < k1 ? a[u] * b[u] : 0.0;
  }
#pragma unroll
  for (int w = U / 2; w >= 1; w /= 2)
#pragma unroll
    for (int u = 0; u < w; ++u) accu[u] += accu[u + w];
  return accu[0];
}

template <int U>
TC_DEV double lanes_k_dot_flat(const double* __restrict__ A, const double* __restrict__ B, const Offs& aK,
                               const Offs& bK, int64_t k0, int64_t k1, int lane) {
  const bool unit = !aK.tab && !bK.tab && aK.stride == 1 && bK.stride == 1;
  if ((unit && ((reinterpret_cast<uintptr_t>(A + k0) | reinterpret_cast<uintptr_t>(B + k0)) & 15) == 0) || k0 >= k1)
    return lanes_k_dot<U>(A, B, aK, bK, k0, k1, lane);
  if (aK.tab)
    return bK.tab ? lanes_k_steps<U, true, true>(A, B, aK, bK, k0, k1, lane)
                  : lanes_k_steps<U, true, false>(A, B, aK, bK, k0, k1, lane);
  return bK.tab ? lanes_k_steps<U, false, true>(A, B, aK, bK, k0, k1, lane)
                : lanes_k_steps<U, false, false>(A, B, aK, bK, k0, k1, lane);
}

// Lanes along k over a contracted group walked in blocks of at most 64
// entries: this lane's share of the sum over blocks [j0, j1), block j adding
// A[ta[j] + la] B[tb[j] + lb] where the lane's position (lp, lq) lies inside
// the block's extents (tl[j]: bits 0-7 along p, 8-15 along q).  The block
// tables are indexed by wavefront-uniform j (scalar loads, one per 64 entries
// instead of one per entry), and the next step's entries are looked up while
// the current step's loads are in flight.
template <int U>
TC_DEV double lanes_k_blocks(const double* __restrict__ A, const double* __restrict__ B,
                             const int64_t* __restrict__ ta, const int64_t* __restrict__ tb,
                             const int64_t* __restrict__ tl, int64_t j0, int64_t j1, int64_t la, int64_t lb, int lp,
                             int lq) {
  double accu[U];
  int64_t oa[U], ob[U];
  bool ok[U];
  auto look = [&](int u, int64_t j) {
    const int64_t jj = j < j1 ? j : j0;
    const int64_t lim = tl[jj];
    ok[u] = j < j1 && lp < (int)(lim & 255) && lq < (int)((lim >> 8) & 255);
    oa[u] = ta[jj] + (ok[u] ? la : 0);
    ob[u] = tb[jj] + (ok[u] ? lb : 0);
  };
#pragma unroll
  for (int u = 0; u < U; ++u) {
    accu[u] = 0.0;
    look(u, j0 + u);
  }
  for (int64_t j = j0; j < j1; j += U) {
    double a[U], b[U];
    bool v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] = A[oa[u]];
      b[u] = B[ob[u]];
      v[u] = ok[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) look(u, j + U + u);
#pragma unroll
    for (int u = 0; u < U; ++u) accu[u] += v[u] ? a[u] * b[u] : 0.0;
  }
#pragma unroll
  for (int w = U / 2; w >= 1; w /= 2)
#pragma unroll
    for (int u = 0; u < w; ++u) accu[u] += accu[u + w];
  return accu[0];
}

template <bool TA, bool TB>
TC_DEV double lanes_out_steps(const double* __restrict__ A, const double* __restrict__ B, const Offs& aK,
                              const Offs& bK, int64_t k0, int64_t k1) {
  auto offa = [&](int64_t kk) { return TA ? aK.tab[kk] : kk * aK.stride; };
  auto offb = [&](int64_t kk) { return TB ? bK.tab[kk] : kk * bK.stride; };
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t oa[4], ob[4];
  int64_t k = k0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t kk = k + u < k1 ? k + u : k0;
    oa[u] = offa(kk);
    ob[u] = offb(kk);
  }
  for (; k < k1; k += 4) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = A[oa[u]];
      b[u] = B[ob[u]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t kk = k + 4 + u < k1 ? k + 4 + u : k0;
      oa[u] = offa(kk);
      ob[u] = offb(kk);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += k + u < k1 ? a[u] * b[u] : 0.0;
  }
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

TC_DEV double lanes_out_dot_flat(const double* __restrict__ A, const double* __restrict__ B, const Offs& aK,
                                 const Offs& bK, int64_t k0, int64_t k1) {
  if (k0 >= k1) return 0.0;
  if (aK.tab)
    return bK.tab ? lanes_out_steps<true, true>(A, B, aK, bK, k0, k1) : lanes_out_steps<true, false>(A, B, aK, bK, k0, k1);
  return bK.tab ? lanes_out_steps<false, true>(A, B, aK, bK, k0, k1) : lanes_out_steps<false, false>(A, B, aK, bK, k0, k1);
}

}  // namespace tc
