// Host planner: validation, normalisation, the paper's classification and
// the layout of index groups for the kernels.
//
// Classification follows Sec. 3.2 of the paper: with p contracted indices,
// Delta(t) = N(t) - p counts the free indices of each input; Class 1 has no
// free index in either, Class 2 in exactly one, Class 3 in both.  Class 3
// splits on the stride-1 modes (Sec. 3.2, "Class 3.1" / "Class 3.2"): when
// the two inputs' stride-1 modes are different contracted indices no slicing
// meets R1-R3 of Sec. 3.1 and GEMM needs a copy first (3.1); otherwise a
// direct GEMM exists (3.2).  Readings where the paper is silent: extent-1
// modes are dropped before classifying; batch indices (in A, B and C) are
// sliced everywhere and not counted in N(t); an input with no stride-1 mode,
// or whose stride-1 mode is a batch index, cannot meet R1 (Class 3.1); p = 0
// (an outer product) is reported as class 0.
#include "planner.hpp"

#include "kernels.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <tuple>
#include <vector>
#include <climits>
#include <cmath>
#include <initializer_list>

namespace tc {
namespace {

struct LabelInfo {
  int32_t label;
  int64_t ext;
  int pos[3];  // position in A, B, C (-1 if absent)
};

int find_label(const TensorDesc& t, int32_t l) {
  for (int i = 0; i < t.rank; ++i)
    if (t.lab[i] == l) return i;
  return -1;
}

std::string fmt(const char* f, long long a = 0, long long b = 0) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), f, a, b);
  return buf;
}

// Output entries must not alias: after sorting the modes of extent > 1 by
// stride, each stride must be positive and reach past the span of the
// previous ones.  (A sufficient test; it rejects some exotic injective layouts.)
bool output_overlaps(const TensorDesc& C) {
  std::vector<std::pair<int64_t, int64_t>> m;  // (stride, extent)
  for (int i = 0; i < C.rank; ++i) {
    if (C.ext[i] == 0) return false;  // empty: nothing is written
    if (C.ext[i] > 1) m.push_back({C.str[i], C.ext[i]});
  }
  std::sort(m.begin(), m.end());
  int64_t span = 1;  // entries covered by the modes so far
  for (auto& se : m) {
    if (se.first <= 0 || se.first < span) return true;
    span = se.first * se.second;
  }
  return false;
}

TensorDesc squeeze(const TensorDesc& t) {
  TensorDesc s;
  for (int i = 0; i < t.rank; ++i) {
    if (t.ext[i] == 1) continue;
    s.ext[s.rank] = t.ext[i];
    s.str[s.rank] = t.str[i];
    s.lab[s.rank] = t.lab[i];
    s.rank++;
  }
  return s;
}

int unit_mode(const TensorDesc& t) {
  for (int i = 0; i < t.rank; ++i)
    if (t.str[i] == 1 && t.ext[i] > 1) return i;
  return -1;
}

// Sort a group's modes by the strides of one slot (ties: the next slot's),
// so that the slot whose stride-1 mode lives in the group reads it first.
void order_group(Group& g, int key, int tie) {
  std::vector<int> idx(g.n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (g.str[key][a] != g.str[key][b]) return g.str[key][a] < g.str[key][b];
    return g.str[tie][a] < g.str[tie][b];
  });
  Group o = g;
  for (int i = 0; i < g.n; ++i) {
    o.ext[i] = g.ext[idx[i]];
    o.lab[i] = g.lab[idx[i]];
    for (int s = 0; s < 3; ++s) o.str[s][i] = g.str[s][idx[i]];
  }
  g = o;
}

// Merge neighbouring modes that every holder of the group stores
// contiguously one after the other (stride of the next = stride * extent).
void fuse_group(Group& g, const bool holders[3]) {
  if (g.n <= 1) return;
  Group o;
  o.n = 0;
  for (int i = 0; i < g.n; ++i) {
    bool merge = o.n > 0;
    if (merge) {
      for (int s = 0; s < 3; ++s)
        if (holders[s] && g.str[s][i] != o.str[s][o.n - 1] * o.ext[o.n - 1]) merge = false;
    }
    if (merge) {
      o.ext[o.n - 1] *= g.ext[i];
    } else {
      o.ext[o.n] = g.ext[i];
      o.lab[o.n] = g.lab[i];
      for (int s = 0; s < 3; ++s) o.str[s][o.n] = g.str[s][i];
      o.n++;
    }
  }
  g = o;
}

int64_t product(const TensorDesc& t) {
  int64_t p = 1;
  for (int i = 0; i < t.rank; ++i) p *= t.ext[i];
  return p;
}

// Every size the planner derives is a product of extents.  analyze() first
// checks, with overflow-checked multiplication, that each tensor's element
// count and address span and the contraction's whole iteration space stay at
// or below kMaxCount; after that the products it forms from subsets of the
// extents cannot wrap, and the byte and padded-tile sizes built on them are
// checked again where they are formed.
constexpr int64_t kMaxCount = (int64_t)1 << 56;
// Host offset tables (int64 entries, one per index of an unfused group) are
// built and uploaded at plan time: at most this many entries per plan.
constexpr int64_t kMaxTableEntries = (int64_t)1 << 31;

bool mul_capped(int64_t a, int64_t b, int64_t* r) { return !__builtin_mul_overflow(a, b, r) && *r <= kMaxCount; }

// a byte count sum of products: off += f0 * f1 * ... (false on overflow)
bool add_product(size_t* off, std::initializer_list<int64_t> f) {
  uint64_t v = 1;
  for (int64_t x : f) {
    if (x < 0 || __builtin_mul_overflow(v, (uint64_t)x, &v)) return false;
  }
  return !__builtin_add_overflow((uint64_t)*off, v, (uint64_t*)off) && *off <= ((uint64_t)1 << 62);
}

// Element count and address span of each tensor, and the iteration space
// (product of the extents of all distinct labels), within kMaxCount.
bool sizes_fit(const TensorDesc* const T[3], std::string* err) {
  const char* name[3] = {"A", "B", "C"};
  bool empty = false;
  for (int s = 0; s < 3; ++s)
    for (int i = 0; i < T[s]->rank; ++i) empty = empty || T[s]->ext[i] == 0;
  for (int s = 0; s < 3; ++s) {
    const TensorDesc& t = *T[s];
    int64_t elems = 1, span = 0;
    for (int i = 0; i < t.rank; ++i) {
      if (t.ext[i] == 0) continue;
      int64_t reach = 0;
      if (!mul_capped(t.ext[i] - 1, t.str[i], &reach) || __builtin_add_overflow(span, reach, &span) ||
          span > kMaxCount) {
        *err = std::string("address span of ") + name[s] + " exceeds 2^56 elements";
        return false;
      }
      if (!empty && !mul_capped(elems, t.ext[i], &elems)) {
        *err = std::string("element count of ") + name[s] + " exceeds 2^56";
        return false;
      }
    }
  }
  if (empty) return true;
  int64_t space = 1;
  for (int s = 0; s < 3; ++s)
    for (int i = 0; i < T[s]->rank; ++i) {
      bool seen = false;
      for (int u = 0; u < s && !seen; ++u) seen = find_label(*T[u], T[s]->lab[i]) >= 0;
      if (!seen && !mul_capped(space, T[s]->ext[i], &space)) {
        *err = "iteration space (product of all distinct extents) exceeds 2^56";
        return false;
      }
    }
  return true;
}

// Rule picker for the GEMM tile: the largest tile (most wavefronts per
// workgroup, most reuse per byte staged) that still gives each of the 256
// compute units a workgroup; smaller tiles as the problem shrinks.
int pick_tile(int64_t M, int64_t N, int64_t K, int64_t L) {
  auto tiles = [&](int bm, int bn) { return ((M + bm - 1) / bm) * ((N + bn - 1) / bn) * L; };
  if (K >= 2048) {
    // Long contracted range: 128 x 128 tiles (else 64 x 64) when they waste
    // under a quarter of their area on padding and split-K (below 128 tiles)
    // turns them into at least 256 workgroups.  Larger tiles would leave each
    // segment too few k-steps; smaller ones stage too little per byte.
    // A narrow column range beside a long row range: 128 x 32 tiles when it
    // is at most 32 wide, 128 x 64 when at most 48 (and the same transposed
    // for a narrow row range), with split-K (measured ahead of 32 x 32 and
    // 64 x 64 tiles on the coupled-cluster shapes with short indices of 30
    // and 45).
    if (N <= 32 && M >= 512 && tiles(128, 32) < 128) return 18;
    if (M <= 32 && N >= 512 && tiles(32, 128) < 128) return 19;
    if (N <= 48 && M >= 512 && tiles(128, 64) < 128) return 2;
    for (int id : {9, 1}) {
      const TileCfg& t = kTiles[id];
      const int64_t Mp = (M + t.bm - 1) / t.bm * t.bm, Np = (N + t.bn - 1) / t.bn * t.bn;
      const int64_t n = tiles(t.bm, t.bn);
      if (n >= 128 || 4 * M * N < 3 * Mp * Np) continue;
      int split;
      int64_t len;
      choose_split(n, K, t.bk, &split, &len);
      if (n * split >= 256) return id;
    }
  }
  if (tiles(256, 128) >= 256) return 11;
  if (tiles(128, 256) >= 256) return 12;
  if (tiles(128, 128) >= 256) return 9;
  if (tiles(64, 64) >= 256) return 1;
  // Fewer output tiles than the chip has compute units, over a long
  // contracted range: split-K makes up the workgroup count, but only below
  // 128 tiles, so take a tile size that lands there (32 x 32 tiles at 128 or
  // more would run one long k loop per tile on too few workgroups).
  if (K >= 2048 && tiles(32, 32) >= 128) return tiles(64, 64) >= 128 ? 9 : 1;
  return 8;
}

// A batch-dominated contraction: at least 64 batch indices and per-point
// slabs of A, B and C small enough for several points per workgroup.
bool batched_fits(const tc_plan_info& info, const Group* G) {
  if (G[GL].n == 0 || info.L < 64) return false;
  if (info.M > 1024 || info.N > 1024 || info.K > 1024) return false;
  const int64_t per = info.M * info.K + info.N * info.K + info.M * info.N;
  return per * 2 + info.K <= kBatchedLdsDoubles;
}

// Slab descriptors: each operand's non-batch modes sorted by global stride,
// with strides into the canonical LDS slab ([m][k] for A, [n][k] for B,
// [m][n] for C; the group's own mode order decodes column-major).
void build_slabs(Analysis& an) {
  const Group* G = an.g;
  const int64_t M = an.info.M, N = an.info.N, K = an.info.K;
  struct Use {
    int group;
    int64_t lweight;  // LDS stride of the group's linear index
  };
  const Use uses[3][2] = {{{GM, K}, {GK, 1}}, {{GN, K}, {GK, 1}}, {{GM, N}, {GN, 1}}};
  for (int slot = 0; slot < 3; ++slot) {
    std::vector<std::tuple<int64_t, int, int>> modes;  // (gstride, ext, lstride)
    for (const Use& u : uses[slot]) {
      const Group& g = G[u.group];
      int64_t w = u.lweight;
      for (int i = 0; i < g.n; ++i) {
        modes.emplace_back(g.str[slot][i], (int)g.ext[i], (int)w);
        w *= g.ext[i];
      }
    }
    std::sort(modes.begin(), modes.end());
    an.slab_n[slot] = (int)modes.size();
    int size = 1;
    for (size_t i = 0; i < modes.size(); ++i) {
      an.slab_gstr[slot][i] = std::get<0>(modes[i]);
      an.slab_ext[slot][i] = std::get<1>(modes[i]);
      an.slab_lstr[slot][i] = std::get<2>(modes[i]);
      size *= std::get<1>(modes[i]);
    }
    an.slab_size[slot] = size;
    const int64_t min_slab = modes.empty() ? INT64_MAX : std::get<0>(modes[0]);
    an.slab_batch_fast[slot] = G[GL].n > 0 && G[GL].str[slot][0] < min_slab ? 1 : 0;
    // dense: each mode's stride is the previous one times its extent, so the
    // slab is one strided run in storage order
    bool dense = !modes.empty() && std::get<0>(modes[0]) > 0;
    for (size_t i = 1; dense && i < modes.size(); ++i)
      dense = std::get<0>(modes[i]) == std::get<0>(modes[i - 1]) * std::get<1>(modes[i - 1]);
    an.slab_dense[slot] = dense ? 1 : 0;
    an.slab_s0[slot] = dense ? std::get<0>(modes[0]) : 0;
  }
  const int per = an.slab_size[0] + an.slab_size[1] + an.slab_size[2];
  an.batched_P = slab_points(per, (int)K, kBatchedSlabLdsDoubles);
  (void)M;
  (void)N;
}

}  // namespace

void picker_features(const Analysis& an, const TensorDesc& A, const TensorDesc& B, const TensorDesc& C, float* f) {
  const tc_plan_info& in = an.info;
  const Group* G = an.g;
  auto lg = [](double x) { return (float)std::log2(x < 1.0 ? 1.0 : x); };
  for (int i = 0; i < TC_PICKER_FEATURES; ++i) f[i] = 0.f;
  const double M = (double)in.M, N = (double)in.N, K = (double)in.K, L = (double)in.L;
  f[0] = lg(M);
  f[1] = lg(N);
  f[2] = lg(K);
  f[3] = lg(L);
  f[4] = (float)in.nM;
  f[5] = (float)in.nN;
  f[6] = (float)in.nK;
  f[7] = (float)in.nL;
  f[8] = (float)A.rank;
  f[9] = (float)B.rank;
  f[10] = (float)C.rank;
  const int cls[5] = {0, 1, 2, 31, 32};
  for (int i = 0; i < 5; ++i) f[11 + i] = in.paper_class == cls[i] ? 1.f : 0.f;
  f[16] = an.a_mfast ? 1.f : 0.f;
  f[17] = an.a_kfast ? 1.f : 0.f;
  f[18] = an.b_nfast ? 1.f : 0.f;
  f[19] = an.b_kfast ? 1.f : 0.f;
  f[20] = G[GN].n > 0 && G[GN].str[SC][0] == 1 ? 1.f : 0.f;
  f[21] = (float)in.swapped;
  f[22] = G[GM].n > 0 ? lg((double)G[GM].ext[0]) : 0.f;
  f[23] = G[GN].n > 0 ? lg((double)G[GN].ext[0]) : 0.f;
  f[24] = G[GK].n > 0 ? lg((double)G[GK].ext[0]) : 0.f;
  f[25] = lg((double)an.elems[SA]);
  f[26] = lg((double)an.elems[SB]);
  f[27] = lg((double)an.elems[SC]);
  f[28] = lg(in.flops);
  f[29] = lg(in.bytes);
  f[30] = in.bytes > 0 ? (float)std::log2(std::max(1e-3, in.flops / in.bytes)) : 0.f;
  f[31] = lg(std::min(M, N));
}

int candidate_of(const Analysis& an) {
  for (int c = 0; c < TC_PICKER_CANDIDATES - 1; ++c) {
    if (kCandidates[c].recipe != an.info.recipe) continue;
    if (an.kernel == Analysis::KERNEL_BATCHED || an.kernel == Analysis::KERNEL_SPLIT) return -1;
    if (kCandidates[c].tile < 0 || kCandidates[c].tile == an.info.tile_id) return c;
  }
  return -1;
}

int paper_class(const TensorDesc& A, const TensorDesc& B, const TensorDesc& C, int unitA, int unitB) {
  int p = 0, batchA = 0, batchB = 0;
  auto is_batch = [&](int32_t l) { return find_label(A, l) >= 0 && find_label(B, l) >= 0 && find_label(C, l) >= 0; };
  for (int i = 0; i < A.rank; ++i) {
    if (is_batch(A.lab[i])) {
      batchA++;
    } else if (find_label(B, A.lab[i]) >= 0) {
      p++;
    }
  }
  for (int i = 0; i < B.rank; ++i)
    if (is_batch(B.lab[i])) batchB++;
  int dA = A.rank - batchA - p, dB = B.rank - batchB - p;
  if (p == 0) return 0;
  if (dA == 0 && dB == 0) return 1;
  if (dA == 0 || dB == 0) return 2;
  if (unitA < 0 || unitB < 0) return 31;
  int32_t ua = A.lab[unitA], ub = B.lab[unitB];
  if (is_batch(ua) || is_batch(ub)) return 31;
  bool ua_con = find_label(B, ua) >= 0;
  bool ub_con = find_label(A, ub) >= 0;
  if (ua != ub && ua_con && ub_con) return 31;
  return 32;
}

tc_status analyze(const TensorDesc& A0, const TensorDesc& B0, const TensorDesc& C0, const tc_options& opt,
                  Analysis* out, std::string* err, bool allow_copy) {
  Analysis an;
  const TensorDesc* T[3] = {&A0, &B0, &C0};
  const char* name[3] = {"A", "B", "C"};
  for (int s = 0; s < 3; ++s) {
    const TensorDesc& t = *T[s];
    if (t.rank < 0 || t.rank > TC_MAX_RANK) {
      *err = std::string("rank of ") + name[s] + fmt(" is %lld (allowed 0..%lld)", t.rank, TC_MAX_RANK);
      return TC_ERR_RANK;
    }
    for (int i = 0; i < t.rank; ++i) {
      if (t.ext[i] < 0) {
        *err = std::string("negative extent in ") + name[s] + fmt(" mode %lld", i);
        return TC_ERR_INVALID_ARG;
      }
      if (t.str[i] < 0) {
        *err = std::string("negative stride in ") + name[s] + fmt(" mode %lld", i);
        return TC_ERR_INVALID_ARG;
      }
      for (int j = 0; j < i; ++j)
        if (t.lab[j] == t.lab[i]) {
          *err = std::string("label repeated within ") + name[s] + fmt(" (label %lld)", t.lab[i]);
          return TC_ERR_LABEL;
        }
    }
  }
  if (opt.precision < TC_PREC_F64 || opt.precision > TC_PREC_F64_CRT_INT8 || opt.recipe < TC_RECIPE_AUTO ||
      opt.recipe > TC_RECIPE_DOT || opt.tile_id < -1 || opt.tile_id >= kNumTiles || opt.split_slices < 0 ||
      opt.copy_tile < -1 || opt.copy_tile >= kDmaShapes) {
    *err = "invalid tc_options field";
    return TC_ERR_INVALID_ARG;
  }
  // Every label: in A and B (contracted), A and C, B and C, or all three.
  for (int s = 0; s < 3; ++s) {
    const TensorDesc& t = *T[s];
    for (int i = 0; i < t.rank; ++i) {
      int in = 0;
      for (int u = 0; u < 3; ++u) {
        int j = find_label(*T[u], t.lab[i]);
        if (j >= 0) {
          in++;
          if (T[u]->ext[j] != t.ext[i]) {
            *err = fmt("label %lld has extents %lld", t.lab[i], t.ext[i]) + fmt(" and %lld", T[u]->ext[j]);
            return TC_ERR_EXTENT_MISMATCH;
          }
        }
      }
      if (in < 2) {
        *err = fmt("label %lld appears only in ", t.lab[i]) + name[s] +
               " (a contraction sums an index shared by both inputs)";
        return TC_ERR_LABEL;
      }
    }
  }
  if (!sizes_fit(T, err)) return TC_ERR_INVALID_ARG;
  if (output_overlaps(C0)) {
    *err = "output strides overlap (two entries of C would share an address)";
    return TC_ERR_OUTPUT_OVERLAP;
  }

  tc_plan_info& info = an.info;
  info.precision = opt.precision;
  info.split_slices = opt.split_slices;
  info.copy_operand = -1;
  info.tile_id = -1;
  info.k_split = 1;
  info.picked_candidate = -1;
  info.split_bits = 0;
  info.copy_fed = 0;
  info.unit_a = unit_mode(A0);
  info.unit_b = unit_mode(B0);
  info.unit_c = unit_mode(C0);

  for (int i = 0; i < C0.rank; ++i)
    if (C0.ext[i] == 0) an.empty_out = true;
  for (int i = 0; i < A0.rank; ++i)
    if (A0.ext[i] == 0 && find_label(B0, A0.lab[i]) >= 0 && find_label(C0, A0.lab[i]) < 0) an.empty_sum = true;

  TensorDesc A = squeeze(A0), B = squeeze(B0), C = squeeze(C0);
  int ua = unit_mode(A), ub = unit_mode(B);
  info.paper_class = paper_class(A, B, C, ua, ub);

  tc_recipe recipe = opt.recipe;
  if (recipe == TC_RECIPE_AUTO) {
    switch (info.paper_class) {
      case 32: recipe = TC_RECIPE_GEMM; break;
      case 31: recipe = TC_RECIPE_COPY_GEMM; break;
      case 2: recipe = TC_RECIPE_GEMV; break;
      case 1: recipe = TC_RECIPE_DOT; break;
      default: recipe = TC_RECIPE_GER; break;
    }
  }
  info.recipe = recipe;

  // The kernels write C along their column index with consecutive lanes, so
  // C's stride-1 mode belongs in the column group: exchange the inputs when
  // it is a free index of A (the result does not depend on the operand
  // order, Sec. 2.3 footnote).
  int uc = unit_mode(C);
  bool swap = false;
  if (uc >= 0) {
    int32_t l = C.lab[uc];
    swap = find_label(A, l) >= 0 && find_label(B, l) < 0;
  }
  info.swapped = swap ? 1 : 0;
  const TensorDesc& KA = swap ? B : A;
  const TensorDesc& KB = swap ? A : B;
  an.elems[SA] = product(KA);
  an.elems[SB] = product(KB);
  an.elems[SC] = product(C);

  // Distribute the modes over the four groups.
  Group* G = an.g;
  for (int gi = 0; gi < 4; ++gi) G[gi] = Group();
  auto add = [&](int gi, int32_t lab, int64_t ext, int64_t sa, int64_t sb, int64_t sc) {
    Group& g = G[gi];
    g.lab[g.n] = lab;
    g.ext[g.n] = ext;
    g.str[SA][g.n] = sa;
    g.str[SB][g.n] = sb;
    g.str[SC][g.n] = sc;
    g.n++;
  };
  for (int i = 0; i < KA.rank; ++i) {
    int jb = find_label(KB, KA.lab[i]), jc = find_label(C, KA.lab[i]);
    if (jb >= 0 && jc >= 0)
      add(GL, KA.lab[i], KA.ext[i], KA.str[i], KB.str[jb], C.str[jc]);
    else if (jb >= 0)
      add(GK, KA.lab[i], KA.ext[i], KA.str[i], KB.str[jb], 0);
    else
      add(GM, KA.lab[i], KA.ext[i], KA.str[i], 0, C.str[jc]);
  }
  for (int i = 0; i < KB.rank; ++i) {
    if (find_label(KA, KB.lab[i]) >= 0) continue;
    int jc = find_label(C, KB.lab[i]);
    add(GN, KB.lab[i], KB.ext[i], 0, KB.str[i], C.str[jc]);
  }

  auto unit_in = [&](const Group& g, int slot) {
    for (int i = 0; i < g.n; ++i)
      if (g.str[slot][i] == 1) return true;
    return false;
  };

  // COPY_GEMM: copy the input with fewer entries (ties: kernel B) into a
  // packed layout [its free group, contracted group, batch group].
  // (Split precision gathers both inputs into digit planes: no copy there.)
  if (recipe == TC_RECIPE_COPY_GEMM && opt.precision == TC_PREC_F64)
    an.copy_slot = an.elems[SA] < an.elems[SB] ? SA : SB;
  // The inner-product recipes (DOT, and GEMV along k) read both inputs along
  // the contracted index with consecutive lanes.  When the two stride-1 modes
  // are different contracted indices (the situation of Class 3.1, failure
  // F1), one input could only be read with strided lanes, so -- as for
  // COPY+GEMM -- the smaller input is first copied into the other's
  // contracted order.
  if (allow_copy && opt.precision == TC_PREC_F64 && (recipe == TC_RECIPE_DOT || recipe == TC_RECIPE_GEMV) &&
      !an.empty_out && !an.empty_sum) {
    const int kua = unit_mode(KA), kub = unit_mode(KB);
    auto contracted = [&](int32_t l) { return find_label(KA, l) >= 0 && find_label(KB, l) >= 0 && find_label(C, l) < 0; };
    if (kua >= 0 && kub >= 0 && KA.lab[kua] != KB.lab[kub] && contracted(KA.lab[kua]) && contracted(KB.lab[kub]))
      an.copy_slot = an.elems[SA] < an.elems[SB] ? SA : SB;
  }
  info.copy_operand = an.copy_slot < 0 ? -1 : ((an.copy_slot == SA) != swap ? 0 : 1);

  order_group(G[GM], SA, SC);
  if (unit_in(G[GN], SB))
    order_group(G[GN], SB, SC);
  else
    order_group(G[GN], SC, SB);
  {
    int key = SA;
    bool a_unit = unit_in(G[GK], SA) && an.copy_slot != SA;
    bool b_unit = unit_in(G[GK], SB) && an.copy_slot != SB;
    if (!a_unit && b_unit) key = SB;
    if (a_unit && b_unit && an.elems[SB] > an.elems[SA]) key = SB;  // the larger operand reads contiguously
    if (an.copy_slot == SA) key = SB;
    order_group(G[GK], key, key == SA ? SB : SA);
  }
  order_group(G[GL], SC, SA);

  if (an.copy_slot >= 0) {
    int cs = an.copy_slot;
    int free_g = cs == SA ? GM : GN;
    const TensorDesc& X = cs == SA ? KA : KB;
    // packed strides per label in group order
    int64_t stride = 1;
    int32_t labs[TC_MAX_RANK];
    int64_t dst[TC_MAX_RANK];
    int nl = 0;
    for (int gi : {free_g, (int)GK, (int)GL}) {
      Group& g = G[gi];
      for (int i = 0; i < g.n; ++i) {
        g.str[cs][i] = stride;
        labs[nl] = g.lab[i];
        dst[nl] = stride;
        nl++;
        stride *= g.ext[i];
      }
    }
    an.copy_rank = X.rank;
    for (int i = 0; i < X.rank; ++i) {
      an.copy_ext[i] = X.ext[i];
      an.copy_src_str[i] = X.str[i];
      an.copy_dst_str[i] = 0;
      for (int q = 0; q < nl; ++q)
        if (labs[q] == X.lab[i]) an.copy_dst_str[i] = dst[q];
    }
    info.workspace_bytes = (size_t)an.elems[cs] * sizeof(double);
  }

  const bool hold[4][3] = {{true, false, true}, {false, true, true}, {true, true, false}, {true, true, true}};
  for (int gi = 0; gi < 4; ++gi) fuse_group(G[gi], hold[gi]);

  bool a_mfast = G[GM].n > 0 && G[GM].str[SA][0] == 1;
  bool b_nfast = G[GN].n > 0 && G[GN].str[SB][0] == 1;
  an.a_kfast = !a_mfast && G[GK].n > 0 && G[GK].str[SA][0] == 1;
  an.b_kfast = !b_nfast && G[GK].n > 0 && G[GK].str[SB][0] == 1;
  an.a_mfast = a_mfast;
  an.b_nfast = b_nfast;
  {
    // 16-byte pairs along each operand's stride-1 mode (see Analysis::dma_ok)
    auto pairs = [&](int slot, int rowg, bool rowfast, bool kfast) {
      if (!rowfast && !kfast) return false;
      const int lead = rowfast ? rowg : GK;
      if (G[lead].ext[0] % 2 != 0) return false;
      for (int g : {rowg, (int)GK, (int)GL})
        for (int i = 0; i < G[g].n; ++i)
          if (!(g == lead && i == 0) && G[g].str[slot][i] % 2 != 0) return false;
      return true;
    };
    an.dma_ok = G[GK].n >= 1 && G[GK].n <= kDmaMaxKModes && G[GK].size() <= 0x7fffffffLL &&
                pairs(SA, GM, a_mfast, an.a_kfast) && pairs(SB, GN, b_nfast, an.b_kfast);
  }

  {
    // offset tables: one per (group of two or more modes, tensor holding it)
    int64_t entries = 0;
    const int holders[4] = {2, 2, 2, 3};
    for (int gi = 0; gi < 4; ++gi)
      if (G[gi].n > 1 && !an.empty_out) entries += holders[gi] * G[gi].size();
    if (entries > kMaxTableEntries) {
      *err = fmt("index groups that do not fuse need %lld offset-table entries (at most %lld)", entries,
                 kMaxTableEntries);
      return TC_ERR_UNSUPPORTED;
    }
  }
  info.M = G[GM].size();
  info.N = G[GN].size();
  info.K = G[GK].size();
  info.L = G[GL].size();
  if (an.empty_out) info.M = info.N = info.L = 0;
  info.nM = G[GM].n;
  info.nN = G[GN].n;
  info.nK = G[GK].n;
  info.nL = G[GL].n;
  info.flops = 2.0 * (double)info.M * (double)info.N * (double)info.K * (double)info.L;
  info.bytes = 8.0 * ((double)product(A0) + (double)product(B0) + (double)product(C0));
  if (opt.precision != TC_PREC_F64) {
    // Split precision: every recipe runs as digit planes (gathered through the
    // strides once) multiplied on the BF16 / FP8 matrix cores.
    const bool fp8 = opt.precision == TC_PREC_F64_SPLIT_FP8;
    const bool crt = opt.precision == TC_PREC_F64_CRT_INT8;
    const int maxs = crt ? kCrtMaxModuli : (fp8 ? kSplitMaxFp8 : kSplitMaxBf16);
    int S = opt.split_slices > 0 ? opt.split_slices
                                 : (crt ? crt_default_moduli(info.K) : (fp8 ? kSplitDefaultFp8 : kSplitDefaultBf16));
    if (S > maxs || (crt && S < 2)) {
      *err = fmt("split_slices %lld is outside the range %lld to ", S, crt ? 2 : 1) +
             fmt("%lld for this digit type", maxs);
      return TC_ERR_INVALID_ARG;
    }
    if (info.L > 1) {
      *err = "split precision does not take batch indices (labels in A, B and C)";
      return TC_ERR_UNSUPPORTED;
    }
    info.recipe = TC_RECIPE_GEMM;
    an.kernel = Analysis::KERNEL_SPLIT;
    info.split_slices = S;
    an.slices = S;
    if (crt) {
      if (opt.tile_id >= kCrtNumTiles) {
        *err = fmt("tile_id %lld is not a residue GEMM configuration (0 to %lld)", opt.tile_id, kCrtNumTiles - 1);
        return TC_ERR_INVALID_ARG;
      }
      info.tile_id = opt.tile_id >= 0 ? opt.tile_id : kCrtDefaultTile;
      an.crt_bits = crt_bits(S, info.K);
      if (an.crt_bits < 1) {
        *err = fmt("%lld moduli cannot hold sums of %lld products; use more moduli", S, info.K);
        return TC_ERR_UNSUPPORTED;
      }
      info.split_bits = an.crt_bits;
      an.crt_c_nfast = G[GN].n > 0 && G[GN].str[SC][0] == 1;
    } else {
      info.split_bits = fp8 ? 4 + 5 * (S - 1) : 8 + 9 * (S - 1);
    }
    const SplitTile t = crt ? SplitTile{kCrtTiles[info.tile_id].bm, kCrtTiles[info.tile_id].bn, kCrtBK}
                            : split_tile(fp8, S);
    auto up = [](int64_t v, int64_t m) { return v <= 0 ? m : (v + m - 1) / m * m; };
    an.Mp = up(info.M, t.bm);
    an.Np = up(info.N, t.bn);
    an.Kp = up(info.K, fp8 ? 128 : t.bk);
    const int64_t esz = fp8 || crt ? 1 : 2;
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    // scratch of the row-maximum pass, used by each input in turn
    const int64_t needA = row_max_segments(info.M, info.K) * info.M;
    const int64_t needB = row_max_segments(info.N, info.K) * info.N;
    size_t off = 0;
    bool ok = true;
    an.planesA_off = off;
    ok = ok && add_product(&off, {S, an.Mp, an.Kp, esz});
    an.planesB_off = off = al(off);
    ok = ok && add_product(&off, {S, an.Np, an.Kp, esz});
    an.zres_off = off = al(off);
    if (crt) ok = ok && add_product(&off, {S, an.Mp, an.Np});
    an.sigA_off = off = al(off);
    ok = ok && add_product(&off, {an.Mp, (int64_t)sizeof(double)});
    an.sigB_off = off = al(off);
    ok = ok && add_product(&off, {an.Np, (int64_t)sizeof(double)});
    an.part_off = off = al(off);
    ok = ok && add_product(&off, {needA > needB ? needA : needB, (int64_t)sizeof(double)});
    if (!ok) {
      *err = "split-precision workspace size overflows";
      return TC_ERR_INVALID_ARG;
    }
    info.workspace_bytes = al(off);
  } else if (opt.recipe == TC_RECIPE_AUTO && batched_fits(info, G)) {
    // Many tiny contractions sharing one layout (the batch group dominates):
    // per-point slabs through LDS, all batch indices in one launch.
    an.kernel = Analysis::KERNEL_BATCHED;
    build_slabs(an);
  } else if (recipe == TC_RECIPE_GEMM || recipe == TC_RECIPE_COPY_GEMM) {
    info.tile_id = opt.tile_id >= 0 ? opt.tile_id : pick_tile(info.M, info.N, info.K, info.L);
    // few output tiles over a long contracted range: cut the range into
    // segments so that more workgroups share the work (split-K)
    const TileCfg& t = kTiles[info.tile_id];
    const int64_t tiles = ((info.M + t.bm - 1) / t.bm) * ((info.N + t.bn - 1) / t.bn) * info.L;
    int split = 1;
    int64_t len = info.K;
    if (!an.empty_out && !an.empty_sum) choose_split(tiles, info.K, t.bk, &split, &len);
    info.k_split = split;
    an.seg_len = len;
    if (split > 1) {
      an.part_offset = (info.workspace_bytes + 255) / 256 * 256;
      size_t ws = an.part_offset;
      if (!add_product(&ws, {tiles, split, t.bm, t.bn, (int64_t)sizeof(double)})) {
        *err = "split-K workspace size overflows";
        return TC_ERR_INVALID_ARG;
      }
      info.workspace_bytes = ws;
    }
    // the copy-fed kernel stands in for the large tiles (also after the copy
    // of COPY+GEMM, whose packed operand qualifies like any other); its
    // output tile follows the tile asked for, else the round rule
    an.dma_ok = an.dma_ok && (recipe == TC_RECIPE_GEMM || recipe == TC_RECIPE_COPY_GEMM) && split == 1 &&
                (info.tile_id == kDmaTile || info.tile_id == kDmaTileWide);
    if (an.dma_ok)
      an.dma_shape = opt.copy_tile >= 0 ? opt.copy_tile
                     : opt.tile_id < 0  ? dma_shape(info.M, info.N, info.L)
                                        : (info.tile_id == kDmaTile ? kDma256x128 : kDma128x256);
    info.copy_fed = an.dma_ok ? 1 + an.dma_shape : 0;
  } else {
    // Memory-bound recipes (Sec. 3.2, Classes 1 and 2, and the GER slicing).
    // GER sums its rank-1 updates in registers, one thread per output entry.
    // GEMV walks the matrix along whichever index is stride-1: its free index
    // (one thread per output) or its contracted index (lanes along k, with a
    // cross-lane sum).  DOT always puts the lanes along k.
    bool c_nfast = G[GN].n > 0 && G[GN].str[SC][0] == 1;
    an.n_fastest = b_nfast || (c_nfast && !a_mfast);
    const int64_t outputs = info.M * info.N * info.L;
    bool lanes_k;
    if (recipe == TC_RECIPE_GER) {
      lanes_k = false;
    } else if (recipe == TC_RECIPE_DOT) {
      lanes_k = true;
    } else {
      // the matrix operand is the one with more entries
      const bool a_is_matrix = an.elems[SA] >= an.elems[SB];
      const bool matrix_kfast = a_is_matrix ? an.a_kfast : an.b_kfast;
      lanes_k = matrix_kfast || (outputs < 4096 && info.K > 4096);
    }
    an.kernel = lanes_k ? Analysis::KERNEL_LANES_K : Analysis::KERNEL_LANES_OUT;
    if (!an.empty_out && !an.empty_sum) {
      an.seg = lanes_k ? k_segments(outputs, info.K) : out_segments(outputs, info.K);
      if (an.seg > 1) {
        an.part_offset = (info.workspace_bytes + 255) / 256 * 256;
        size_t ws = an.part_offset;
        if (!add_product(&ws, {outputs, an.seg, (int64_t)sizeof(double)})) {
          *err = "partial-sum workspace size overflows";
          return TC_ERR_INVALID_ARG;
        }
        info.workspace_bytes = ws;
      }
    }
  }
  info.kernel = an.kernel;
  *out = an;
  return TC_OK;
}

// Layout advice (Sec. 3.3 and the closing remarks of Sec. 5): when the inputs
// can be generated in any storage order and both have a free index, storing a
// free index at stride 1 puts the contraction in Class 3.2, so GEMM applies
// without a copy.  The suggestion stores A as [free-A, contracted, batch], B
// as [contracted, free-B, batch] and C as [free-A, free-B, batch]: the
// column-major GEMM C(M,N) = A(M,K) B(K,N) per batch index.  Each index group
// keeps one order in every tensor that holds it (taken from a fixed tensor
// when there is one), so each group fuses into a single mode.  When A is
// fixed with a contracted (or batch) index at stride 1, B leads with its free
// indices instead, which keeps the class at 3.2 when B has a free index.
tc_status suggest_layout(const TensorDesc& A, const TensorDesc& B, const TensorDesc& C, int fixed,
                         int* order[3], TensorDesc out_desc[3], Analysis* out, std::string* err) {
  tc_options o;
  tc_options_default(&o);
  Analysis an;
  tc_status s = analyze(A, B, C, o, &an, err);
  if (s != TC_OK) return s;
  const TensorDesc* T[3] = {&A, &B, &C};
  // storage order of a tensor: its modes by ascending stride (ties: position)
  auto storage = [](const TensorDesc& t) {
    std::vector<int> idx(t.rank);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return t.str[a] < t.str[b]; });
    return idx;
  };
  // the order a group's labels take from tensor t: its storage order when
  // fixed, its listing order otherwise
  auto source = [&](int t) {
    if (fixed & (1 << t)) return storage(*T[t]);
    std::vector<int> idx(T[t]->rank);
    std::iota(idx.begin(), idx.end(), 0);
    return idx;
  };
  // role of a label: 0 free-A, 1 free-B, 2 contracted, 3 batch
  auto role = [&](int32_t l) {
    const bool a = find_label(A, l) >= 0, b = find_label(B, l) >= 0, c = find_label(C, l) >= 0;
    return a && b && c ? 3 : a && b ? 2 : a ? 0 : 1;
  };
  // group labels in the order of the first fixed tensor that holds the group
  // (by preference), else of the first preferred tensor that holds it
  const int prefs[4][3] = {{0, 2, -1}, {1, 2, -1}, {0, 1, -1}, {2, 0, 1}};
  std::vector<int32_t> group[4];
  for (int g = 0; g < 4; ++g) {
    int src = -1;
    for (int pass = 0; pass < 2 && src < 0; ++pass)
      for (int q = 0; q < 3 && src < 0; ++q) {
        const int t = prefs[g][q];
        if (t < 0 || (pass == 0 && !(fixed & (1 << t)))) continue;
        src = t;
      }
    for (int i : source(src))
      if (role(T[src]->lab[i]) == g) group[g].push_back(T[src]->lab[i]);
  }
  // A fixed with a contracted or batch index at stride 1: B leads with free-B
  bool b_free_first = false;
  if (fixed & 1) {
    const int ua = unit_mode(squeeze(A));
    const TensorDesc sa = squeeze(A);
    b_free_first = ua >= 0 && role(sa.lab[ua]) >= 2;
  }
  const int seq[3][3] = {{0, 2, 3}, {b_free_first ? 1 : 2, b_free_first ? 2 : 1, 3}, {0, 1, 3}};
  for (int t = 0; t < 3; ++t) {
    const TensorDesc& x = *T[t];
    TensorDesc& d = out_desc[t];
    d = x;
    std::vector<int> ord;
    if (fixed & (1 << t)) {
      ord = storage(x);
    } else {
      for (int g : seq[t])
        for (int32_t l : group[g]) {
          const int i = find_label(x, l);
          if (i >= 0) ord.push_back(i);
        }
      int64_t stride = 1;
      for (int i : ord) {
        d.str[i] = stride;
        stride *= x.ext[i] > 0 ? x.ext[i] : 1;
      }
    }
    for (int j = 0; j < x.rank; ++j) order[t][j] = ord[j];
  }
  return analyze(out_desc[0], out_desc[1], out_desc[2], o, out, err);
}

}  // namespace tc
