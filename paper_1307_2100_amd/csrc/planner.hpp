// Host-side planner: validation, normalisation, the paper's classification
// and the index-group layout the kernels consume.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tc.h"

namespace tc {

// One tensor as given by the caller (extents, element strides, labels).
struct TensorDesc {
  int rank = 0;
  int64_t ext[TC_MAX_RANK] = {};
  int64_t str[TC_MAX_RANK] = {};
  int32_t lab[TC_MAX_RANK] = {};
};

// Operand slots inside a group: the two inputs in kernel roles and the output.
enum Slot { SA = 0, SB = 1, SC = 2 };

// Index groups: free indices of the kernel's A (rows), free indices of the
// kernel's B (columns), contracted indices, batch indices.
enum GroupId { GM = 0, GN = 1, GK = 2, GL = 3 };

// An ordered list of modes sharing one role.  The group's linear index g
// decodes column-major over the modes (mode 0 fastest); each operand holding
// the group has the stride of every mode (0 where it lacks the mode).
struct Group {
  int n = 0;
  int64_t ext[TC_MAX_RANK] = {};
  int64_t str[3][TC_MAX_RANK] = {};
  int32_t lab[TC_MAX_RANK] = {};
  int64_t size() const {
    int64_t s = 1;
    for (int i = 0; i < n; ++i) s *= ext[i];
    return s;
  }
  // Offset of linear index g for operand slot `slot`.
  int64_t offset(int slot, int64_t g) const {
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
      int64_t v = g % ext[i];
      g /= ext[i];
      off += v * str[slot][i];
    }
    return off;
  }
};

struct Analysis {
  tc_plan_info info{};
  Group g[4];
  bool empty_out = false;   // some extent of C is 0: nothing to compute
  bool empty_sum = false;   // some contracted extent is 0: C <- beta * C
  bool a_kfast = false;     // kernel A's stride-1 mode leads the contracted group
  bool b_kfast = false;     // kernel B's stride-1 mode leads the contracted group
  // GEMV / DOT / GER recipes: which memory-bound kernel runs them
  enum { KERNEL_GETT = 0, KERNEL_LANES_OUT = 1, KERNEL_LANES_K = 2, KERNEL_BATCHED = 3, KERNEL_SPLIT = 4 };
  int kernel = KERNEL_GETT;
  bool n_fastest = false;   // lanes-over-outputs: consecutive lanes along n
  int64_t seg = 1;          // lanes-over-k: contracted segments per output
  size_t part_offset = 0;   // byte offset of the partial sums in the workspace
  int64_t seg_len = 0;      // split-K GEMM: contracted indices per segment
  bool a_mfast = false;     // kernel A's stride-1 mode leads its free group
  bool b_nfast = false;     // kernel B's stride-1 mode leads its free group
  // GEMM: both operands can be copied in 16-byte pairs along their stride-1
  // mode (it leads the row or contracted group with an even extent, every
  // other stride is even) and the contracted group has at most
  // kDmaMaxKModes modes
  bool dma_ok = false;
  int dma_shape = 0;        // copy-fed output tile (kDma256x128, kDma128x256, kDma192x192)
  // split precision: padded sizes of the digit planes and workspace offsets
  int slices = 0;
  int crt_bits = 0;         // residue form: bits of the integer inputs
  bool crt_c_nfast = false; // residue form: C's stride-1 mode is in the N group
  int64_t Mp = 0, Np = 0, Kp = 0;
  size_t planesA_off = 0, planesB_off = 0, zres_off = 0, sigA_off = 0, sigB_off = 0, part_off = 0;
  int64_t elems[3] = {};    // entries of kernel A, kernel B, C (products of extents)
  // batched small contractions: slab descriptors (without pointers)
  int batched_P = 0;
  int slab_n[3] = {}, slab_size[3] = {}, slab_batch_fast[3] = {}, slab_dense[3] = {};
  int64_t slab_s0[3] = {};
  int slab_ext[3][TC_MAX_RANK] = {};
  int64_t slab_gstr[3][TC_MAX_RANK] = {};
  int slab_lstr[3][TC_MAX_RANK] = {};
  // COPY_GEMM: the copied operand (kernel slot) and its modes before and after
  // the copy, in the copied tensor's own storage order.
  int copy_slot = -1;
  int copy_rank = 0;
  int64_t copy_ext[TC_MAX_RANK] = {};
  int64_t copy_src_str[TC_MAX_RANK] = {};
  int64_t copy_dst_str[TC_MAX_RANK] = {};
};

// Validates, classifies (Sec. 3.2) and lays out the contraction.  On error
// returns the status and writes a message to *err.  allow_copy = false keeps
// the inner-product recipes from planning a copy of an input (a batch has no
// copy pass).
tc_status analyze(const TensorDesc& A, const TensorDesc& B, const TensorDesc& C, const tc_options& opt,
                  Analysis* out, std::string* err, bool allow_copy = true);

// Storage orders that let the contraction run as one direct GEMM (the
// paper's layout advice).  Bit t of `fixed` keeps tensor t (A, B, C) as
// given.  order[t][j] receives the mode of tensor t stored j-th (j = 0 at
// stride 1); out_desc[t] the tensor with packed column-major strides in that
// order (a fixed tensor keeps its strides); *out the analysis of that layout.
tc_status suggest_layout(const TensorDesc& A, const TensorDesc& B, const TensorDesc& C, int fixed,
                         int* order[3], TensorDesc out_desc[3], Analysis* out, std::string* err);

// Picker features of an analysis (TC_PICKER_FEATURES floats).
void picker_features(const Analysis& an, const TensorDesc& A, const TensorDesc& B, const TensorDesc& C, float* f);

// The picker's candidates: (recipe, GEMM tile).
struct Candidate {
  tc_recipe recipe;
  int tile;
};
constexpr Candidate kCandidates[TC_PICKER_CANDIDATES] = {
    {TC_RECIPE_GEMM, 8},       {TC_RECIPE_GEMM, 14},      {TC_RECIPE_GEMM, 1},       {TC_RECIPE_GEMM, 9},
    {TC_RECIPE_GEMM, 11},      {TC_RECIPE_GEMM, 12},      {TC_RECIPE_COPY_GEMM, 8},  {TC_RECIPE_COPY_GEMM, 1},
    {TC_RECIPE_COPY_GEMM, 9},  {TC_RECIPE_COPY_GEMM, 11}, {TC_RECIPE_COPY_GEMM, 12}, {TC_RECIPE_GEMV, -1},
    {TC_RECIPE_DOT, -1},       {TC_RECIPE_GER, -1},       {TC_RECIPE_AUTO, -1}};
// The first candidate of the explicit table (not the last, TC_RECIPE_AUTO)
// that an analysis corresponds to (-1 if none).
int candidate_of(const Analysis& an);

// The paper's class (0, 1, 2, 31, 32) from labels and stride-1 positions of
// the two inputs after normalisation (exposed for tests through tc_analyze).
int paper_class(const TensorDesc& A, const TensorDesc& B, const TensorDesc& C, int unitA, int unitB);

}  // namespace tc
