// C ABI of the contraction library: plans, execution, permute, errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/tc.h"
#include "kernels.hpp"
#include "planner.hpp"

namespace {

thread_local std::string g_last_error;

tc_status fail(tc_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

tc_status hip_fail(hipError_t e, const char* what) {
  return fail(TC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

tc_status fill_desc(tc::TensorDesc* d, int rank, const int64_t* ext, const int64_t* str, const int32_t* lab,
                    const char* name) {
  if (rank < 0 || rank > TC_MAX_RANK)
    return fail(TC_ERR_RANK, std::string("rank of ") + name + " outside 0.." + std::to_string(TC_MAX_RANK));
  if (rank > 0 && (!ext || !str || !lab))
    return fail(TC_ERR_INVALID_ARG, std::string("null extent/stride/label array for ") + name);
  d->rank = rank;
  for (int i = 0; i < rank; ++i) {
    d->ext[i] = ext[i];
    d->str[i] = str[i];
    d->lab[i] = lab[i];
  }
  return TC_OK;
}

tc_status analyze_args(int ra, const int64_t* ea, const int64_t* sa, const int32_t* la, int rb, const int64_t* eb,
                       const int64_t* sb, const int32_t* lb, int rc, const int64_t* ec, const int64_t* sc,
                       const int32_t* lc, const tc_options* opt, tc::Analysis* an) {
  tc::TensorDesc A, B, C;
  tc_status s;
  if ((s = fill_desc(&A, ra, ea, sa, la, "A")) != TC_OK) return s;
  if ((s = fill_desc(&B, rb, eb, sb, lb, "B")) != TC_OK) return s;
  if ((s = fill_desc(&C, rc, ec, sc, lc, "C")) != TC_OK) return s;
  tc_options o;
  tc_options_default(&o);
  if (opt) o = *opt;
  std::string err;
  s = tc::analyze(A, B, C, o, an, &err);
  if (s != TC_OK) return fail(s, err);
  return TC_OK;
}

}  // namespace

struct tc_plan_s {
  tc::Analysis an;
  int device = 0;
  int64_t* d_tables = nullptr;
  // per-group offsets of each kernel operand (A: M,K,L; B: N,K,L; C: M,N,L)
  tc::Offs aM{}, aK{}, aL{}, bN{}, bK{}, bL{}, cM{}, cN{}, cL{};
};

extern "C" {

void tc_options_default(tc_options* opt) {
  if (!opt) return;
  opt->precision = TC_PREC_F64;
  opt->recipe = TC_RECIPE_AUTO;
  opt->picker = TC_PICKER_RULES;
  opt->split_slices = 0;
  opt->tile_id = -1;
}

tc_status tc_analyze(int ra, const int64_t* ea, const int64_t* sa, const int32_t* la, int rb, const int64_t* eb,
                     const int64_t* sb, const int32_t* lb, int rc, const int64_t* ec, const int64_t* sc,
                     const int32_t* lc, const tc_options* opt, tc_plan_info* info) {
  if (!info) return fail(TC_ERR_INVALID_ARG, "info is null");
  tc::Analysis an;
  tc_status s = analyze_args(ra, ea, sa, la, rb, eb, sb, lb, rc, ec, sc, lc, opt, &an);
  if (s != TC_OK) return s;
  *info = an.info;
  return TC_OK;
}

tc_status tc_plan_create(tc_plan_t* out, int ra, const int64_t* ea, const int64_t* sa, const int32_t* la, int rb,
                         const int64_t* eb, const int64_t* sb, const int32_t* lb, int rc, const int64_t* ec,
                         const int64_t* sc, const int32_t* lc, const tc_options* opt) {
  if (!out) return fail(TC_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  tc_plan_s* p = new (std::nothrow) tc_plan_s();
  if (!p) return fail(TC_ERR_NOMEM, "host allocation failed");
  tc_status s = analyze_args(ra, ea, sa, la, rb, eb, sb, lb, rc, ec, sc, lc, opt, &p->an);
  if (s != TC_OK) {
    delete p;
    return s;
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  // Offset tables: one per (group, operand) with more than one mode; a group
  // of zero or one mode is affine and needs none.
  const tc::Group* G = p->an.g;
  struct Want {
    int group, slot;
    tc::Offs* dst;
  } want[9] = {{tc::GM, tc::SA, &p->aM}, {tc::GK, tc::SA, &p->aK}, {tc::GL, tc::SA, &p->aL},
               {tc::GN, tc::SB, &p->bN}, {tc::GK, tc::SB, &p->bK}, {tc::GL, tc::SB, &p->bL},
               {tc::GM, tc::SC, &p->cM}, {tc::GN, tc::SC, &p->cN}, {tc::GL, tc::SC, &p->cL}};
  std::vector<int64_t> host;
  std::vector<std::pair<int, size_t>> pos;  // (want index, start in host)
  for (int w = 0; w < 9; ++w) {
    const tc::Group& g = G[want[w].group];
    if (g.n <= 1 || p->an.empty_out) {
      want[w].dst->tab = nullptr;
      want[w].dst->stride = g.n == 1 ? g.str[want[w].slot][0] : 0;
      continue;
    }
    int64_t n = g.size();
    pos.push_back({w, host.size()});
    for (int64_t i = 0; i < n; ++i) host.push_back(g.offset(want[w].slot, i));
  }
  if (!host.empty()) {
    e = hipMalloc((void**)&p->d_tables, host.size() * sizeof(int64_t));
    if (e != hipSuccess) {
      delete p;
      return fail(TC_ERR_NOMEM, std::string("hipMalloc of offset tables: ") + hipGetErrorString(e));
    }
    e = hipMemcpy(p->d_tables, host.data(), host.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(p->d_tables);
      delete p;
      return hip_fail(e, "hipMemcpy of offset tables");
    }
    for (auto& wp : pos) {
      want[wp.first].dst->tab = p->d_tables + wp.second;
      want[wp.first].dst->stride = 0;
    }
  }
  *out = p;
  return TC_OK;
}

tc_status tc_plan_query(tc_plan_t plan, tc_plan_info* info) {
  if (!plan || !info) return fail(TC_ERR_INVALID_ARG, "null plan or info");
  *info = plan->an.info;
  return TC_OK;
}

tc_status tc_plan_destroy(tc_plan_t plan) {
  if (!plan) return TC_OK;
  if (plan->d_tables) (void)hipFree(plan->d_tables);
  delete plan;
  return TC_OK;
}

tc_status tc_execute(tc_plan_t plan, const double* A, const double* B, double* C, double alpha, double beta,
                     void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return fail(TC_ERR_INVALID_ARG, "plan is null");
  const tc::Analysis& an = plan->an;
  const tc_plan_info& info = an.info;
  if (an.empty_out) return TC_OK;
  if (!C) return fail(TC_ERR_INVALID_ARG, "C is null");
  if (!an.empty_sum && (!A || !B)) return fail(TC_ERR_INVALID_ARG, "A or B is null");
  if (workspace_bytes < info.workspace_bytes || (info.workspace_bytes && !workspace))
    return fail(TC_ERR_WORKSPACE, "workspace of " + std::to_string(workspace_bytes) + " bytes, plan needs " +
                                      std::to_string(info.workspace_bytes));
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != plan->device) return fail(TC_ERR_INVALID_ARG, "plan was created on another device");
  hipStream_t s = (hipStream_t)stream;

  if (an.empty_sum) {
    e = tc::launch_scale(C, plan->cM, plan->cN, plan->cL, info.M, info.N, info.L, beta, s);
    return e == hipSuccess ? TC_OK : hip_fail(e, "scale launch");
  }
  const double* KA = info.swapped ? B : A;
  const double* KB = info.swapped ? A : B;

  if (info.precision != TC_PREC_F64) {
    tc::SplitParams sp{};
    sp.A = KA;
    sp.B = KB;
    sp.C = C;
    sp.aM = plan->aM;
    sp.aK = plan->aK;
    sp.bN = plan->bN;
    sp.bK = plan->bK;
    sp.cM = plan->cM;
    sp.cN = plan->cN;
    sp.M = info.M;
    sp.N = info.N;
    sp.K = info.K;
    sp.Mp = an.Mp;
    sp.Np = an.Np;
    sp.Kp = an.Kp;
    sp.a_rfast = an.a_mfast;
    sp.a_kfast = an.a_kfast;
    sp.b_rfast = an.b_nfast;
    sp.b_kfast = an.b_kfast;
    sp.slices = an.slices;
    sp.fp8 = info.precision == TC_PREC_F64_SPLIT_FP8;
    char* ws = (char*)workspace;
    sp.planesA = ws + an.planesA_off;
    sp.planesB = ws + an.planesB_off;
    sp.sigA = (double*)(ws + an.sigA_off);
    sp.sigB = (double*)(ws + an.sigB_off);
    sp.part = (double*)(ws + an.part_off);
    sp.alpha = alpha;
    sp.beta = beta;
    e = tc::launch_split_contraction(sp, s);
    return e == hipSuccess ? TC_OK : hip_fail(e, "split-precision launch");
  }

  if (info.recipe == TC_RECIPE_COPY_GEMM && an.copy_slot >= 0) {
    tc::PermuteParams pp{};
    pp.X = an.copy_slot == tc::SA ? KA : KB;
    pp.Y = (double*)workspace;
    pp.rank = an.copy_rank;
    for (int i = 0; i < an.copy_rank; ++i) {
      pp.ext[i] = an.copy_ext[i];
      pp.sx[i] = an.copy_src_str[i];
      pp.sy[i] = an.copy_dst_str[i];
    }
    e = tc::launch_permute(pp, s);
    if (e != hipSuccess) return hip_fail(e, "permute launch");
    if (an.copy_slot == tc::SA)
      KA = (const double*)workspace;
    else
      KB = (const double*)workspace;
  }

  tc::GettParams gp{};
  gp.A = KA;
  gp.B = KB;
  gp.C = C;
  gp.aM = plan->aM;
  gp.aK = plan->aK;
  gp.aL = plan->aL;
  gp.bN = plan->bN;
  gp.bK = plan->bK;
  gp.bL = plan->bL;
  gp.cM = plan->cM;
  gp.cN = plan->cN;
  gp.cL = plan->cL;
  gp.M = info.M;
  gp.N = info.N;
  gp.K = info.K;
  gp.L = info.L;
  gp.alpha = alpha;
  gp.beta = beta;
  if (an.kernel == tc::Analysis::KERNEL_LANES_OUT) {
    e = tc::launch_lanes_over_outputs(gp, an.n_fastest, s);
    return e == hipSuccess ? TC_OK : hip_fail(e, "lanes-over-outputs launch");
  }
  if (an.kernel == tc::Analysis::KERNEL_LANES_K) {
    double* part = an.seg > 1 ? (double*)((char*)workspace + an.part_offset) : nullptr;
    e = tc::launch_lanes_over_k(gp, an.seg, part, s);
    return e == hipSuccess ? TC_OK : hip_fail(e, "lanes-over-k launch");
  }
  int tile = info.tile_id >= 0 ? info.tile_id : 1;
  e = tc::launch_gett_f64(gp, tile, an.a_kfast, an.b_kfast, s);
  if (e != hipSuccess) return hip_fail(e, "gett launch");
  return TC_OK;
}

tc_status tc_permute(int rank, const int64_t* ext, const int64_t* str_x, const int64_t* str_y, const double* X,
                     double* Y, void* stream) {
  if (rank < 0 || rank > TC_MAX_RANK) return fail(TC_ERR_RANK, "rank outside 0..16");
  if (rank > 0 && (!ext || !str_x || !str_y)) return fail(TC_ERR_INVALID_ARG, "null extent or stride array");
  tc::TensorDesc y;
  y.rank = rank;
  int64_t total = 1;
  for (int i = 0; i < rank; ++i) {
    if (ext[i] < 0 || str_x[i] < 0 || str_y[i] < 0) return fail(TC_ERR_INVALID_ARG, "negative extent or stride");
    y.ext[i] = ext[i];
    y.str[i] = str_y[i];
    total *= ext[i];
  }
  if (total == 0) return TC_OK;
  if (!X || !Y) return fail(TC_ERR_INVALID_ARG, "null X or Y");
  // reuse the output-overlap test of the planner through a trivial analysis
  {
    std::vector<std::pair<int64_t, int64_t>> m;
    for (int i = 0; i < rank; ++i)
      if (ext[i] > 1) m.push_back({str_y[i], ext[i]});
    std::sort(m.begin(), m.end());
    int64_t span = 1;
    for (auto& se : m) {
      if (se.first <= 0 || se.first < span) return fail(TC_ERR_OUTPUT_OVERLAP, "Y strides overlap");
      span = se.first * se.second;
    }
  }
  tc::PermuteParams pp{};
  pp.X = X;
  pp.Y = Y;
  pp.rank = 0;
  for (int i = 0; i < rank; ++i) {
    if (ext[i] == 1) continue;
    pp.ext[pp.rank] = ext[i];
    pp.sx[pp.rank] = str_x[i];
    pp.sy[pp.rank] = str_y[i];
    pp.rank++;
  }
  hipError_t e = tc::launch_permute(pp, (hipStream_t)stream);
  return e == hipSuccess ? TC_OK : hip_fail(e, "permute launch");
}

tc_status tc_batch_create(tc_batch_t* out, int, const tc_plan_t*) {
  if (out) *out = nullptr;
  return fail(TC_ERR_UNSUPPORTED, "batches are not built in");
}
tc_status tc_batch_workspace(tc_batch_t, size_t* bytes) {
  if (bytes) *bytes = 0;
  return fail(TC_ERR_UNSUPPORTED, "batches are not built in");
}
tc_status tc_batch_execute(tc_batch_t, const double* const*, const double* const*, double* const*, const double*,
                           const double*, void*, size_t, void*) {
  return fail(TC_ERR_UNSUPPORTED, "batches are not built in");
}
tc_status tc_batch_destroy(tc_batch_t) { return TC_OK; }

const char* tc_status_string(tc_status s) {
  switch (s) {
    case TC_OK: return "TC_OK";
    case TC_ERR_INVALID_ARG: return "TC_ERR_INVALID_ARG";
    case TC_ERR_LABEL: return "TC_ERR_LABEL";
    case TC_ERR_EXTENT_MISMATCH: return "TC_ERR_EXTENT_MISMATCH";
    case TC_ERR_OUTPUT_OVERLAP: return "TC_ERR_OUTPUT_OVERLAP";
    case TC_ERR_RANK: return "TC_ERR_RANK";
    case TC_ERR_WORKSPACE: return "TC_ERR_WORKSPACE";
    case TC_ERR_UNSUPPORTED: return "TC_ERR_UNSUPPORTED";
    case TC_ERR_HIP: return "TC_ERR_HIP";
    case TC_ERR_NOMEM: return "TC_ERR_NOMEM";
  }
  return "unknown tc_status";
}

const char* tc_last_error(void) { return g_last_error.c_str(); }

const char* tc_version(void) { return TC_VERSION; }

}  // extern "C"
