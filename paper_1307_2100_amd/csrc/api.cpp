// C ABI of the contraction library: plans, execution, permute, errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
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
                       const int32_t* lc, const tc_options* opt, tc::Analysis* an, tc::TensorDesc* keep = nullptr,
                       tc_options* keep_opt = nullptr) {
  tc::TensorDesc A, B, C;
  tc_status s;
  if ((s = fill_desc(&A, ra, ea, sa, la, "A")) != TC_OK) return s;
  if ((s = fill_desc(&B, rb, eb, sb, lb, "B")) != TC_OK) return s;
  if ((s = fill_desc(&C, rc, ec, sc, lc, "C")) != TC_OK) return s;
  tc_options o;
  tc_options_default(&o);
  if (opt) {
    // A C caller may store any integer in the enum fields: check them as
    // plain ints before any is read as its enum type
    static_assert(sizeof(tc_precision) == sizeof(int) && sizeof(tc_recipe) == sizeof(int) &&
                      sizeof(tc_picker) == sizeof(int),
                  "enum fields of tc_options are int-sized");
    int prec, rec, pick;
    std::memcpy(&prec, &opt->precision, sizeof(int));
    std::memcpy(&rec, &opt->recipe, sizeof(int));
    std::memcpy(&pick, &opt->picker, sizeof(int));
    if (prec < TC_PREC_F64 || prec > TC_PREC_F64_CRT_INT8 || rec < TC_RECIPE_AUTO || rec > TC_RECIPE_DOT ||
        pick < TC_PICKER_RULES || pick > TC_PICKER_TUNED)
      return fail(TC_ERR_INVALID_ARG, "invalid tc_options field");
    o = *opt;
  }
  std::string err;
  s = tc::analyze(A, B, C, o, an, &err);
  if (s != TC_OK) return fail(s, err);
  if (keep) {
    keep[0] = A;
    keep[1] = B;
    keep[2] = C;
  }
  if (keep_opt) *keep_opt = o;
  return TC_OK;
}

// Offset tables of an analysis: one per (group, operand) with more than one
// mode, appended to `host`; a group of zero or one mode is affine.  `pos`
// pairs each table-backed Offs with its start in `host`, to be pointed at the
// device copy once uploaded.
struct OffsTargets {
  tc::Offs *aM, *aK, *aL, *bN, *bK, *bL, *cM, *cN, *cL;
};
// Block tables of a contracted group of several modes, for inner products
// with lanes along the contracted range: the entries go in blocks of at most
// 64 over two modes p and q -- A's and B's stride-1 modes when they differ
// (then b_p x b_q = 8 x 8 where the extents allow, so both operands are read
// in runs of neighbours instead of one of them with strided lanes), else the
// stride-1 mode (up to 64 of it) and the next mode.  Blocks go column-major
// over (p's block, q's block, the other modes); each gets its base offset in
// A and B and its extents along p and q (ragged at the ends of p and q).
void build_k_blocks(const tc::Group& g, tc::BatchItem& it, std::vector<int64_t>& host,
                    std::vector<std::pair<tc::Offs*, size_t>>& pos) {
  int p = -1, q = -1;
  for (int d = 0; d < g.n; ++d) {
    if (g.str[tc::SA][d] == 1 && p < 0) p = d;
    if (g.str[tc::SB][d] == 1 && q < 0) q = d;
  }
  const bool f1 = p >= 0 && q >= 0 && p != q;
  if (!f1) {
    if (p < 0) p = q >= 0 ? q : 0;
    q = p == 0 ? 1 : 0;  // g.n >= 2
  }
  const int64_t ep = g.ext[p], eq = g.ext[q];
  const int64_t bp = f1 ? std::min<int64_t>(ep, 8) : std::min<int64_t>(ep, 64);
  const int64_t bq = std::min<int64_t>(eq, 64 / bp);
  int64_t ext[TC_MAX_RANK], sa[TC_MAX_RANK], sb[TC_MAX_RANK];
  int n = 0;
  ext[n] = (ep + bp - 1) / bp, sa[n] = bp * g.str[tc::SA][p], sb[n] = bp * g.str[tc::SB][p], ++n;
  ext[n] = (eq + bq - 1) / bq, sa[n] = bq * g.str[tc::SA][q], sb[n] = bq * g.str[tc::SB][q], ++n;
  for (int d = 0; d < g.n; ++d)
    if (d != p && d != q) ext[n] = g.ext[d], sa[n] = g.str[tc::SA][d], sb[n] = g.str[tc::SB][d], ++n;
  int64_t nblk = 1;
  for (int d = 0; d < n; ++d) nblk *= ext[d];
  it.kblk = 1;
  it.kbp = (int)bp;
  it.nblk = nblk;
  it.ksa_p = g.str[tc::SA][p], it.ksa_q = g.str[tc::SA][q];
  it.ksb_p = g.str[tc::SB][p], it.ksb_q = g.str[tc::SB][q];
  tc::Offs* dst[3] = {&it.g.aK, &it.g.bK, &it.klim};
  for (int t = 0; t < 3; ++t) {
    *dst[t] = tc::Offs{};
    pos.push_back({dst[t], host.size()});
    int64_t idx[TC_MAX_RANK] = {};
    int64_t off = 0;
    const int64_t* st = t == 0 ? sa : sb;
    for (int64_t j = 0; j < nblk; ++j) {
      if (t < 2) {
        host.push_back(off);
      } else {
        const int64_t lp = std::min(bp, ep - idx[0] * bp), lq = std::min(bq, eq - idx[1] * bq);
        host.push_back(lp | (lq << 8));
      }
      for (int d = 0; d < n; ++d) {
        if (t < 2) off += st[d];
        if (++idx[d] < ext[d]) break;
        if (t < 2) off -= st[d] * ext[d];
        idx[d] = 0;
      }
    }
  }
}

void build_tables(const tc::Analysis& an, const OffsTargets& t, std::vector<int64_t>& host,
                  std::vector<std::pair<tc::Offs*, size_t>>& pos, bool skip_k = false) {
  const tc::Group* G = an.g;
  struct Want {
    int group, slot;
    tc::Offs* dst;
  } want[9] = {{tc::GM, tc::SA, t.aM}, {tc::GK, tc::SA, t.aK}, {tc::GL, tc::SA, t.aL},
               {tc::GN, tc::SB, t.bN}, {tc::GK, tc::SB, t.bK}, {tc::GL, tc::SB, t.bL},
               {tc::GM, tc::SC, t.cM}, {tc::GN, tc::SC, t.cN}, {tc::GL, tc::SC, t.cL}};
  for (int w = 0; w < 9; ++w) {
    const tc::Group& g = G[want[w].group];
    *want[w].dst = tc::Offs{};
    if (g.n <= 1 || an.empty_out) {
      want[w].dst->tab = nullptr;
      want[w].dst->stride = g.n == 1 ? g.str[want[w].slot][0] : 0;
      continue;
    }
    if (skip_k && want[w].group == tc::GK) continue;  // the caller builds block tables
    const int64_t n = g.size();
    pos.push_back({want[w].dst, host.size()});
    // column-major walk of the group's multi-index with a running offset (no
    // division per entry): the same values as g.offset(slot, i) for i < n
    const int64_t* st = g.str[want[w].slot];
    int64_t idx[TC_MAX_RANK] = {};
    int64_t off = 0;
    for (int64_t i = 0; i < n; ++i) {
      host.push_back(off);
      for (int d = 0; d < g.n; ++d) {
        off += st[d];
        if (++idx[d] < g.ext[d]) break;
        off -= st[d] * g.ext[d];
        idx[d] = 0;
      }
    }
  }
}

// Uploads the tables in one allocation and points the Offs at it.
tc_status upload_tables(const std::vector<int64_t>& host, const std::vector<std::pair<tc::Offs*, size_t>>& pos,
                        int64_t** dev) {
  *dev = nullptr;
  if (host.empty()) return TC_OK;
  hipError_t e = hipMalloc((void**)dev, host.size() * sizeof(int64_t));
  if (e != hipSuccess) return fail(TC_ERR_NOMEM, std::string("hipMalloc of offset tables: ") + hipGetErrorString(e));
  e = hipMemcpy(*dev, host.data(), host.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(*dev);
    *dev = nullptr;
    return hip_fail(e, "hipMemcpy of offset tables");
  }
  for (auto& wp : pos) {
    wp.first->tab = *dev + wp.second;
    wp.first->stride = 0;
  }
  return TC_OK;
}

// Slab-engine parameters of a batch-dominated contraction: the operands'
// slab descriptors, the per-index LDS offset tables (appended to `host`), the
// points per workgroup for `lds_doubles` of LDS and the fast divisors.  The
// batch offsets bp.aL, bp.bL, bp.cL must already be set by build_tables.
tc_status fill_slab(const tc::Analysis& an, tc::BatchedParams& bp, int lds_doubles, std::vector<int64_t>& host,
                    std::vector<std::pair<tc::Offs*, size_t>>& pos) {
  const tc::Group* G = an.g;
  const tc_plan_info& info = an.info;
  tc::SlabDesc* d[3] = {&bp.a, &bp.b, &bp.c};
  const tc::Offs* xl[3] = {&bp.aL, &bp.bL, &bp.cL};
  for (int slot = 0; slot < 3; ++slot) {
    tc::SlabDesc& sd = *d[slot];
    sd.n = an.slab_n[slot];
    sd.size = an.slab_size[slot];
    sd.size_div = tc::make_fastdiv((uint32_t)an.slab_size[slot]);
    sd.batch_fast = an.slab_batch_fast[slot];
    sd.dense = an.slab_dense[slot];
    sd.s0 = an.slab_s0[slot];
    // contiguous: dense with unit stride and the batch offset an affine step of one slab
    sd.contig = sd.dense && !sd.batch_fast && sd.s0 == 1 && xl[slot]->tab == nullptr &&
                        xl[slot]->stride == (int64_t)sd.size && G[tc::GL].n <= 1
                    ? 1
                    : 0;
    for (int i = 0; i < an.slab_n[slot]; ++i) {
      sd.div[i] = tc::make_fastdiv((uint32_t)an.slab_ext[slot][i]);
      sd.gstr[i] = an.slab_gstr[slot][i];
      sd.lstr[i] = an.slab_lstr[slot][i];
    }
  }
  // LDS offset tables: (slot, group, offsets, canonical weight of the group's linear index)
  struct Want {
    int slot, group;
    tc::Offs* dst;
    int64_t canon;
  } want[6] = {{tc::SA, tc::GM, &bp.am, info.K}, {tc::SA, tc::GK, &bp.ak, 1},
               {tc::SB, tc::GN, &bp.bn, info.K}, {tc::SB, tc::GK, &bp.bk, 1},
               {tc::SC, tc::GM, &bp.cm, info.N}, {tc::SC, tc::GN, &bp.cn, 1}};
  for (const Want& w : want) {
    const tc::Group& g = G[w.group];
    *w.dst = tc::Offs{};
    if (!an.slab_dense[w.slot]) {
      w.dst->stride = w.canon;
      continue;
    }
    const int64_t s0 = an.slab_s0[w.slot];
    if (g.n <= 1) {
      w.dst->stride = g.n == 1 ? g.str[w.slot][0] / s0 : 0;
      continue;
    }
    pos.push_back({w.dst, host.size()});
    for (int64_t i = 0; i < g.size(); ++i) host.push_back(g.offset(w.slot, i) / s0);
  }
  const int per = an.slab_size[0] + an.slab_size[1] + an.slab_size[2];
  const int P = tc::slab_points(per, (int)info.K, lds_doubles);
  if (P < 1) return fail(TC_ERR_UNSUPPORTED, "per-point slabs do not fit the workgroup's LDS");
  bp.P = P;
  bp.M = (int)info.M;
  bp.N = (int)info.N;
  bp.K = (int)info.K;
  bp.L = info.L;
  bp.P_div = tc::make_fastdiv((uint32_t)P);
  bp.N_div = tc::make_fastdiv((uint32_t)bp.N);
  bp.sC_div = tc::make_fastdiv((uint32_t)bp.c.size);
  return TC_OK;
}

}  // namespace

struct tc_plan_s {
  tc::Analysis an;
  tc::TensorDesc desc[3];  // A, B, C as given
  tc_options opt{};
  int device = 0;
  int64_t* d_tables = nullptr;
  // per-group offsets of each kernel operand (A: M,K,L; B: N,K,L; C: M,N,L)
  tc::Offs aM{}, aK{}, aL{}, bN{}, bK{}, bL{}, cM{}, cN{}, cL{};
  tc::BatchedParams slab{};  // slab-engine layout (batch-dominated plans)
};

// The picker's network on the device: parameters, Adam moments, gradients
// and the activations of one batch of at most max_batch rows.
struct tc_mlp_s {
  tc::MlpDims d{};
  int max_batch = 0;
  int step = 0;
  float* params = nullptr;
  float* grads = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* sums = nullptr;
  tc::MlpScratch w{};
  std::vector<float*> owned;
  ~tc_mlp_s() {
    for (float* p : owned) (void)hipFree(p);
  }
  hipError_t alloc(float** p, int64_t n) {
    hipError_t e = hipMalloc((void**)p, (size_t)(n > 0 ? n : 1) * sizeof(float));
    if (e == hipSuccess) owned.push_back(*p);
    return e;
  }
  hipError_t init() {
    const int64_t np = d.num_params(), B = max_batch;
    hipError_t e;
    if ((e = alloc(&params, np)) || (e = alloc(&grads, np)) || (e = alloc(&m, np)) || (e = alloc(&v, np)) ||
        (e = alloc(&sums, 2)) || (e = alloc(&w.H1, B * d.hidden)) || (e = alloc(&w.H2, B * d.hidden)) ||
        (e = alloc(&w.Y, B * d.n_out)) || (e = alloc(&w.dY, B * d.n_out)) || (e = alloc(&w.dH2, B * d.hidden)) ||
        (e = alloc(&w.dH1, B * d.hidden)))
      return e;
    if ((e = hipMemset(m, 0, np * sizeof(float))) || (e = hipMemset(v, 0, np * sizeof(float)))) return e;
    return hipSuccess;
  }
};

namespace {

// The model TC_PICKER_MLP plans consult, and the tune cache of TC_PICKER_TUNED.
struct Picker {
  std::mutex mu;
  tc_mlp_s* net = nullptr;
  int device = -1;
  std::vector<float> mean, stdev;
  float* d_in = nullptr;
  float* d_out = nullptr;
  // private non-blocking stream: a prediction at plan time does not wait for
  // the caller's queued work
  hipStream_t stream = nullptr;
  std::map<std::string, int> tune;  // shape signature -> candidate
  void drop() {
    delete net;
    net = nullptr;
    if (d_in) (void)hipFree(d_in);
    if (d_out) (void)hipFree(d_out);
    if (stream) (void)hipStreamDestroy(stream);
    d_in = d_out = nullptr;
    stream = nullptr;
  }
};
Picker g_picker;

// Candidates ordered by predicted time, fastest first (empty without a model
// for the current device, or on failure).
std::vector<int> picker_order(const float* feat) {
  std::vector<int> order;
  std::lock_guard<std::mutex> lock(g_picker.mu);
  if (!g_picker.net) return order;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != g_picker.device) return order;
  float x[TC_PICKER_FEATURES], y[TC_PICKER_CANDIDATES];
  for (int i = 0; i < TC_PICKER_FEATURES; ++i)
    x[i] = (feat[i] - g_picker.mean[i]) / (g_picker.stdev[i] > 0.f ? g_picker.stdev[i] : 1.f);
  tc_mlp_s* n = g_picker.net;
  hipStream_t st = g_picker.stream;
  if (hipMemcpyAsync(g_picker.d_in, x, sizeof(x), hipMemcpyHostToDevice, st) != hipSuccess) return order;
  if (tc::mlp_forward(n->d, n->params, g_picker.d_in, n->w.H1, n->w.H2, g_picker.d_out, 1, st) != hipSuccess)
    return order;
  if (hipMemcpyAsync(y, g_picker.d_out, sizeof(y), hipMemcpyDeviceToHost, st) != hipSuccess) return order;
  if (hipStreamSynchronize(st) != hipSuccess) return order;
  for (int c = 0; c < TC_PICKER_CANDIDATES; ++c) order.push_back(c);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return y[a] < y[b]; });
  return order;
}

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

// A shape's signature: extents, strides and label pattern of A, B and C.
std::string shape_signature(const tc::TensorDesc* d) {
  std::ostringstream os;
  for (int t = 0; t < 3; ++t) {
    os << (t ? "|" : "");
    for (int i = 0; i < d[t].rank; ++i) {
      // labels renumbered by first appearance, so that renaming does not matter
      int idx = 0;
      bool found = false;
      for (int u = 0; u < 3 && !found; ++u)
        for (int j = 0; j < d[u].rank && !found; ++j) {
          if (d[u].lab[j] == d[t].lab[i]) found = true;
          else idx++;
        }
      os << idx << ":" << d[t].ext[i] << ":" << d[t].str[i] << ",";
    }
  }
  return os.str();
}

}  // namespace

// A batch: items (layouts of its contractions) and the task list of the
// current tile configuration live on the device; pointers and scalars go
// through a pinned host buffer and a small device array at every execution.
struct tc_batch_s {
  int n = 0;
  int device = 0;
  int num_cus = 256;
  int lds_per_cu = 160 * 1024;
  int slab_lds = tc::kBatchSlabLdsDoubles;  // slab LDS (doubles) of the current configuration
  int config = -1;
  int use_graph = 1;
  int64_t ntasks = 0;
  std::vector<tc::BatchItem> items;
  std::vector<tc_plan_info> analyses;
  int64_t* d_tables = nullptr;
  tc::BatchItem* d_items = nullptr;
  tc::BatchTask* d_tasks = nullptr;
  int64_t* d_chunks = nullptr;
  int64_t nchunks = 0;                          // chunks of all engines
  int64_t chunk_base[tc::kBatchEngines] = {};   // engine e's bounds start at d_chunks + chunk_base[e]
  int64_t engine_chunks[tc::kBatchEngines] = {};
  std::vector<int> direct_items;                // slab items launched on their own
  std::vector<int64_t> direct_blocks;
  tc::BatchPtrs* h_ptrs = nullptr;
  hipStream_t capture_stream = nullptr;
  hipEvent_t done = nullptr;
  bool done_recorded = false;
  bool staged = false;  // h_ptrs holds the pointers of the last execution
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* graph_ws = nullptr;

  ~tc_batch_s() {
    if (done_recorded) (void)hipEventSynchronize(done);
    drop_graph();
    if (done) (void)hipEventDestroy(done);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    if (h_ptrs) (void)hipHostFree(h_ptrs);
    if (d_tasks) (void)hipFree(d_tasks);
    if (d_chunks) (void)hipFree(d_chunks);
    if (d_items) (void)hipFree(d_items);
    if (d_tables) (void)hipFree(d_tables);
  }

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    graph_ws = nullptr;
  }

  // workspace: [pointers][task counter][completion counters][partial sums]
  int64_t n_cnt = 0;      // completion counters of the current configuration
  int64_t n_parts = 0;    // partial sums (doubles) of the current configuration
  size_t max_ws = 0;      // largest workspace over all configurations
  size_t ptrs_bytes() const { return ((size_t)n * sizeof(tc::BatchPtrs) + 255) / 256 * 256; }
  size_t cnt_offset() const { return ptrs_bytes() + 256; }
  size_t parts_offset(int64_t ncnt) const { return cnt_offset() + ((size_t)ncnt * 4 + 255) / 256 * 256; }
  size_t workspace_for(int64_t ncnt, int64_t nparts) const {
    return parts_offset(ncnt) + (size_t)nparts * sizeof(double);
  }
  size_t workspace_bytes() const { return max_ws; }

  // Split-K for a GEMM item with `tiles` output tiles: long contracted ranges
  // are cut into segments of at least 1024 indices so that no task dominates.
  static void item_split(int64_t tiles, int64_t K, int* S, int64_t* len) {
    *S = 1;
    *len = K;
    if (K <= 2048 || tiles >= 256) return;
    int64_t l = (K + 255) / 256;
    if (l < 1024) l = 1024;
    l = (l + 15) / 16 * 16;
    *S = (int)((K + l - 1) / l);
    *len = l;
  }

  // Tiles and task list for one tile configuration, longest tasks first.
  tc_status set_config(int cfg) {
    try {
      return set_config_lists(cfg);
    } catch (const std::bad_alloc&) {
      return fail(TC_ERR_NOMEM, "host allocation of the batch task list failed");
    }
  }

  tc_status set_config_lists(int cfg) {
    if (done_recorded) (void)hipEventSynchronize(done);
    drop_graph();
    const int BM = tc::kBatchTileBM[cfg], BN = tc::kBatchTileBN[cfg];
    struct HT {
      double cost;
      tc::BatchTask t;
    };
    std::vector<HT> tasks;
    n_cnt = 0;
    n_parts = 0;
    direct_items.clear();
    direct_blocks.clear();
    // Slab tasks run in their own launch with 16 KB of LDS per workgroup (the
    // budget measured best for the grid contractions on their own).
    slab_lds = tc::kBatchSlabLdsDoubles;
    for (tc::BatchItem& it : items) {
      if (it.kind != tc::kBatchSlab) continue;
      const int per = it.b.a.size + it.b.b.size + it.b.c.size;
      it.b.P = std::max(1, tc::slab_points(per, it.b.K, slab_lds));
      it.b.P_div = tc::make_fastdiv((uint32_t)it.b.P);
    }
    for (int i = 0; i < n; ++i) {
      tc::BatchItem& it = items[i];
      if (it.kind == tc::kBatchLanesK || it.kind == tc::kBatchLanesOut) {
        // memory-bound: groups of outputs; long contracted ranges in segments
        const bool lk = it.kind == tc::kBatchLanesK;
        const int64_t outputs = it.g.M * it.g.N * it.g.L;
        // contracted indices per segment (blocked items: blocks of up to 64)
        const int64_t target = lk ? (it.kblk ? 1024 : 16384) : 512;
        const int64_t range = it.kblk ? it.nblk : it.g.K;
        int S = 1;
        int64_t len = range;
        if (range > 2 * target) {
          S = (int)((range + target - 1) / target);
          len = (range + S - 1) / S;
        }
        it.ksplit = S;
        it.seg_len = len;
        it.part_off = S > 1 ? n_parts : 0;
        it.cnt_off = S > 1 ? n_cnt : 0;
        if (lk) {
          // four (output, segment) units per task, one per wavefront; one
          // completion counter per output
          if (S > 1) {
            n_parts += outputs * S;
            n_cnt += outputs;
          }
          const int64_t ntask = (outputs * S + tc::kLanesKOutputs - 1) / tc::kLanesKOutputs;
          const double cost = 16.0 * tc::kLanesKOutputs * (double)len * (it.kblk ? 64.0 : 1.0) / 8e12;
          for (int64_t t = 0; t < ntask; ++t) tasks.push_back({cost, tc::BatchTask{i, 0, t}});
        } else {
          // 256 outputs along lanes per task, one task per (output group, segment)
          const int64_t groups = (outputs + tc::kLanesOutOutputs - 1) / tc::kLanesOutOutputs;
          if (S > 1) {
            n_parts += outputs * S;
            n_cnt += groups;
          }
          const double cost = 16.0 * tc::kLanesOutOutputs * (double)len / 8e12;
          for (int64_t t = 0; t < groups; ++t)
            for (int sg = 0; sg < S; ++sg) tasks.push_back({cost, tc::BatchTask{i, sg, t}});
        }
      } else if (it.kind == tc::kBatchGemm) {
        it.tilesM = (it.g.M + BM - 1) / BM;
        it.tilesN = (it.g.N + BN - 1) / BN;
        const int64_t nt = it.tilesM * it.tilesN * it.g.L;
        int S;
        int64_t len;
        item_split(nt, it.g.K, &S, &len);
        it.ksplit = S;
        it.seg_len = len;
        it.part_off = S > 1 ? n_parts : 0;
        it.cnt_off = S > 1 ? n_cnt : 0;
        if (S > 1) {
          n_parts += nt * S * BM * BN;
          n_cnt += nt;
        }
        // cost of a task: the larger of its FP64 MFMA time and its load time
        const double k = (double)(S > 1 ? len : it.g.K);
        const double flops = 2.0 * BM * BN * k, bytes = 8.0 * (BM + BN) * k + 8.0 * BM * BN;
        const double cost = std::max(flops / 78.6e12, bytes / 8e12);
        for (int64_t t = 0; t < nt; ++t)
          for (int sg = 0; sg < S; ++sg) tasks.push_back({cost, tc::BatchTask{i, sg, t}});
      } else {
        const int64_t nt = (it.b.L + it.b.P - 1) / it.b.P;
        if (nt >= (int64_t)tc::kBatchDirectSlabBlocksPerCu * num_cus && nt <= 0x7fffffffLL) {
          // fills the chip on its own: a launch of its own, no task-list overhead
          direct_items.push_back(i);
          direct_blocks.push_back(nt);
          continue;
        }
        const double bytes = 8.0 * it.b.P * (it.b.a.size + it.b.b.size + it.b.c.size);
        const double cost = bytes / 8e12;
        for (int64_t t = 0; t < nt; ++t) tasks.push_back({cost, tc::BatchTask{i, 0, t}});
      }
    }
    // One task list per engine, longest tasks first, laid out one after the
    // other; each engine's list is cut into chunks of about its total / (128
    // per CU) cost: the costly tasks at the front get chunks of their own,
    // the many cheap ones share (measured on a 2000-contraction batch: 4 per
    // CU 8.7 ms, 16 per CU 7.0, 64 per CU 6.6, 128 to 1024 per CU 6.55).
    std::stable_sort(tasks.begin(), tasks.end(), [&](const HT& a, const HT& b) {
      const int ea = tc::batch_engine_of(items[a.t.item].kind), eb = tc::batch_engine_of(items[b.t.item].kind);
      return ea != eb ? ea < eb : a.cost > b.cost;
    });
    std::vector<tc::BatchTask> flat(tasks.size());
    for (size_t i = 0; i < tasks.size(); ++i) flat[i] = tasks[i].t;
    std::vector<int64_t> bounds;
    size_t first = 0;
    for (int e = 0; e < tc::kBatchEngines; ++e) {
      size_t last = first;
      double total = 0.0;
      while (last < tasks.size() && tc::batch_engine_of(items[tasks[last].t.item].kind) == e)
        total += tasks[last++].cost;
      chunk_base[e] = (int64_t)bounds.size();
      bounds.push_back((int64_t)first);
      const double target = total / (128.0 * num_cus);
      double acc = 0.0;
      for (size_t i = first; i < last; ++i) {
        acc += tasks[i].cost;
        if (acc >= target || i + 1 == last) {
          bounds.push_back((int64_t)i + 1);
          acc = 0.0;
        }
      }
      engine_chunks[e] = (int64_t)bounds.size() - 1 - chunk_base[e];
      first = last;
    }
    nchunks = 0;
    for (int e = 0; e < tc::kBatchEngines; ++e) nchunks += engine_chunks[e];
    if (d_chunks) (void)hipFree(d_chunks);
    d_chunks = nullptr;
    if (hipMalloc((void**)&d_chunks, bounds.size() * sizeof(int64_t)) != hipSuccess)
      return fail(TC_ERR_NOMEM, "batch chunk list");
    if (hipMemcpy(d_chunks, bounds.data(), bounds.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess)
      return fail(TC_ERR_HIP, "upload of batch chunk list");
    if (d_tasks) (void)hipFree(d_tasks);
    d_tasks = nullptr;
    ntasks = (int64_t)flat.size();
    if (ntasks > 0) {
      if (hipMalloc((void**)&d_tasks, flat.size() * sizeof(tc::BatchTask)) != hipSuccess)
        return fail(TC_ERR_NOMEM, "batch task list");
      if (hipMemcpy(d_tasks, flat.data(), flat.size() * sizeof(tc::BatchTask), hipMemcpyHostToDevice) != hipSuccess)
        return fail(TC_ERR_HIP, "upload of batch task list");
    }
    if (!d_items && hipMalloc((void**)&d_items, items.size() * sizeof(tc::BatchItem)) != hipSuccess)
      return fail(TC_ERR_NOMEM, "batch items");
    if (hipMemcpy(d_items, items.data(), items.size() * sizeof(tc::BatchItem), hipMemcpyHostToDevice) != hipSuccess)
      return fail(TC_ERR_HIP, "upload of batch items");
    config = cfg;
    return TC_OK;
  }

  hipError_t enqueue(void* ws, hipStream_t st) {
    tc::BatchPtrs* d_ptrs = (tc::BatchPtrs*)ws;
    unsigned long long* counter = (unsigned long long*)((char*)ws + ptrs_bytes());
    unsigned* cnt = (unsigned*)((char*)ws + cnt_offset());
    double* parts = (double*)((char*)ws + parts_offset(n_cnt));
    hipError_t e = hipMemcpyAsync(d_ptrs, h_ptrs, sizeof(tc::BatchPtrs) * n, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    tc::BatchLaunch bl{};
    bl.items = d_items;
    bl.ptrs = d_ptrs;
    bl.tasks = d_tasks;
    bl.ntasks = ntasks;
    for (int e = 0; e < tc::kBatchEngines; ++e) {
      bl.chunks[e] = d_chunks + chunk_base[e];
      bl.nchunks[e] = engine_chunks[e];
    }
    bl.counter = counter;
    bl.parts = parts;
    bl.tile_cnt = cnt;
    bl.n_cnt = n_cnt;
    bl.config = config;
    bl.slab_lds_doubles = slab_lds;
    bl.num_cus = num_cus;
    bl.direct_items = direct_items.data();
    bl.direct_blocks = direct_blocks.data();
    bl.ndirect = (int)direct_items.size();
    bl.host_items = items.data();
    return tc::launch_batch(bl, st);
  }

  tc_status execute(const double* const* A, const double* const* B, double* const* C, const double* alpha,
                    const double* beta, void* ws, size_t wsb, hipStream_t st, int graph_on) {
    if (!A || !B || !C || !alpha || !beta) return fail(TC_ERR_INVALID_ARG, "null pointer array");
    if (!ws || wsb < workspace_for(n_cnt, n_parts))
      return fail(TC_ERR_WORKSPACE, "batch workspace of " + std::to_string(wsb) + " bytes, needs " +
                                        std::to_string(workspace_bytes()));
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != device)
      return fail(TC_ERR_INVALID_ARG, "batch was created on another device");
    for (int i = 0; i < n; ++i) {
      if (analyses[i].M * analyses[i].N * analyses[i].L > 0 && !C[i])
        return fail(TC_ERR_INVALID_ARG, "null C in batch entry " + std::to_string(i));
    }
    // New pointers or scalars go through the pinned staging buffer, which the
    // previous execution must have consumed first.  Unchanged ones (the usual
    // serving loop over the same buffers) are already staged: no wait.
    bool same = staged;
    for (int i = 0; i < n && same; ++i) {
      const tc::BatchPtrs v{A[i], B[i], C[i], alpha[i], beta[i]};
      same = std::memcmp(&v, &h_ptrs[i], sizeof(v)) == 0;
    }
    if (!same) {
      if (done_recorded && hipEventSynchronize(done) != hipSuccess) return fail(TC_ERR_HIP, "batch event sync");
      for (int i = 0; i < n; ++i) h_ptrs[i] = tc::BatchPtrs{A[i], B[i], C[i], alpha[i], beta[i]};
      staged = true;
    }
    hipError_t e;
    if (graph_on) {
      if (!exec || graph_ws != ws) {
        drop_graph();
        e = hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t eq = enqueue(ws, capture_stream);
        e = hipStreamEndCapture(capture_stream, &graph);
        if (eq != hipSuccess) return hip_fail(eq, "batch capture");
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        graph_ws = ws;
      }
      e = hipGraphLaunch(exec, st);
      if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    } else {
      e = enqueue(ws, st);
      if (e != hipSuccess) return hip_fail(e, "batch launch");
    }
    e = hipEventRecord(done, st);
    if (e != hipSuccess) return hip_fail(e, "batch event record");
    done_recorded = true;
    return TC_OK;
  }
};

namespace tc {
tc_status set_error(tc_status s, const char* msg) { return fail(s, msg ? msg : ""); }
}  // namespace tc

extern "C" {

void tc_options_default(tc_options* opt) {
  if (!opt) return;
  opt->precision = TC_PREC_F64;
  opt->recipe = TC_RECIPE_AUTO;
  opt->picker = TC_PICKER_RULES;
  opt->split_slices = 0;
  opt->tile_id = -1;
  opt->copy_tile = -1;
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

tc_status tc_suggest_layout(int ra, const int64_t* ea, const int64_t* sa, const int32_t* la, int rb,
                            const int64_t* eb, const int64_t* sb, const int32_t* lb, int rc, const int64_t* ec,
                            const int64_t* sc, const int32_t* lc, int fixed, int32_t* order_a, int32_t* order_b,
                            int32_t* order_c, tc_plan_info* info) {
  if (fixed < 0 || fixed > 7) return fail(TC_ERR_INVALID_ARG, "fixed must be a mask of bits 0 (A), 1 (B), 2 (C)");
  const int rank[3] = {ra, rb, rc};
  const int64_t* ext[3] = {ea, eb, ec};
  const int64_t* str[3] = {sa, sb, sc};
  const int32_t* lab[3] = {la, lb, lc};
  int32_t* ord[3] = {order_a, order_b, order_c};
  const char* name[3] = {"A", "B", "C"};
  tc::TensorDesc T[3];
  for (int t = 0; t < 3; ++t) {
    if (rank[t] > 0 && !ord[t]) return fail(TC_ERR_INVALID_ARG, std::string("null order array for ") + name[t]);
    // without strides: packed column-major in the listed order
    std::vector<int64_t> packed(rank[t] > 0 && rank[t] <= TC_MAX_RANK ? rank[t] : 0);
    int64_t stride = 1;
    for (size_t i = 0; i < packed.size() && ext[t]; ++i) {
      packed[i] = stride;
      stride *= ext[t][i] > 0 ? ext[t][i] : 1;
    }
    tc_status s = fill_desc(&T[t], rank[t], ext[t], str[t] ? str[t] : packed.data(), lab[t], name[t]);
    if (s != TC_OK) return s;
  }
  int order[3][TC_MAX_RANK];
  int* op[3] = {order[0], order[1], order[2]};
  tc::TensorDesc suggested[3];
  tc::Analysis an;
  std::string err;
  tc_status s = tc::suggest_layout(T[0], T[1], T[2], fixed, op, suggested, &an, &err);
  if (s != TC_OK) return fail(s, err);
  for (int t = 0; t < 3; ++t)
    for (int j = 0; j < rank[t]; ++j) ord[t][j] = order[t][j];
  if (info) *info = an.info;
  return TC_OK;
}

tc_status tc_plan_create(tc_plan_t* out, int ra, const int64_t* ea, const int64_t* sa, const int32_t* la, int rb,
                         const int64_t* eb, const int64_t* sb, const int32_t* lb, int rc, const int64_t* ec,
                         const int64_t* sc, const int32_t* lc, const tc_options* opt) {
  if (!out) return fail(TC_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  tc_plan_s* p = new (std::nothrow) tc_plan_s();
  if (!p) return fail(TC_ERR_NOMEM, "host allocation failed");
  tc_status s = analyze_args(ra, ea, sa, la, rb, eb, sb, lb, rc, ec, sc, lc, opt, &p->an, p->desc, &p->opt);
  if (s != TC_OK) {
    delete p;
    return s;
  }
  p->an.info.picked_candidate = -1;
  if (p->opt.precision == TC_PREC_F64 && p->opt.recipe == TC_RECIPE_AUTO && p->opt.tile_id < 0 &&
      (p->opt.picker == TC_PICKER_MLP || p->opt.picker == TC_PICKER_TUNED)) {
    std::vector<int> order;
    if (p->opt.picker == TC_PICKER_MLP) {
      float f[TC_PICKER_FEATURES];
      tc::picker_features(p->an, p->desc[0], p->desc[1], p->desc[2], f);
      order = picker_order(f);
    } else {
      std::lock_guard<std::mutex> lock(g_picker.mu);
      auto it = g_picker.tune.find(shape_signature(p->desc));
      if (it != g_picker.tune.end()) order.push_back(it->second);
    }
    // re-plan with the first candidate this shape can take; with none, keep the rules' plan
    for (int c : order) {
      tc_options o = p->opt;
      o.recipe = tc::kCandidates[c].recipe;
      o.tile_id = tc::kCandidates[c].tile;
      tc::Analysis an2;
      std::string err;
      if (tc::analyze(p->desc[0], p->desc[1], p->desc[2], o, &an2, &err) == TC_OK) {
        if (an2.dma_ok && p->opt.copy_tile < 0) {  // the picker chooses the tile; the copy-fed output tile follows the round rule
          an2.dma_shape = tc::dma_shape(an2.info.M, an2.info.N, an2.info.L);
          an2.info.copy_fed = 1 + an2.dma_shape;
        }
        p->an = an2;
        p->an.info.picked_candidate = c;
        break;
      }
    }
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  std::vector<int64_t> host;
  std::vector<std::pair<tc::Offs*, size_t>> pos;
  const bool slab = p->an.kernel == tc::Analysis::KERNEL_BATCHED;
  try {
    build_tables(p->an, OffsTargets{&p->aM, &p->aK, &p->aL, &p->bN, &p->bK, &p->bL, &p->cM, &p->cN, &p->cL}, host,
                 pos);
    if (slab) {
      p->slab.aL = p->aL;
      p->slab.bL = p->bL;
      p->slab.cL = p->cL;
      s = fill_slab(p->an, p->slab, tc::kBatchedSlabLdsDoubles, host, pos);
    }
  } catch (const std::bad_alloc&) {
    s = fail(TC_ERR_NOMEM, "host allocation of offset tables failed");
  }
  if (s != TC_OK) {
    delete p;
    return s;
  }
  s = upload_tables(host, pos, &p->d_tables);
  if (s != TC_OK) {
    delete p;
    return s;
  }
  if (slab) {  // the batch offsets as uploaded
    p->slab.aL = p->aL;
    p->slab.bL = p->bL;
    p->slab.cL = p->cL;
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
    sp.crt = info.precision == TC_PREC_F64_CRT_INT8;
    sp.bits = an.crt_bits;
    sp.crt_tile = info.tile_id;
    sp.c_nfast = an.crt_c_nfast;
    char* ws = (char*)workspace;
    sp.planesA = ws + an.planesA_off;
    sp.planesB = ws + an.planesB_off;
    sp.zres = ws + an.zres_off;
    sp.sigA = (double*)(ws + an.sigA_off);
    sp.sigB = (double*)(ws + an.sigB_off);
    sp.part = (double*)(ws + an.part_off);
    sp.alpha = alpha;
    sp.beta = beta;
    e = tc::launch_split_contraction(sp, s);
    return e == hipSuccess ? TC_OK : hip_fail(e, "split-precision launch");
  }

  if (an.copy_slot >= 0) {
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
  if (an.kernel == tc::Analysis::KERNEL_BATCHED) {
    tc::BatchedParams bp = plan->slab;
    bp.A = KA;
    bp.B = KB;
    bp.C = C;
    bp.alpha = alpha;
    bp.beta = beta;
    e = tc::launch_batched_small(bp, s);
    return e == hipSuccess ? TC_OK : hip_fail(e, "batched launch");
  }
  if (an.kernel == tc::Analysis::KERNEL_LANES_OUT) {
    double* part = an.seg > 1 ? (double*)((char*)workspace + an.part_offset) : nullptr;
    e = tc::launch_lanes_over_outputs(gp, an.n_fastest, an.seg, part, s);
    return e == hipSuccess ? TC_OK : hip_fail(e, "lanes-over-outputs launch");
  }
  if (an.kernel == tc::Analysis::KERNEL_LANES_K) {
    double* part = an.seg > 1 ? (double*)((char*)workspace + an.part_offset) : nullptr;
    e = tc::launch_lanes_over_k(gp, an.seg, part, s);
    return e == hipSuccess ? TC_OK : hip_fail(e, "lanes-over-k launch");
  }
  int tile = info.tile_id >= 0 ? info.tile_id : 1;
  double* parts = info.k_split > 1 ? (double*)((char*)workspace + an.part_offset) : nullptr;
  // the copy-fed kernel needs both operands (after any COPY step) on 16-byte boundaries
  const bool dma = an.dma_ok && ((reinterpret_cast<uintptr_t>(KA) | reinterpret_cast<uintptr_t>(KB)) & 15) == 0;
  tc::DmaK dk{};
  if (dma) {
    const tc::Group& gk = an.g[tc::GK];
    dk.n = gk.n;
    dk.shape = an.dma_shape;
    for (int i = 0; i < gk.n && i < tc::kDmaMaxKModes; ++i) {
      dk.ext[i] = gk.ext[i];
      dk.sa[i] = gk.str[tc::SA][i];
      dk.sb[i] = gk.str[tc::SB][i];
    }
  }
  e = tc::launch_gett_f64(gp, tile, an.a_kfast, an.b_kfast, info.k_split, an.seg_len, parts, s, dma ? &dk : nullptr);
  if (e != hipSuccess) return hip_fail(e, "gett launch");
  return TC_OK;
}

tc_status tc_permute(int rank, const int64_t* ext, const int64_t* str_x, const int64_t* str_y, const double* X,
                     double* Y, void* stream) {
  if (rank < 0 || rank > TC_MAX_RANK) return fail(TC_ERR_RANK, "rank outside 0..16");
  if (rank > 0 && (!ext || !str_x || !str_y)) return fail(TC_ERR_INVALID_ARG, "null extent or stride array");
  tc::TensorDesc y;
  y.rank = rank;
  bool empty = false;
  for (int i = 0; i < rank; ++i) {
    if (ext[i] < 0 || str_x[i] < 0 || str_y[i] < 0) return fail(TC_ERR_INVALID_ARG, "negative extent or stride");
    y.ext[i] = ext[i];
    y.str[i] = str_y[i];
    empty = empty || ext[i] == 0;
  }
  if (empty) return TC_OK;
  {
    // element count and both address spans within 2^56 (checked products)
    const int64_t cap = (int64_t)1 << 56;
    int64_t total = 1, span_x = 0, span_y = 0, r = 0;
    for (int i = 0; i < rank; ++i) {
      bool ok = !__builtin_mul_overflow(total, ext[i], &total) && total <= cap;
      ok = ok && !__builtin_mul_overflow(ext[i] - 1, str_x[i], &r) && !__builtin_add_overflow(span_x, r, &span_x);
      ok = ok && !__builtin_mul_overflow(ext[i] - 1, str_y[i], &r) && !__builtin_add_overflow(span_y, r, &span_y);
      if (!ok || span_x > cap || span_y > cap)
        return fail(TC_ERR_INVALID_ARG, "element count or address span exceeds 2^56");
    }
  }
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

tc_status tc_batch_create(tc_batch_t* out, int n, const tc_plan_t* plans) {
  if (!out) return fail(TC_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (n < 1 || !plans) return fail(TC_ERR_INVALID_ARG, "a batch needs n >= 1 plans");
  tc_batch_s* b = new (std::nothrow) tc_batch_s();
  if (!b) return fail(TC_ERR_NOMEM, "host allocation failed");
  b->n = n;
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipGetDevice");
  }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, b->device);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipGetDeviceProperties");
  }
  b->num_cus = prop.multiProcessorCount;
  if (prop.maxSharedMemoryPerMultiProcessor > 0) b->lds_per_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
  std::vector<int64_t> host;
  std::vector<std::pair<tc::Offs*, size_t>> pos;
  try {
    b->items.resize(n);
    b->analyses.resize(n);
  } catch (const std::bad_alloc&) {
    delete b;
    return fail(TC_ERR_NOMEM, "host allocation of batch items failed");
  }
  for (int i = 0; i < n; ++i) {
    const tc_plan_s* p = plans[i];
    if (!p) {
      delete b;
      return fail(TC_ERR_INVALID_ARG, "null plan in batch");
    }
    if (p->opt.precision != TC_PREC_F64) {
      delete b;
      return fail(TC_ERR_UNSUPPORTED, "batches run FP64 plans only");
    }
    if (p->device != b->device) {
      delete b;
      return fail(TC_ERR_INVALID_ARG, "plans of a batch must share the current device");
    }
    // Re-plan for the batch's engines: batch-dominated contractions keep the
    // slab engine, the memory-bound matrix-vector and inner-product shapes
    // their lanes kernels, everything else runs as direct GEMM tiles (a batch
    // has no per-contraction copy pass).
    tc_options o = p->opt;
    o.recipe = TC_RECIPE_AUTO;
    tc::Analysis an;
    std::string err;
    tc_status s = tc::analyze(p->desc[0], p->desc[1], p->desc[2], o, &an, &err, false);
    const bool keep = an.kernel == tc::Analysis::KERNEL_BATCHED || an.kernel == tc::Analysis::KERNEL_LANES_K ||
                      an.kernel == tc::Analysis::KERNEL_LANES_OUT;
    if (s == TC_OK && !keep) {
      o.recipe = TC_RECIPE_GEMM;
      s = tc::analyze(p->desc[0], p->desc[1], p->desc[2], o, &an, &err, false);
    }
    if (s != TC_OK) {
      delete b;
      return fail(s, err);
    }
    tc::BatchItem& it = b->items[i];
    std::memset(&it, 0, sizeof(it));
    it.swapped = an.info.swapped;
    try {
      if (an.kernel == tc::Analysis::KERNEL_BATCHED) {
        build_tables(an, OffsTargets{&it.g.aM, &it.g.aK, &it.b.aL, &it.g.bN, &it.g.bK, &it.b.bL, &it.g.cM, &it.g.cN,
                                     &it.b.cL},
                     host, pos);
        s = fill_slab(an, it.b, tc::kBatchSlabLdsDoubles, host, pos);
      } else {
        // inner products over a contracted group of several modes address
        // it through block tables
        const bool kblk = an.kernel == tc::Analysis::KERNEL_LANES_K && an.g[tc::GK].n >= 2 && !an.empty_out &&
                          an.g[tc::GK].size() > 0;  // an empty sum keeps the plain (empty) tables
        build_tables(an, OffsTargets{&it.g.aM, &it.g.aK, &it.g.aL, &it.g.bN, &it.g.bK, &it.g.bL, &it.g.cM, &it.g.cN,
                                     &it.g.cL},
                     host, pos, kblk);
        if (kblk) build_k_blocks(an.g[tc::GK], it, host, pos);
      }
    } catch (const std::bad_alloc&) {
      s = fail(TC_ERR_NOMEM, "host allocation of offset tables failed");
    }
    if (s != TC_OK) {
      delete b;
      return s;
    }
    if (an.kernel == tc::Analysis::KERNEL_BATCHED) {
      it.kind = 1;
    } else {
      it.kind = an.kernel == tc::Analysis::KERNEL_LANES_K     ? tc::kBatchLanesK
                : an.kernel == tc::Analysis::KERNEL_LANES_OUT ? tc::kBatchLanesOut
                                                              : tc::kBatchGemm;
      it.n_fastest = an.n_fastest ? 1 : 0;
      it.akf = an.a_kfast ? 1 : 0;
      it.bkf = an.b_kfast ? 1 : 0;
      it.g.M = an.empty_out ? 0 : an.info.M;
      it.g.N = an.empty_out ? 0 : an.info.N;
      it.g.K = an.info.K;
      it.g.L = an.empty_out ? 0 : an.info.L;
    }
    b->analyses[i] = an.info;
  }
  // table pointers live inside the items: patch them after the upload
  tc_status s = upload_tables(host, pos, &b->d_tables);
  if (s != TC_OK) {
    delete b;
    return s;
  }
  e = hipHostMalloc((void**)&b->h_ptrs, sizeof(tc::BatchPtrs) * n, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete b;
    return fail(TC_ERR_NOMEM, "pinned host staging of batch pointers");
  }
  e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "batch stream/event");
  }
  // the workspace must serve every tile configuration (the autotuner switches)
  for (int cfg = tc::kNumBatchTiles - 1; cfg >= 0; --cfg) {
    s = b->set_config(cfg);
    if (s != TC_OK) {
      delete b;
      return s;
    }
    b->max_ws = std::max(b->max_ws, b->workspace_for(b->n_cnt, b->n_parts));
  }
  *out = b;
  return TC_OK;
}

tc_status tc_batch_workspace(tc_batch_t batch, size_t* bytes) {
  if (!batch || !bytes) return fail(TC_ERR_INVALID_ARG, "null batch or bytes");
  *bytes = batch->workspace_bytes();
  return TC_OK;
}

tc_status tc_batch_execute(tc_batch_t batch, const double* const* A, const double* const* B, double* const* C,
                           const double* alpha, const double* beta, void* workspace, size_t workspace_bytes,
                           void* stream) {
  if (!batch) return fail(TC_ERR_INVALID_ARG, "batch is null");
  return batch->execute(A, B, C, alpha, beta, workspace, workspace_bytes, (hipStream_t)stream, batch->use_graph);
}

tc_status tc_batch_set_options(tc_batch_t batch, int tile_config, int use_graph) {
  if (!batch) return fail(TC_ERR_INVALID_ARG, "batch is null");
  if (tile_config < -1 || tile_config >= tc::kNumBatchTiles)
    return fail(TC_ERR_INVALID_ARG, "batch tile configuration out of range");
  if (tile_config >= 0 && tile_config != batch->config) {
    tc_status s = batch->set_config(tile_config);
    if (s != TC_OK) return s;
  }
  batch->use_graph = use_graph ? 1 : 0;
  return TC_OK;
}

tc_status tc_batch_query(tc_batch_t batch, int64_t* ntasks, int* tile_config, int* use_graph) {
  if (!batch) return fail(TC_ERR_INVALID_ARG, "batch is null");
  if (ntasks) {
    *ntasks = batch->ntasks;
    for (int64_t b : batch->direct_blocks) *ntasks += b;
  }
  if (tile_config) *tile_config = batch->config;
  if (use_graph) *use_graph = batch->use_graph;
  return TC_OK;
}

tc_status tc_batch_autotune(tc_batch_t batch, const double* const* A, const double* const* B, double* const* C,
                            const double* alpha, const double* beta, void* workspace, size_t workspace_bytes,
                            void* stream, int* best_config, double* best_ms) {
  if (!batch) return fail(TC_ERR_INVALID_ARG, "batch is null");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(TC_ERR_HIP, "event create");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(TC_ERR_HIP, "event create");
  }
  int best = -1;
  float best_t = 0.f;
  tc_status s = TC_OK;
  for (int cfg = 0; cfg < tc::kNumBatchTiles && s == TC_OK; ++cfg) {
    s = batch->set_config(cfg);
    if (s != TC_OK) break;
    // one untimed run, then the median of three timed ones
    s = batch->execute(A, B, C, alpha, beta, workspace, workspace_bytes, st, 0);
    float t[3];
    for (int r = 0; r < 3 && s == TC_OK; ++r) {
      (void)hipEventRecord(e0, st);
      s = batch->execute(A, B, C, alpha, beta, workspace, workspace_bytes, st, 0);
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) s = fail(TC_ERR_HIP, "event sync");
      (void)hipEventElapsedTime(&t[r], e0, e1);
    }
    if (s != TC_OK) break;
    std::sort(t, t + 3);
    if (best < 0 || t[1] < best_t) {
      best = cfg;
      best_t = t[1];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != TC_OK) return s;
  s = batch->set_config(best);
  if (s != TC_OK) return s;
  if (best_config) *best_config = best;
  if (best_ms) *best_ms = best_t;
  return TC_OK;
}

tc_status tc_batch_destroy(tc_batch_t batch) {
  delete batch;
  return TC_OK;
}

tc_status tc_picker_candidate(int index, tc_recipe* recipe, int* tile_id) {
  if (index < 0 || index >= TC_PICKER_CANDIDATES) return fail(TC_ERR_INVALID_ARG, "candidate index out of range");
  if (recipe) *recipe = tc::kCandidates[index].recipe;
  if (tile_id) *tile_id = tc::kCandidates[index].tile;
  return TC_OK;
}

tc_status tc_picker_features(int ra, const int64_t* ea, const int64_t* sa, const int32_t* la, int rb,
                             const int64_t* eb, const int64_t* sb, const int32_t* lb, int rc, const int64_t* ec,
                             const int64_t* sc, const int32_t* lc, float* feat, int* rule_candidate) {
  if (!feat) return fail(TC_ERR_INVALID_ARG, "feat is null");
  tc::Analysis an;
  tc::TensorDesc d[3];
  tc_status s = analyze_args(ra, ea, sa, la, rb, eb, sb, lb, rc, ec, sc, lc, nullptr, &an, d);
  if (s != TC_OK) return s;
  tc::picker_features(an, d[0], d[1], d[2], feat);
  if (rule_candidate) *rule_candidate = tc::candidate_of(an);
  return TC_OK;
}

tc_status tc_picker_install(const float* params, int64_t n_params, int n_in, int hidden, int n_out,
                            const float* feat_mean, const float* feat_std) {
  if (!params || !feat_mean || !feat_std) return fail(TC_ERR_INVALID_ARG, "null model array");
  if (n_in != TC_PICKER_FEATURES || n_out != TC_PICKER_CANDIDATES || hidden < 1 || hidden > 4096)
    return fail(TC_ERR_INVALID_ARG, "model dimensions do not match the picker");
  tc_mlp_t net = nullptr;
  tc_status s = tc_mlp_create(&net, n_in, hidden, n_out, 1);
  if (s != TC_OK) return s;
  if (n_params != net->d.num_params()) {
    tc_mlp_destroy(net);
    return fail(TC_ERR_INVALID_ARG, "parameter count does not match the dimensions");
  }
  s = tc_mlp_set_params(net, params);
  if (s != TC_OK) {
    tc_mlp_destroy(net);
    return s;
  }
  std::lock_guard<std::mutex> lock(g_picker.mu);
  g_picker.drop();
  g_picker.net = net;
  (void)hipGetDevice(&g_picker.device);
  g_picker.mean.assign(feat_mean, feat_mean + n_in);
  g_picker.stdev.assign(feat_std, feat_std + n_in);
  if (hipMalloc((void**)&g_picker.d_in, n_in * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&g_picker.d_out, n_out * sizeof(float)) != hipSuccess ||
      hipStreamCreateWithFlags(&g_picker.stream, hipStreamNonBlocking) != hipSuccess) {
    g_picker.drop();
    return fail(TC_ERR_NOMEM, "picker buffers");
  }
  return TC_OK;
}

tc_status tc_picker_uninstall(void) {
  std::lock_guard<std::mutex> lock(g_picker.mu);
  g_picker.drop();
  return TC_OK;
}

tc_status tc_plan_autotune(tc_plan_t plan, const double* A, const double* B, double* C, void* stream,
                           int* best_candidate, double* best_ms, double* candidate_ms) {
  if (!plan || !A || !B || !C) return fail(TC_ERR_INVALID_ARG, "null plan or buffer");
  hipStream_t st = (hipStream_t)stream;
  // plans of every candidate the shape can take, and one workspace for all
  tc_plan_t cand[TC_PICKER_CANDIDATES] = {};
  size_t ws_max = 0;
  const tc::TensorDesc* d = plan->desc;
  for (int c = 0; c < TC_PICKER_CANDIDATES; ++c) {
    tc_options o = plan->opt;
    o.recipe = tc::kCandidates[c].recipe;
    o.tile_id = tc::kCandidates[c].tile;
    o.picker = TC_PICKER_RULES;
    if (tc_plan_create(&cand[c], d[0].rank, d[0].ext, d[0].str, d[0].lab, d[1].rank, d[1].ext, d[1].str, d[1].lab,
                       d[2].rank, d[2].ext, d[2].str, d[2].lab, &o) != TC_OK)
      cand[c] = nullptr;  // a candidate this shape cannot take
    else
      ws_max = std::max(ws_max, cand[c]->an.info.workspace_bytes);
  }
  auto destroy_all = [&]() {
    for (tc_plan_t& c : cand)
      if (c) tc_plan_destroy(c), c = nullptr;
  };
  void* ws = nullptr;
  if (ws_max && hipMalloc(&ws, ws_max) != hipSuccess) {
    destroy_all();
    return fail(TC_ERR_NOMEM, "autotune workspace");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  tc_status result = TC_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) result = fail(TC_ERR_HIP, "event create");
  // time per execution of `reps` back-to-back executions, in ms
  auto timed = [&](tc_plan_t cp, int reps, float* ms) -> tc_status {
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) {
      tc_status s = tc_execute(cp, A, B, C, 1.0, 0.0, ws, ws_max, stream);
      if (s != TC_OK) return s;
    }
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) return fail(TC_ERR_HIP, "event sync");
    if (hipEventElapsedTime(ms, e0, e1) != hipSuccess) return fail(TC_ERR_HIP, "event time");
    *ms /= (float)reps;
    return TC_OK;
  };
  int best = -1;
  float best_t = 0.f;
  for (int c = 0; c < TC_PICKER_CANDIDATES && result == TC_OK; ++c) {
    if (candidate_ms) candidate_ms[c] = -1.0;
    if (!cand[c]) continue;
    float t1 = 0.f, t[3] = {0.f, 0.f, 0.f};
    // a candidate that cannot run on this shape (an error status, not a
    // device fault) is skipped; a failing stream ends the tuning
    tc_status cs = timed(cand[c], 1, &t1);  // warm-up, and an estimate of the time
    const int reps = (int)std::min(64.0, std::max(1.0, std::ceil(0.2 / std::max(t1, 1e-4f))));
    for (int r = 0; r < 3 && cs == TC_OK; ++r) cs = timed(cand[c], reps, &t[r]);
    if (cs != TC_OK) {
      if (hipStreamSynchronize(st) != hipSuccess) result = fail(TC_ERR_HIP, "stream failed during autotune");
      continue;
    }
    std::sort(t, t + 3);
    if (candidate_ms) candidate_ms[c] = t[1];
    if (best < 0 || t[1] < best_t) {
      best = c;
      best_t = t[1];
    }
  }
  if (result == TC_OK && hipStreamSynchronize(st) != hipSuccess) result = fail(TC_ERR_HIP, "stream sync");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (ws) (void)hipFree(ws);
  destroy_all();
  if (result != TC_OK) return result;
  if (best < 0) return fail(TC_ERR_UNSUPPORTED, "no candidate could run");
  {
    std::lock_guard<std::mutex> lock(g_picker.mu);
    g_picker.tune[shape_signature(plan->desc)] = best;
  }
  if (best_candidate) *best_candidate = best;
  if (best_ms) *best_ms = best_t;
  return TC_OK;
}

tc_status tc_tune_cache_save(const char* path) {
  if (!path) return fail(TC_ERR_INVALID_ARG, "path is null");
  std::ofstream f(path);
  if (!f) return fail(TC_ERR_INVALID_ARG, std::string("cannot write ") + path);
  const std::string arch = device_arch();
  std::lock_guard<std::mutex> lock(g_picker.mu);
  for (auto& kv : g_picker.tune) f << TC_VERSION << " " << arch << " " << kv.first << " " << kv.second << "\n";
  return f ? TC_OK : fail(TC_ERR_INVALID_ARG, "write failed");
}

tc_status tc_tune_cache_load(const char* path) {
  if (!path) return fail(TC_ERR_INVALID_ARG, "path is null");
  std::ifstream f(path);
  if (!f) return fail(TC_ERR_INVALID_ARG, std::string("cannot read ") + path);
  const std::string arch = device_arch();
  std::string ver, ar, sig;
  int c;
  std::lock_guard<std::mutex> lock(g_picker.mu);
  while (f >> ver >> ar >> sig >> c) {
    if (ver != TC_VERSION || ar != arch || c < 0 || c >= TC_PICKER_CANDIDATES) continue;  // stale entry
    g_picker.tune[sig] = c;
  }
  return TC_OK;
}

tc_status tc_mlp_create(tc_mlp_t* out, int n_in, int hidden, int n_out, int max_batch) {
  if (!out) return fail(TC_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (n_in < 1 || hidden < 1 || n_out < 1 || max_batch < 1) return fail(TC_ERR_INVALID_ARG, "MLP sizes must be >= 1");
  tc_mlp_s* n = new (std::nothrow) tc_mlp_s();
  if (!n) return fail(TC_ERR_NOMEM, "host allocation failed");
  n->d = tc::MlpDims{n_in, hidden, n_out};
  n->max_batch = max_batch;
  if (n->init() != hipSuccess) {
    delete n;
    return fail(TC_ERR_NOMEM, "MLP device buffers");
  }
  *out = n;
  return TC_OK;
}

tc_status tc_mlp_num_params(tc_mlp_t mlp, int64_t* n) {
  if (!mlp || !n) return fail(TC_ERR_INVALID_ARG, "null argument");
  *n = mlp->d.num_params();
  return TC_OK;
}

tc_status tc_mlp_set_params(tc_mlp_t mlp, const float* host_params) {
  if (!mlp || !host_params) return fail(TC_ERR_INVALID_ARG, "null argument");
  hipError_t e = hipMemcpy(mlp->params, host_params, mlp->d.num_params() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "MLP parameter upload");
  mlp->step = 0;
  const size_t bytes = mlp->d.num_params() * sizeof(float);
  if ((e = hipMemset(mlp->m, 0, bytes)) != hipSuccess || (e = hipMemset(mlp->v, 0, bytes)) != hipSuccess)
    return hip_fail(e, "MLP moment reset");
  return TC_OK;
}

tc_status tc_mlp_get_params(tc_mlp_t mlp, float* host_params) {
  if (!mlp || !host_params) return fail(TC_ERR_INVALID_ARG, "null argument");
  hipError_t e = hipMemcpy(host_params, mlp->params, mlp->d.num_params() * sizeof(float), hipMemcpyDeviceToHost);
  return e == hipSuccess ? TC_OK : hip_fail(e, "MLP parameter download");
}

tc_status tc_mlp_forward(tc_mlp_t mlp, const float* X, float* Y, int batch, void* stream) {
  if (!mlp || !X || !Y) return fail(TC_ERR_INVALID_ARG, "null argument");
  if (batch < 0 || batch > mlp->max_batch) return fail(TC_ERR_INVALID_ARG, "batch exceeds max_batch");
  hipError_t e = tc::mlp_forward(mlp->d, mlp->params, X, mlp->w.H1, mlp->w.H2, Y, batch, (hipStream_t)stream);
  return e == hipSuccess ? TC_OK : hip_fail(e, "MLP forward");
}

tc_status tc_mlp_loss_grad(tc_mlp_t mlp, const float* X, const float* T, const float* M, int batch, float* grads,
                           float* loss, void* stream) {
  if (!mlp || !X || !T || !M) return fail(TC_ERR_INVALID_ARG, "null argument");
  if (batch < 1 || batch > mlp->max_batch) return fail(TC_ERR_INVALID_ARG, "batch outside 1..max_batch");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = tc::mlp_forward(mlp->d, mlp->params, X, mlp->w.H1, mlp->w.H2, mlp->w.Y, batch, st);
  if (e == hipSuccess) e = tc::mlp_backward(mlp->d, mlp->params, X, T, M, mlp->w, mlp->grads, mlp->sums, batch, st);
  if (e == hipSuccess && grads)
    e = hipMemcpyAsync(grads, mlp->grads, mlp->d.num_params() * sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, mlp->sums, sizeof(float), hipMemcpyDeviceToDevice, st);
  return e == hipSuccess ? TC_OK : hip_fail(e, "MLP loss/gradient");
}

tc_status tc_mlp_train_step(tc_mlp_t mlp, const float* X, const float* T, const float* M, int batch, float lr,
                            float* loss, void* stream) {
  tc_status s = tc_mlp_loss_grad(mlp, X, T, M, batch, nullptr, loss, stream);
  if (s != TC_OK) return s;
  mlp->step++;
  hipError_t e = tc::mlp_adam(mlp->params, mlp->grads, mlp->m, mlp->v, mlp->d.num_params(), lr, mlp->step,
                              (hipStream_t)stream);
  return e == hipSuccess ? TC_OK : hip_fail(e, "MLP Adam step");
}

tc_status tc_mlp_destroy(tc_mlp_t mlp) {
  delete mlp;
  return TC_OK;
}

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
