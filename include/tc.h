/*
 * tc.h -- binary tensor contractions on AMD Instinct MI355X (gfx950).
 *
 * Computes C <- alpha * sum A*B + beta * C for two dense FP64 tensors of any
 * order, any sets of contracted and free indices and any storage strides.
 * The operation is the paper's contraction (arXiv:1307.2100, "Towards an
 * Efficient Use of the BLAS Library for Multilinear Tensor Contractions"):
 * every index repeated in A and B and absent from C is summed over its whole
 * range (Sec. 2.3 and Appendix A); alpha and beta follow the BLAS GEMM
 * definition (Sec. 2.1).  Plans are classified with the paper's Delta-rule
 * and stride-1 test (Sec. 3.2: Classes 1, 2, 3.1, 3.2) and executed with the
 * recipe of the class (direct GEMM, COPY+GEMM, GEMV, DOT, GER; Sec. 3.2).
 *
 * Conventions shared by every entry point
 *   - A tensor is described by its rank r and three arrays of r entries:
 *     extents (int64, >= 0), strides in ELEMENTS (int64, >= 0) and labels
 *     (int32).  Mode 0 is the first index.  Equal labels name the same index.
 *   - A label in A and B but not C is contracted; in A and C only, a free
 *     index of A; in B and C only, a free index of B; in A, B and C, a batch
 *     index (all three are sliced along it -- an extension, the paper has no
 *     such index).  Any other placement, or a label repeated inside one
 *     tensor, is rejected with TC_ERR_LABEL.
 *   - Host arrays passed to the library are copied; the caller keeps
 *     ownership of every buffer it passes.  Device buffers (A, B, C,
 *     workspace) are caller-owned device memory; the library never frees them.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *     Execution is asynchronous on that stream.
 *   - Errors are reported as tc_status codes only; tc_last_error() returns a
 *     thread-local message describing the last failure of the calling thread.
 *     A call that fails at validation writes nothing to C.
 *   - Sizes: every count is a product of extents, formed with overflow-checked
 *     multiplication.  Each tensor's element count and address span
 *     (sum of (extent - 1) * stride) and the iteration space (product of the
 *     extents of all distinct labels) must not exceed 2^56, else
 *     TC_ERR_INVALID_ARG; a plan whose unfused index groups would need more
 *     than 2^31 offset-table entries gets TC_ERR_UNSUPPORTED.  Host allocation
 *     failures return TC_ERR_NOMEM; no C++ exception crosses the ABI.
 */
#ifndef TC_H_
#define TC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TC_MAX_RANK 16
#define TC_VERSION "1.0.0"

typedef struct tc_plan_s* tc_plan_t;
typedef struct tc_batch_s* tc_batch_t;

typedef enum {
  TC_OK = 0,
  TC_ERR_INVALID_ARG = 1,      /* null pointer, negative extent or stride, bad option */
  TC_ERR_LABEL = 2,            /* label repeated in a tensor or summed out of one operand */
  TC_ERR_EXTENT_MISMATCH = 3,  /* one label with two different extents */
  TC_ERR_OUTPUT_OVERLAP = 4,   /* C's strides map two entries to one address */
  TC_ERR_RANK = 5,             /* rank < 0 or > TC_MAX_RANK */
  TC_ERR_WORKSPACE = 6,        /* workspace smaller than tc_plan_info.workspace_bytes */
  TC_ERR_UNSUPPORTED = 7,      /* valid request the library does not implement */
  TC_ERR_HIP = 8,              /* a HIP runtime call failed (message in tc_last_error) */
  TC_ERR_NOMEM = 9             /* host or device allocation failed */
} tc_status;

typedef enum {
  TC_PREC_F64 = 0,             /* FP64 MFMA / FP64 vector arithmetic throughout */
  TC_PREC_F64_SPLIT_BF16 = 1,  /* FP64 operands split into BF16 slices, BF16 MFMA, FP32 exact chunks, FP64 sum */
  TC_PREC_F64_SPLIT_FP8 = 2,   /* the same with FP8 E4M3 slices */
  TC_PREC_F64_CRT_INT8 = 3     /* FP64 operands rounded to integers of split_bits bits, multiplied exactly
                                  as INT8 residues modulo split_slices coprime moduli (INT8 MFMA, INT32
                                  accumulation), the product rebuilt by the Chinese remainder theorem */
} tc_precision;

/* Residue GEMM configurations of TC_PREC_F64_CRT_INT8 plans (tc_options.tile_id). */
#define TC_CRT_NUM_TILES 12

/* Recipes of Sec. 3.2.  AUTO takes the class's recipe (3.2 -> GEMM, 3.1 ->
 * COPY_GEMM, 2 -> GEMV, 1 -> DOT, no contracted index -> GER); any other
 * value forces that recipe, which every class can run (results agree to
 * rounding; only speed differs). */
typedef enum {
  TC_RECIPE_AUTO = 0,
  TC_RECIPE_GEMM = 1,          /* one strided-gather MFMA GEMM over fused index groups */
  TC_RECIPE_COPY_GEMM = 2,     /* permute one operand into the workspace, then GEMM */
  TC_RECIPE_GEMV = 3,          /* matrix-vector products, one per output column */
  TC_RECIPE_GER = 4,           /* sum over the contracted index of rank-1 updates */
  TC_RECIPE_DOT = 5            /* one inner product per output entry */
} tc_recipe;

typedef enum {
  TC_PICKER_RULES = 0,         /* the paper's recipe for the class, largest index unsliced */
  TC_PICKER_MLP = 1,           /* learned model (falls back to rules when absent) */
  TC_PICKER_TUNED = 2          /* autotune cache (falls back to rules when absent) */
} tc_picker;

typedef struct {
  tc_precision precision;      /* default TC_PREC_F64 */
  tc_recipe recipe;            /* default TC_RECIPE_AUTO */
  tc_picker picker;            /* default TC_PICKER_RULES */
  int split_slices;            /* slices per operand for split precision (moduli for TC_PREC_F64_CRT_INT8,
                                  2 to 14); 0 = default (5 BF16, 8 FP8; for residues the fewest moduli
                                  that keep at least 40 bits per input for the plan's K) */
  int tile_id;                 /* GEMM tile configuration; -1 = chosen by the picker.  For
                                  TC_PREC_F64_CRT_INT8 plans: residue GEMM configuration, 0 to
                                  TC_CRT_NUM_TILES - 1, -1 = the default */
  int copy_tile;               /* output tile of the copy-fed FP64 kernel (taken for the 256x128 and
                                  128x256 tiles when tc_plan_info.copy_fed is set): 0 256x128, 1 128x256,
                                  2 192x192; -1 (default) = the tile_id's own shape when tile_id is given,
                                  else the shape whose workgroups, dealt out one per compute unit in
                                  rounds, leave the least output area in flight */
} tc_options;

typedef struct {
  int paper_class;             /* 0 (no contracted index), 1, 2, 31 (Class 3.1), 32 (Class 3.2) */
  tc_recipe recipe;            /* recipe the plan executes */
  int tile_id;                 /* tile configuration of the GEMM recipes, -1 otherwise */
  int swapped;                 /* 1 when A and B exchange roles inside the kernels */
  int copy_operand;            /* COPY_GEMM: 0 copies A, 1 copies B; -1 otherwise */
  int unit_a, unit_b, unit_c;  /* position of the stride-1 mode of A, B, C (-1: none) */
  int64_t M, N, K, L;          /* products of free-A, free-B, contracted, batch extents */
  int nM, nN, nK, nL;          /* modes per group after fusing contiguous modes */
  double flops;                /* 2 M N K L */
  double bytes;                /* 8 (|A| + |B| + |C|): algorithmic traffic with beta = 0 */
  size_t workspace_bytes;      /* device workspace tc_execute needs (0 = none) */
  tc_precision precision;
  int split_slices;            /* digits per input (split precision), 0 otherwise */
  int kernel;                  /* kernel family: 0 MFMA GEMM, 1 lanes over outputs, 2 lanes over k,
                                  3 batched small slabs, 4 split precision (digits or residues) */
  int k_split;                 /* MFMA GEMM: segments of the contracted range (1 = none) */
  int picked_candidate;        /* candidate chosen by the MLP or the tune cache, -1: rules */
  int split_bits;              /* split precision: bits each input keeps relative to its row's power-of-two
                                  scale (every input is exact to 2^-split_bits of that scale), 0 otherwise */
  int copy_fed;                /* nonzero: the GEMM runs the kernel fed by direct global-to-LDS copies
                                  (operand layouts allow 16-byte pairs; taken when A and B, after any
                                  COPY step, are 16-byte aligned), with output tiles of 256x128 (1),
                                  128x256 (2) or 192x192 (3); 0: the gathering GEMM kernel or another */
} tc_plan_info;

/* Fills *opt with the defaults listed in tc_options. */
void tc_options_default(tc_options* opt);

/* Host-only analysis: validates and classifies the contraction and reports
 * the plan it would build (Sec. 3.1 requirements, Sec. 3.2 classes and
 * recipes), without touching any GPU.  Arguments as for tc_plan_create;
 * info must be non-null. */
tc_status tc_analyze(int rank_a, const int64_t* ext_a, const int64_t* str_a, const int32_t* lab_a,
                     int rank_b, const int64_t* ext_b, const int64_t* str_b, const int32_t* lab_b,
                     int rank_c, const int64_t* ext_c, const int64_t* str_c, const int32_t* lab_c,
                     const tc_options* opt, tc_plan_info* info);

/* Host only.  Layout advice of Sec. 3.3 (and the closing remarks of Sec. 5):
 * storage orders under which the contraction runs as one direct GEMM, with no
 * copy.  Arguments as tc_analyze, except that any stride array may be NULL
 * (the tensor is then packed column-major in the listed order); strides
 * matter only for fixed tensors.  fixed: bit 0 keeps A's storage as given,
 * bit 1 B's, bit 2 C's.  order_x (rank_x entries, caller-owned) receives the
 * suggested storage order: order_x[j] is the listed mode of X stored j-th,
 * j = 0 at stride 1 (for a fixed tensor, its modes by ascending stride).  A
 * free tensor is stored as A [free-A, contracted, batch], B [contracted,
 * free-B, batch] (B [free-B, contracted, batch] when A is fixed with a
 * contracted or batch index at stride 1), C [free-A, free-B, batch]; each
 * index group keeps one order in all tensors that hold it, taken from a fixed
 * tensor when there is one.  When both inputs have a free index, A or B is not
 * fixed and no fixed input has a batch index at stride 1, the suggested
 * layout is Class 3.2 and each index group of a free tensor is contiguous
 * (with nothing fixed, every group fuses into one mode).  info (may be NULL)
 * receives the analysis of the suggested layout: free tensors packed
 * column-major in their suggested order, fixed tensors with their own
 * strides.  Errors: those of tc_analyze; TC_ERR_INVALID_ARG for a null order
 * array or fixed outside 0..7.  Nothing is written to the order arrays on
 * error. */
tc_status tc_suggest_layout(int rank_a, const int64_t* ext_a, const int64_t* str_a, const int32_t* lab_a,
                            int rank_b, const int64_t* ext_b, const int64_t* str_b, const int32_t* lab_b,
                            int rank_c, const int64_t* ext_c, const int64_t* str_c, const int32_t* lab_c,
                            int fixed, int32_t* order_a, int32_t* order_b, int32_t* order_c,
                            tc_plan_info* info);

/* Builds an immutable plan for C <- alpha * sum A*B + beta * C (Sec. 2.3;
 * classification and recipe as in Sec. 3.2).  The plan copies the host
 * arrays, builds its index-offset tables and uploads them to the current
 * device.  opt may be NULL for defaults.  On success *out holds a plan the
 * caller releases with tc_plan_destroy. */
tc_status tc_plan_create(tc_plan_t* out,
                         int rank_a, const int64_t* ext_a, const int64_t* str_a, const int32_t* lab_a,
                         int rank_b, const int64_t* ext_b, const int64_t* str_b, const int32_t* lab_b,
                         int rank_c, const int64_t* ext_c, const int64_t* str_c, const int32_t* lab_c,
                         const tc_options* opt);

/* Copies the plan's description into *info: the paper's class of the
 * contraction (Sec. 3.2), the recipe taken (Sec. 3.2; the slicing it stands
 * for, Sec. 2.4 and 3.1), the extents of the fused index groups and the
 * algorithmic work, flops = 2 M N K L (Sec. 2.1's operation count of GEMM,
 * carried over to the fused groups).  Errors: TC_ERR_INVALID_ARG for a null
 * plan or info; nothing else. */
tc_status tc_plan_query(tc_plan_t plan, tc_plan_info* info);

/* Enqueues C <- alpha * sum A*B + beta * C (the contraction of Sec. 2.3, with
 * alpha and beta as in the BLAS GEMM of Sec. 2.1) on `stream`.  A, B: device
 * pointers to the first element (index 0 in every mode) of each input, laid
 * out by the extents and strides the plan was built with; C: device pointer
 * to the output, read only when beta != 0 (BLAS convention, so NaNs in C are
 * harmless with beta = 0).  An empty contracted range gives C = beta * C; an
 * empty output writes nothing.  workspace: device memory of at least
 * info.workspace_bytes bytes (may be NULL when that is 0), caller-owned; it
 * must not be used concurrently by another call.  A plan may run on several
 * streams at once with distinct workspaces.  Errors (nothing is enqueued):
 * TC_ERR_INVALID_ARG for a null plan, null A, B or C where they are read or
 * written, or a current device other than the plan's; TC_ERR_WORKSPACE for a
 * workspace below info.workspace_bytes; TC_ERR_HIP when a launch fails. */
tc_status tc_execute(tc_plan_t plan, const double* A, const double* B, double* C,
                     double alpha, double beta, void* workspace, size_t workspace_bytes,
                     void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): tc_execute with the
 * workspace taken from a fixed device array of TC_NOALLOC_SCRATCH_BYTES bytes
 * (64 MiB) that the library holds on each device it runs on, from its load
 * until the process ends.  The caller passes the plan, inputs, output, alpha,
 * beta and stream exactly as for tc_execute; nothing is allocated or freed.
 * Every call on one device shares that device's array and leaves its
 * contents behind, so calls on one device whose executions overlap in time
 * (several streams or host threads) race: serialise them.  Errors: those of
 * tc_execute; TC_ERR_WORKSPACE, with nothing enqueued, for a plan whose
 * info.workspace_bytes exceeds TC_NOALLOC_SCRATCH_BYTES; TC_ERR_HIP when the
 * array's device address cannot be looked up (first call on a device). */
#define TC_NOALLOC_SCRATCH_BYTES (64ll << 20)
tc_status tc_execute_noalloc(tc_plan_t plan, const double* A, const double* B, double* C,
                             double alpha, double beta, void* stream);

/* Releases a plan from tc_plan_create and its device offset tables (Sec. 2.4:
 * the slicing loops the tables stand for).  NULL is accepted (TC_OK).  The
 * caller must make sure no enqueued tc_execute of the plan is still pending:
 * the tables are freed at once. */
tc_status tc_plan_destroy(tc_plan_t plan);

/* Storage reordering (the copy of Sec. 3.1 F1 / the COPY of COPY+GEMM):
 * Y[sum_i idx_i * str_y[i]] = X[sum_i idx_i * str_x[i]] for every
 * multi-index idx over ext[0..rank).  X and Y are device pointers; Y's
 * addresses must not overlap (checked like C's).  Asynchronous on stream. */
tc_status tc_permute(int rank, const int64_t* ext, const int64_t* str_x, const int64_t* str_y,
                     const double* X, double* Y, void* stream);

/* Batches: many independent FP64 contractions of any shapes run by one
 * persistent kernel launch (an addition to the paper; its general-relativity
 * workload, Sec. 4.2, is the model of the batch-dominated entries).
 * tc_batch_create takes n >= 1 plans on the current device; the batch copies
 * what it needs, so the plans may be destroyed afterwards.  Each contraction
 * runs as FP64 MFMA GEMM tiles, or, when its batch indices dominate, as slabs
 * of batch indices; split precision plans are rejected (TC_ERR_UNSUPPORTED).
 * tc_batch_execute runs C_i <- alpha_i * sum A_i*B_i + beta_i * C_i for every
 * i: A, B, C, alpha and beta are HOST arrays of n entries (device pointers and
 * scalars).  The workspace (device, tc_batch_workspace bytes) holds the
 * pointers and the task counter.  By default the launch sequence is captured
 * once in a hipGraph and replayed; executions of one batch must not overlap
 * (the call waits until the previous execution has read its inputs). */
tc_status tc_batch_create(tc_batch_t* out, int n, const tc_plan_t* plans);
tc_status tc_batch_workspace(tc_batch_t batch, size_t* bytes);
tc_status tc_batch_execute(tc_batch_t batch, const double* const* A, const double* const* B,
                           double* const* C, const double* alpha, const double* beta,
                           void* workspace, size_t workspace_bytes, void* stream);
/* tile_config: -1 keeps the current one, else 0..5 (GEMM tiles rows x columns
 * x depth: 64x64x16, 32x32x16, 32x32x64, 64x64x32, 32x32x128, 64x64x64);
 * use_graph: 0 launches eagerly, 1 replays a hipGraph. */
tc_status tc_batch_set_options(tc_batch_t batch, int tile_config, int use_graph);
/* ntasks: the tasks of the persistent engines plus the workgroups of the slab
 * contractions large enough to run as launches of their own. */
tc_status tc_batch_query(tc_batch_t batch, int64_t* ntasks, int* tile_config, int* use_graph);
/* Autotuner: times every tile configuration on the given buffers (C is
 * overwritten; eager launches, median of three) and keeps the fastest, which
 * it returns in *best_config with its time in *best_ms (either may be NULL). */
tc_status tc_batch_autotune(tc_batch_t batch, const double* const* A, const double* const* B,
                            double* const* C, const double* alpha, const double* beta,
                            void* workspace, size_t workspace_bytes, void* stream,
                            int* best_config, double* best_ms);
tc_status tc_batch_destroy(tc_batch_t batch);

/* ---------------------------------------------------------------------------
 * Learned recipe/tile picker (an addition to the paper; the paper's class
 * rules, Sec. 3.2, remain the fallback and numerical results never depend on
 * the choice).  A contraction is described by TC_PICKER_FEATURES features of
 * its layout; an MLP predicts the log execution time of each of the
 * TC_PICKER_CANDIDATES (recipe, tile) candidates, and the plan takes the
 * fastest.  The MLP is trained on the GPU by the tc_mlp_* kernels.
 * ------------------------------------------------------------------------- */
#define TC_PICKER_FEATURES 32
#define TC_PICKER_CANDIDATES 15

/* Candidate `index` (0 .. TC_PICKER_CANDIDATES-1): recipe and GEMM tile id
 * (-1 for the memory-bound recipes).  The last candidate is TC_RECIPE_AUTO:
 * the rules' own plan, whatever kernel it takes. */
tc_status tc_picker_candidate(int index, tc_recipe* recipe, int* tile_id);

/* Host only: the features of a contraction (arguments as tc_analyze; feat
 * receives TC_PICKER_FEATURES floats) and the candidate the rules would take
 * (*rule_candidate, -1 when the rules pick a kernel outside the table). */
tc_status tc_picker_features(int rank_a, const int64_t* ext_a, const int64_t* str_a, const int32_t* lab_a,
                             int rank_b, const int64_t* ext_b, const int64_t* str_b, const int32_t* lab_b,
                             int rank_c, const int64_t* ext_c, const int64_t* str_c, const int32_t* lab_c,
                             float* feat, int* rule_candidate);

/* Installs a trained model for TC_PICKER_MLP plans of this process (copies
 * the host arrays; creates the network on the current device): params in the
 * tc_mlp layout, n_in must be TC_PICKER_FEATURES and n_out
 * TC_PICKER_CANDIDATES; mean/std normalise the features.  Replaces any
 * previous model.  tc_picker_uninstall returns to the rules. */
tc_status tc_picker_install(const float* params, int64_t n_params, int n_in, int hidden, int n_out,
                            const float* feat_mean, const float* feat_std);
tc_status tc_picker_uninstall(void);

/* Autotuner for one shape: times every candidate on the given buffers (C is
 * overwritten with beta = 0; after a warm-up, the median of three timed runs,
 * each of enough back-to-back executions to last about 0.2 ms; the library
 * allocates the candidates' workspaces itself), records the fastest in the
 * process-wide tune cache used by TC_PICKER_TUNED plans of the same shape, and
 * returns it.  candidate_ms (NULL, or TC_PICKER_CANDIDATES doubles) receives
 * each candidate's time per execution in milliseconds, -1 for a candidate the
 * shape cannot take. */
tc_status tc_plan_autotune(tc_plan_t plan, const double* A, const double* B, double* C, void* stream,
                           int* best_candidate, double* best_ms, double* candidate_ms);
/* The tune cache as a text file (one line per shape: library version, device
 * architecture, shape signature, candidate); entries of another version or
 * architecture are ignored on load. */
tc_status tc_tune_cache_save(const char* path);
tc_status tc_tune_cache_load(const char* path);

/* The MLP itself: n_in -> hidden -> hidden -> n_out, ReLU, FP32, weights
 * row-major W[i][o] followed by biases, layer by layer.  All X/T/M/Y/grads/loss
 * pointers are DEVICE pointers (row-major batch x width); batch <= max_batch.
 * loss_grad: forward, masked mean-squared error sum(M (Y-T)^2) / sum(M) into
 * *loss, and its gradient into grads (either may be NULL).  train_step: the
 * same followed by one Adam step (beta 0.9, 0.999, eps 1e-8). */
typedef struct tc_mlp_s* tc_mlp_t;
tc_status tc_mlp_create(tc_mlp_t* out, int n_in, int hidden, int n_out, int max_batch);
tc_status tc_mlp_num_params(tc_mlp_t mlp, int64_t* n);
tc_status tc_mlp_set_params(tc_mlp_t mlp, const float* host_params);
tc_status tc_mlp_get_params(tc_mlp_t mlp, float* host_params);
tc_status tc_mlp_forward(tc_mlp_t mlp, const float* X, float* Y, int batch, void* stream);
tc_status tc_mlp_loss_grad(tc_mlp_t mlp, const float* X, const float* T, const float* M, int batch, float* grads,
                           float* loss, void* stream);
tc_status tc_mlp_train_step(tc_mlp_t mlp, const float* X, const float* T, const float* M, int batch, float lr,
                            float* loss, void* stream);
tc_status tc_mlp_destroy(tc_mlp_t mlp);

const char* tc_status_string(tc_status s);
const char* tc_last_error(void);
const char* tc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TC_H_ */
