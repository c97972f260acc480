"""Python binding of libtc, the MI355X tensor-contraction library.

Argument marshalling only: every step of a contraction runs inside libtc
(host planner in C++, kernels in HIP).  PyTorch supplies device memory and
streams.  The functions named ``tc_*`` map one-to-one onto the C ABI of
include/tc.h; ``Plan`` and ``contract`` are thin conveniences over them.

The library is loaded from paper_1307_2100_amd/_lib/libtc.so, built by
``paper_1307_2100_amd.build.build()``; importing this module without it
raises ImportError (there is no fallback path).
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TC_LIBRARY names another build of the same sources (the host-sanitized one
# that tests/run_sanitized.py loads); by default the in-tree libtc.so.
LIB_PATH = os.environ.get("TC_LIBRARY") or os.path.join(HERE, "_lib", "libtc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libtc.so is not built (%s); run paper_1307_2100_amd.build.build()" % LIB_PATH)

# PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Loading torch
# first makes libtc bind to that same runtime instead of mapping a second
# copy from /opt/rocm, which would not see the GPU that torch already opened.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

TC_MAX_RANK = 16

# tc_status
TC_OK = 0
STATUS_NAMES = ["TC_OK", "TC_ERR_INVALID_ARG", "TC_ERR_LABEL", "TC_ERR_EXTENT_MISMATCH",
                "TC_ERR_OUTPUT_OVERLAP", "TC_ERR_RANK", "TC_ERR_WORKSPACE", "TC_ERR_UNSUPPORTED",
                "TC_ERR_HIP", "TC_ERR_NOMEM"]
for _i, _n in enumerate(STATUS_NAMES):
    globals()[_n] = _i

# tc_precision
TC_PREC_F64, TC_PREC_F64_SPLIT_BF16, TC_PREC_F64_SPLIT_FP8, TC_PREC_F64_CRT_INT8 = 0, 1, 2, 3
PRECISIONS = {"f64": 0, "split_bf16": 1, "split_fp8": 2, "crt_int8": 3}
# residue-GEMM configurations of TC_PREC_F64_CRT_INT8 plans (tile_id 0 .. CRT_NUM_TILES-1)
CRT_NUM_TILES = 12
# tc_recipe
TC_RECIPE_AUTO, TC_RECIPE_GEMM, TC_RECIPE_COPY_GEMM, TC_RECIPE_GEMV, TC_RECIPE_GER, TC_RECIPE_DOT = range(6)
RECIPES = {"auto": 0, "gemm": 1, "copy_gemm": 2, "gemv": 3, "ger": 4, "dot": 5}
RECIPE_NAMES = {v: k for k, v in RECIPES.items()}
KERNEL_NAMES = {0: "mfma_gemm", 1: "lanes_over_outputs", 2: "lanes_over_k", 3: "batched_small", 4: "split"}
# GEMM tile configurations compiled into libtc (ids 0 .. NUM_TILES-1)
NUM_TILES = 20
# tc_picker
TC_PICKER_RULES, TC_PICKER_MLP, TC_PICKER_TUNED = 0, 1, 2
PICKERS = {"rules": 0, "mlp": 1, "tuned": 2}


class tc_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("recipe", ctypes.c_int), ("picker", ctypes.c_int),
                ("split_slices", ctypes.c_int), ("tile_id", ctypes.c_int), ("copy_tile", ctypes.c_int)]


class tc_plan_info(ctypes.Structure):
    _fields_ = [("paper_class", ctypes.c_int), ("recipe", ctypes.c_int), ("tile_id", ctypes.c_int),
                ("swapped", ctypes.c_int), ("copy_operand", ctypes.c_int),
                ("unit_a", ctypes.c_int), ("unit_b", ctypes.c_int), ("unit_c", ctypes.c_int),
                ("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64), ("L", ctypes.c_int64),
                ("nM", ctypes.c_int), ("nN", ctypes.c_int), ("nK", ctypes.c_int), ("nL", ctypes.c_int),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
                ("workspace_bytes", ctypes.c_size_t), ("precision", ctypes.c_int),
                ("split_slices", ctypes.c_int), ("kernel", ctypes.c_int),
                ("k_split", ctypes.c_int), ("picked_candidate", ctypes.c_int), ("split_bits", ctypes.c_int),
                ("copy_fed", ctypes.c_int)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["recipe_name"] = RECIPE_NAMES.get(self.recipe, "?")
        d["kernel_name"] = KERNEL_NAMES.get(self.kernel, "?")
        return d


_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)
_DESC = [ctypes.c_int, _I64P, _I64P, _I32P]

_lib.tc_options_default.argtypes = [ctypes.POINTER(tc_options)]
_lib.tc_options_default.restype = None
_lib.tc_analyze.argtypes = _DESC * 3 + [ctypes.POINTER(tc_options), ctypes.POINTER(tc_plan_info)]
_lib.tc_analyze.restype = ctypes.c_int
_lib.tc_suggest_layout.argtypes = _DESC * 3 + [ctypes.c_int, _I32P, _I32P, _I32P, ctypes.POINTER(tc_plan_info)]
_lib.tc_suggest_layout.restype = ctypes.c_int
_lib.tc_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p)] + _DESC * 3 + [ctypes.POINTER(tc_options)]
_lib.tc_plan_create.restype = ctypes.c_int
_lib.tc_plan_query.argtypes = [ctypes.c_void_p, ctypes.POINTER(tc_plan_info)]
_lib.tc_plan_query.restype = ctypes.c_int
_lib.tc_execute.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
_lib.tc_execute.restype = ctypes.c_int
_lib.tc_execute_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
_lib.tc_execute_noalloc.restype = ctypes.c_int
_lib.tc_plan_destroy.argtypes = [ctypes.c_void_p]
_lib.tc_plan_destroy.restype = ctypes.c_int
_lib.tc_permute.argtypes = [ctypes.c_int, _I64P, _I64P, _I64P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
_lib.tc_permute.restype = ctypes.c_int
_lib.tc_batch_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
_lib.tc_batch_create.restype = ctypes.c_int
_lib.tc_batch_workspace.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]
_lib.tc_batch_workspace.restype = ctypes.c_int
_lib.tc_batch_execute.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                  ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p]
_lib.tc_batch_execute.restype = ctypes.c_int
_lib.tc_batch_set_options.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
_lib.tc_batch_set_options.restype = ctypes.c_int
_lib.tc_batch_query.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]
_lib.tc_batch_query.restype = ctypes.c_int
_lib.tc_batch_autotune.argtypes = _lib.tc_batch_execute.argtypes + [ctypes.POINTER(ctypes.c_int),
                                                                    ctypes.POINTER(ctypes.c_double)]
_lib.tc_batch_autotune.restype = ctypes.c_int
_lib.tc_batch_destroy.argtypes = [ctypes.c_void_p]
_lib.tc_batch_destroy.restype = ctypes.c_int
_FP = ctypes.POINTER(ctypes.c_float)
_lib.tc_picker_candidate.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.tc_picker_candidate.restype = ctypes.c_int
_lib.tc_picker_features.argtypes = _DESC * 3 + [_FP, ctypes.POINTER(ctypes.c_int)]
_lib.tc_picker_features.restype = ctypes.c_int
_lib.tc_picker_install.argtypes = [_FP, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _FP, _FP]
_lib.tc_picker_install.restype = ctypes.c_int
_lib.tc_picker_uninstall.argtypes = []
_lib.tc_picker_uninstall.restype = ctypes.c_int
_lib.tc_plan_autotune.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
_lib.tc_plan_autotune.restype = ctypes.c_int
_lib.tc_tune_cache_save.argtypes = [ctypes.c_char_p]
_lib.tc_tune_cache_save.restype = ctypes.c_int
_lib.tc_tune_cache_load.argtypes = [ctypes.c_char_p]
_lib.tc_tune_cache_load.restype = ctypes.c_int
_lib.tc_mlp_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int]
_lib.tc_mlp_create.restype = ctypes.c_int
_lib.tc_mlp_num_params.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
_lib.tc_mlp_num_params.restype = ctypes.c_int
_lib.tc_mlp_set_params.argtypes = [ctypes.c_void_p, _FP]
_lib.tc_mlp_set_params.restype = ctypes.c_int
_lib.tc_mlp_get_params.argtypes = [ctypes.c_void_p, _FP]
_lib.tc_mlp_get_params.restype = ctypes.c_int
_lib.tc_mlp_forward.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
_lib.tc_mlp_forward.restype = ctypes.c_int
_lib.tc_mlp_loss_grad.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
_lib.tc_mlp_loss_grad.restype = ctypes.c_int
_lib.tc_mlp_train_step.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p]
_lib.tc_mlp_train_step.restype = ctypes.c_int
_lib.tc_mlp_destroy.argtypes = [ctypes.c_void_p]
_lib.tc_mlp_destroy.restype = ctypes.c_int
_lib.tc_status_string.argtypes = [ctypes.c_int]
_lib.tc_status_string.restype = ctypes.c_char_p
_lib.tc_last_error.restype = ctypes.c_char_p
_lib.tc_version.restype = ctypes.c_char_p

EXPORTED = ["tc_options_default", "tc_analyze", "tc_suggest_layout", "tc_plan_create", "tc_plan_query", "tc_execute",
            "tc_execute_noalloc",
            "tc_plan_destroy", "tc_permute", "tc_batch_create", "tc_batch_workspace", "tc_batch_execute",
            "tc_batch_set_options", "tc_batch_query", "tc_batch_autotune", "tc_batch_destroy",
            "tc_picker_candidate", "tc_picker_features", "tc_picker_install", "tc_picker_uninstall",
            "tc_plan_autotune", "tc_tune_cache_save", "tc_tune_cache_load", "tc_mlp_create", "tc_mlp_num_params",
            "tc_mlp_set_params", "tc_mlp_get_params", "tc_mlp_forward", "tc_mlp_loss_grad", "tc_mlp_train_step",
            "tc_mlp_destroy", "tc_status_string", "tc_last_error", "tc_version"]

PICKER_FEATURES = 32
PICKER_CANDIDATES = 15


class TCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status, msg))
        self.status = status


def _check(status):
    if status != TC_OK:
        raise TCError(status, _lib.tc_last_error().decode())


def library_path():
    return LIB_PATH


# ---------------------------------------------------------------- descriptors
def labels_of(spec):
    """Labels as int32 codes; a string gives one label per character."""
    if isinstance(spec, str):
        return [ord(c) for c in spec]
    return [int(x) for x in spec]


class Desc:
    """(extents, element strides, labels) of one tensor, as ctypes arrays."""

    def __init__(self, extents, strides, labels):
        labels = labels_of(labels)
        if not (len(extents) == len(strides) == len(labels)):
            raise ValueError("extents, strides and labels differ in length")
        self.rank = len(labels)
        n = max(1, self.rank)
        self.ext = (ctypes.c_int64 * n)(*[int(e) for e in extents])
        self.str = (ctypes.c_int64 * n)(*[int(s) for s in strides])
        self.lab = (ctypes.c_int32 * n)(*labels)

    def args(self):
        return [self.rank, self.ext, self.str, self.lab]

    @classmethod
    def of_tensor(cls, t, labels):
        return cls(list(t.shape), list(t.stride()), labels)


# output tiles of the copy-fed FP64 kernel (tc_options.copy_tile, tc_plan_info.copy_fed - 1)
COPY_TILES = {"256x128": 0, "128x256": 1, "192x192": 2}


def make_options(precision="f64", recipe="auto", picker=0, split_slices=0, tile_id=-1, copy_tile=-1):
    o = tc_options()
    _lib.tc_options_default(ctypes.byref(o))
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.recipe = RECIPES[recipe] if isinstance(recipe, str) else int(recipe)
    o.picker = PICKERS[picker] if isinstance(picker, str) else int(picker)
    o.split_slices = int(split_slices)
    o.tile_id = int(tile_id)
    o.copy_tile = COPY_TILES[copy_tile] if isinstance(copy_tile, str) else int(copy_tile)
    return o


# ------------------------------------------------------------ C ABI wrappers
def tc_options_default():
    o = tc_options()
    _lib.tc_options_default(ctypes.byref(o))
    return o


def tc_analyze(dA, dB, dC, options=None):
    info = tc_plan_info()
    _check(_lib.tc_analyze(*dA.args(), *dB.args(), *dC.args(),
                           ctypes.byref(options) if options is not None else None, ctypes.byref(info)))
    return info


def tc_suggest_layout(dA, dB, dC, fixed=0):
    """Storage orders (one list of listed-mode indices per tensor, stride 1
    first) and the analysis of the suggested layout; `fixed` as in the C ABI
    (bit 0 A, bit 1 B, bit 2 C)."""
    info = tc_plan_info()
    orders = [(ctypes.c_int32 * max(1, d.rank))() for d in (dA, dB, dC)]
    _check(_lib.tc_suggest_layout(*dA.args(), *dB.args(), *dC.args(), int(fixed), *orders, ctypes.byref(info)))
    return [list(o)[:d.rank] for o, d in zip(orders, (dA, dB, dC))], info


def tc_plan_create(dA, dB, dC, options=None):
    h = ctypes.c_void_p()
    _check(_lib.tc_plan_create(ctypes.byref(h), *dA.args(), *dB.args(), *dC.args(),
                               ctypes.byref(options) if options is not None else None))
    return h


def tc_plan_query(plan):
    info = tc_plan_info()
    _check(_lib.tc_plan_query(plan, ctypes.byref(info)))
    return info


def tc_execute(plan, A_ptr, B_ptr, C_ptr, alpha, beta, ws_ptr, ws_bytes, stream):
    _check(_lib.tc_execute(plan, A_ptr, B_ptr, C_ptr, float(alpha), float(beta), ws_ptr, int(ws_bytes), stream))


def tc_execute_noalloc(plan, A_ptr, B_ptr, C_ptr, alpha, beta, stream):
    _check(_lib.tc_execute_noalloc(plan, A_ptr, B_ptr, C_ptr, float(alpha), float(beta), stream))


# size of the library's fixed device workspace used by tc_execute_noalloc
NOALLOC_SCRATCH_BYTES = 64 << 20


def tc_plan_destroy(plan):
    _check(_lib.tc_plan_destroy(plan))


def tc_permute(extents, strides_x, strides_y, X_ptr, Y_ptr, stream):
    n = max(1, len(extents))
    e = (ctypes.c_int64 * n)(*[int(v) for v in extents])
    sx = (ctypes.c_int64 * n)(*[int(v) for v in strides_x])
    sy = (ctypes.c_int64 * n)(*[int(v) for v in strides_y])
    _check(_lib.tc_permute(len(extents), e, sx, sy, X_ptr, Y_ptr, stream))


def tc_picker_candidate(index):
    """(recipe, tile_id) of picker candidate `index`."""
    r = ctypes.c_int()
    t = ctypes.c_int()
    _check(_lib.tc_picker_candidate(int(index), ctypes.byref(r), ctypes.byref(t)))
    return r.value, t.value


def tc_picker_features(dA, dB, dC):
    """(features as a list of PICKER_FEATURES floats, the rules' candidate)."""
    f = (ctypes.c_float * PICKER_FEATURES)()
    rc = ctypes.c_int()
    _check(_lib.tc_picker_features(*dA.args(), *dB.args(), *dC.args(), f, ctypes.byref(rc)))
    return list(f), rc.value


def _farr(values):
    values = [float(v) for v in values]
    return (ctypes.c_float * max(1, len(values)))(*values)


def tc_picker_install(params, hidden, mean, std):
    _check(_lib.tc_picker_install(_farr(params), len(params), PICKER_FEATURES, int(hidden), PICKER_CANDIDATES,
                                  _farr(mean), _farr(std)))


def tc_picker_uninstall():
    _check(_lib.tc_picker_uninstall())


def tc_tune_cache_save(path):
    _check(_lib.tc_tune_cache_save(os.fsencode(path)))


def tc_tune_cache_load(path):
    _check(_lib.tc_tune_cache_load(os.fsencode(path)))


def tc_status_string(status):
    return _lib.tc_status_string(int(status)).decode()


def tc_last_error():
    return _lib.tc_last_error().decode()


def tc_version():
    return _lib.tc_version().decode()


# ---------------------------------------------------------------- torch side
def _torch():
    import torch  # device memory and streams only
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _require_f64_cuda(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError("%s must be a float64 CUDA (HIP) tensor" % name)


class Plan:
    """A libtc plan for fixed extents, strides and labels of A, B and C."""

    def __init__(self, dA, dB, dC, precision="f64", recipe="auto", tile_id=-1, split_slices=0, picker=0,
                 copy_tile=-1):
        self.options = make_options(precision, recipe, picker, split_slices, tile_id, copy_tile)
        self.handle = tc_plan_create(dA, dB, dC, self.options)
        self.info = tc_plan_query(self.handle)
        self._ws = None

    @classmethod
    def for_tensors(cls, A, labA, B, labB, C, labC, **kw):
        return cls(Desc.of_tensor(A, labA), Desc.of_tensor(B, labB), Desc.of_tensor(C, labC), **kw)

    def workspace(self, device=None):
        nbytes = self.info.workspace_bytes
        if nbytes == 0:
            return None
        torch = _torch()
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")
        return self._ws

    def execute(self, A, B, C, alpha=1.0, beta=0.0, stream=None, workspace=None):
        _require_f64_cuda(A, "A")
        _require_f64_cuda(B, "B")
        _require_f64_cuda(C, "C")
        ws = workspace if workspace is not None else self.workspace(C.device)
        wptr = ctypes.c_void_p(ws.data_ptr()) if ws is not None else None
        wbytes = ws.numel() * ws.element_size() if ws is not None else 0
        tc_execute(self.handle, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                   ctypes.c_void_p(C.data_ptr()), alpha, beta, wptr, wbytes, _stream_handle(stream))
        return C

    def execute_noalloc(self, A, B, C, alpha=1.0, beta=0.0, stream=None):
        """tc_execute_noalloc: like execute, with the library's fixed device
        workspace in place of an allocated one."""
        _require_f64_cuda(A, "A")
        _require_f64_cuda(B, "B")
        _require_f64_cuda(C, "C")
        tc_execute_noalloc(self.handle, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                           ctypes.c_void_p(C.data_ptr()), alpha, beta, _stream_handle(stream))
        return C

    def autotune(self, A, B, C, stream=None):
        """Times every picker candidate on these buffers (C is overwritten);
        records the fastest in the tune cache; returns (candidate, ms, list of
        per-candidate ms with -1 where a candidate cannot run)."""
        _require_f64_cuda(A, "A")
        _require_f64_cuda(B, "B")
        _require_f64_cuda(C, "C")
        best = ctypes.c_int()
        ms = ctypes.c_double()
        per = (ctypes.c_double * PICKER_CANDIDATES)()
        _check(_lib.tc_plan_autotune(self.handle, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                     ctypes.c_void_p(C.data_ptr()), _stream_handle(stream), ctypes.byref(best),
                                     ctypes.byref(ms), per))
        return best.value, ms.value, list(per)

    def close(self):
        if getattr(self, "handle", None) is not None:
            tc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def output_shape(A, labA, B, labB, labC):
    ext = {}
    for l, e in zip(labels_of(labA), A.shape):
        ext[l] = e
    for l, e in zip(labels_of(labB), B.shape):
        ext[l] = e
    return [ext[l] for l in labels_of(labC)]


def empty_colmajor(shape, device="cuda"):
    """An uninitialised FP64 tensor stored column-major (first index stride 1)."""
    torch = _torch()
    if len(shape) == 0:
        return torch.empty((), dtype=torch.float64, device=device)
    return torch.empty(list(reversed(shape)), dtype=torch.float64, device=device).permute(
        *reversed(range(len(shape))))


def suggest_layout(labA, extA, labB, extB, labC, extC, fixed="", strides=None):
    """The layout advice of the C ABI's tc_suggest_layout on label lists.

    Returns ({"A": labels, "B": labels, "C": labels}, info): each tensor's
    labels in the suggested storage order, stride-1 label first (strings when
    the labels were given as strings).  `fixed` names the tensors kept as
    given ("A", "BC", ...); `strides` optionally maps a fixed tensor's name to
    its element strides (default: packed column-major in the listed order)."""
    strides = strides or {}
    specs = {"A": (labA, extA), "B": (labB, extB), "C": (labC, extC)}
    descs = []
    for name, (lab, ext) in specs.items():
        ext = [int(e) for e in ext]
        st = strides.get(name)
        if st is None:
            st, acc = [], 1
            for e in ext:
                st.append(acc)
                acc *= max(e, 1)
        descs.append(Desc(ext, st, lab))
    mask = sum(1 << i for i, name in enumerate("ABC") if name in fixed.upper())
    orders, info = tc_suggest_layout(*descs, fixed=mask)
    out = {}
    for (name, (lab, _)), order in zip(specs.items(), orders):
        seq = [lab[i] for i in order]
        out[name] = "".join(seq) if isinstance(lab, str) else seq
    return out, info


def contract(A, labA, B, labB, labC, C=None, alpha=1.0, beta=0.0, **plan_kw):
    """C <- alpha * sum A*B + beta * C on the GPU (C allocated column-major when None)."""
    if C is None:
        C = empty_colmajor(output_shape(A, labA, B, labB, labC), device=A.device)
        beta = 0.0
    plan = Plan.for_tensors(A, labA, B, labB, C, labC, **plan_kw)
    try:
        plan.execute(A, B, C, alpha, beta)
    finally:
        # the plan's offset tables and workspace must outlive the kernels
        _torch().cuda.current_stream().synchronize()
        plan.close()
    return C


def permute(X, strides_out, Y):
    """Y[sum idx*strides_out] = X[idx] on the GPU (Y a flat FP64 CUDA tensor)."""
    _require_f64_cuda(X, "X")
    _require_f64_cuda(Y, "Y")
    tc_permute(list(X.shape), list(X.stride()), list(strides_out), ctypes.c_void_p(X.data_ptr()),
               ctypes.c_void_p(Y.data_ptr()), _stream_handle())
    return Y


# ------------------------------------------------------------------- batches
class Batch:
    """A libtc batch: many contractions run by one persistent kernel launch."""

    def __init__(self, plans):
        self.n = len(plans)
        arr = (ctypes.c_void_p * self.n)(*[p.handle.value if isinstance(p, Plan) else p for p in plans])
        h = ctypes.c_void_p()
        _check(_lib.tc_batch_create(ctypes.byref(h), self.n, arr))
        self.handle = h
        nb = ctypes.c_size_t()
        _check(_lib.tc_batch_workspace(h, ctypes.byref(nb)))
        self.workspace_bytes = nb.value
        self._ws = None

    def workspace(self, device=None):
        torch = _torch()
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device or "cuda")
        return self._ws

    def _arrays(self, As, Bs, Cs, alphas, betas):
        n = self.n
        if not (len(As) == len(Bs) == len(Cs) == n):
            raise ValueError("need %d operand triples" % n)
        alphas = [1.0] * n if alphas is None else list(alphas)
        betas = [0.0] * n if betas is None else list(betas)
        a = (ctypes.c_void_p * n)(*[t.data_ptr() for t in As])
        b = (ctypes.c_void_p * n)(*[t.data_ptr() for t in Bs])
        c = (ctypes.c_void_p * n)(*[t.data_ptr() for t in Cs])
        al = (ctypes.c_double * n)(*alphas)
        be = (ctypes.c_double * n)(*betas)
        return a, b, c, al, be

    def execute(self, As, Bs, Cs, alphas=None, betas=None, stream=None):
        a, b, c, al, be = self._arrays(As, Bs, Cs, alphas, betas)
        ws = self.workspace(Cs[0].device)
        _check(_lib.tc_batch_execute(self.handle, a, b, c, al, be, ctypes.c_void_p(ws.data_ptr()),
                                     self.workspace_bytes, _stream_handle(stream)))

    def bind(self, As, Bs, Cs, alphas=None, betas=None):
        """Marshals the operand pointers once; run() then executes the batch on
        them without rebuilding the argument arrays (a serving loop)."""
        self._bound = self._arrays(As, Bs, Cs, alphas, betas) + (self.workspace(Cs[0].device),)
        self._bound_tensors = (As, Bs, Cs)   # keep the buffers alive

    def run(self, stream=None):
        a, b, c, al, be, ws = self._bound
        _check(_lib.tc_batch_execute(self.handle, a, b, c, al, be, ctypes.c_void_p(ws.data_ptr()),
                                     self.workspace_bytes, _stream_handle(stream)))

    def autotune(self, As, Bs, Cs, alphas=None, betas=None, stream=None):
        a, b, c, al, be = self._arrays(As, Bs, Cs, alphas, betas)
        ws = self.workspace(Cs[0].device)
        best = ctypes.c_int()
        ms = ctypes.c_double()
        _check(_lib.tc_batch_autotune(self.handle, a, b, c, al, be, ctypes.c_void_p(ws.data_ptr()),
                                      self.workspace_bytes, _stream_handle(stream), ctypes.byref(best),
                                      ctypes.byref(ms)))
        return best.value, ms.value

    def set_options(self, tile_config=-1, use_graph=1):
        _check(_lib.tc_batch_set_options(self.handle, int(tile_config), int(use_graph)))

    def query(self):
        nt = ctypes.c_int64()
        cfg = ctypes.c_int()
        g = ctypes.c_int()
        _check(_lib.tc_batch_query(self.handle, ctypes.byref(nt), ctypes.byref(cfg), ctypes.byref(g)))
        return {"ntasks": nt.value, "tile_config": cfg.value, "use_graph": g.value}

    def close(self):
        if getattr(self, "handle", None) is not None:
            _lib.tc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ the MLP
class MLP:
    """The picker's network (n_in -> hidden -> hidden -> n_out, ReLU, FP32),
    trained and evaluated by libtc's HIP kernels.  Batches are float32 CUDA
    tensors, row-major (batch, width)."""

    def __init__(self, n_in, hidden, n_out, max_batch):
        h = ctypes.c_void_p()
        _check(_lib.tc_mlp_create(ctypes.byref(h), int(n_in), int(hidden), int(n_out), int(max_batch)))
        self.handle = h
        self.n_in, self.hidden, self.n_out, self.max_batch = n_in, hidden, n_out, max_batch
        n = ctypes.c_int64()
        _check(_lib.tc_mlp_num_params(h, ctypes.byref(n)))
        self.num_params = n.value

    def set_params(self, values):
        if len(values) != self.num_params:
            raise ValueError("need %d parameters" % self.num_params)
        _check(_lib.tc_mlp_set_params(self.handle, _farr(values)))

    def get_params(self):
        buf = (ctypes.c_float * self.num_params)()
        _check(_lib.tc_mlp_get_params(self.handle, buf))
        return list(buf)

    @staticmethod
    def _f32(t, name, cols):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32 \
                or not t.is_contiguous() or t.dim() != 2 or t.shape[1] != cols:
            raise TypeError("%s must be a contiguous float32 CUDA tensor of width %d" % (name, cols))
        return ctypes.c_void_p(t.data_ptr())

    def forward(self, X, stream=None):
        torch = _torch()
        x = self._f32(X, "X", self.n_in)
        Y = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device=X.device)
        _check(_lib.tc_mlp_forward(self.handle, x, ctypes.c_void_p(Y.data_ptr()), X.shape[0],
                                   _stream_handle(stream)))
        return Y

    def loss_grad(self, X, T, M, stream=None):
        """(loss, flat gradient) as CUDA tensors."""
        torch = _torch()
        args = (self._f32(X, "X", self.n_in), self._f32(T, "T", self.n_out), self._f32(M, "M", self.n_out))
        g = torch.empty(self.num_params, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        _check(_lib.tc_mlp_loss_grad(self.handle, *args, X.shape[0], ctypes.c_void_p(g.data_ptr()),
                                     ctypes.c_void_p(loss.data_ptr()), _stream_handle(stream)))
        return loss, g

    def train_step(self, X, T, M, lr, loss=None, stream=None):
        """One Adam step; the loss before the step goes to `loss` (a 1-element
        float32 CUDA tensor) when given."""
        args = (self._f32(X, "X", self.n_in), self._f32(T, "T", self.n_out), self._f32(M, "M", self.n_out))
        lp = ctypes.c_void_p(loss.data_ptr()) if loss is not None else None
        _check(_lib.tc_mlp_train_step(self.handle, *args, X.shape[0], float(lr), lp, _stream_handle(stream)))

    def close(self):
        if getattr(self, "handle", None) is not None:
            _lib.tc_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
