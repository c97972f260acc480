"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no contraction arithmetic: it only draws numbers and
describes workload shapes.  Every operand is generated on the host in FP64
from NumPy's PCG64 with seed 1307*1000 + workload*10 + operand, stored
column-major (first index stride 1, the storage the paper assumes in
Sec. 2.4), so that the oracle and the GPU see identical bits.
"""
import numpy as np

SEED_BASE = 1307 * 1000


def seed_for(workload: int, operand: int) -> int:
    return SEED_BASE + workload * 10 + operand


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# Large tensors are drawn in chunks of CHUNK consecutive entries (storage
# order), chunk c from PCG64(seed) advanced by c jumps of 2^127 draws (chunk 0
# from PCG64(seed) itself), so they can be filled by several threads and the
# values do not depend on the thread count.  A tensor of at most CHUNK
# entries is one plain PCG64(seed) stream.
CHUNK = 1 << 22


def _workers():
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _chunked(shape, seed, draw):
    """Column-major FP64 array of `shape`; draw(gen, out) fills one chunk."""
    n = int(np.prod(shape, dtype=np.int64))
    x = np.empty(n, dtype=np.float64)
    nchunks = (n + CHUNK - 1) // CHUNK

    def job(c):
        g = rng(seed) if c == 0 else np.random.Generator(np.random.PCG64(seed).jumped(c))
        draw(g, x[c * CHUNK:(c + 1) * CHUNK], c * CHUNK)

    if nchunks <= 1:
        if n:
            job(0)
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(job, range(nchunks)))
    return x.reshape(shape, order="F")


def uniform(shape, seed, lo=-1.0, hi=1.0):
    """Entries uniform in [lo, hi), column-major FP64."""
    def draw(g, out, start):
        out[:] = g.uniform(lo, hi, size=out.size)
    return _chunked(shape, seed, draw)


def integers(shape, seed, lo=-4, hi=4):
    """Integer-valued FP64 entries in [lo, hi]: every partial sum of products of
    such values is exact in FP64 (and in BF16/FP8 slices), so results computed
    in any order agree bit for bit."""
    def draw(g, out, start):
        out[:] = g.integers(lo, hi + 1, size=out.size)
    return _chunked(shape, seed, draw)


def scaled_normal(shape, seed, axis=-1, decades=3.0):
    """N(0,1) entries, each slice along `axis` scaled by 10^U(-decades, decades)
    (one factor drawn per slice, from its own stream: PCG64(seed) advanced by
    as many jumps as the tensor has chunks), column-major FP64."""
    shape = tuple(int(e) for e in shape)
    axis = axis % len(shape)
    n = int(np.prod(shape, dtype=np.int64))
    nchunks = max(1, (n + CHUNK - 1) // CHUNK)
    f = np.random.Generator(np.random.PCG64(seed).jumped(nchunks)).uniform(-decades, decades, size=shape[axis])
    f = 10.0 ** f
    inner = int(np.prod(shape[:axis], dtype=np.int64))   # entries per step of the axis (column-major)
    extent = shape[axis]

    def draw(g, out, start):
        g.standard_normal(out=out)
        if inner >= 1024:   # long runs of one factor: scale run by run
            q = start
            while q < start + out.size:
                stop = min(start + out.size, (q // inner + 1) * inner)
                out[q - start:stop - start] *= f[(q // inner) % extent]
                q = stop
        else:
            out *= f[(np.arange(start, start + out.size, dtype=np.int64) // inner) % extent]

    return _chunked(shape, seed, draw)


# Workloads: (labels A, labels B, labels C, extents per label).  Labels are
# single characters; extents map label -> size.
def workload_3d_matrix(n=64):
    """C[i,j,m] = sum_k A[i,k,m] B[k,j], all extents n."""
    return "ikm", "kj", "ijm", {"i": n, "k": n, "m": n, "j": n}


def workload_cc_a(v=128, o=32):
    """Coupled-cluster shape (a): C[a,b,i,j] = sum_{c,d} A[a,b,c,d] B[c,d,i,j]."""
    return "abcd", "cdij", "abij", {"a": v, "b": v, "c": v, "d": v, "i": o, "j": o}


def workload_cc_b(v=128, o=32):
    """Coupled-cluster shape (b): C[a,b,i,j] = sum_{k,c} A[a,k,i,c] B[k,b,c,j]."""
    return "akic", "kbcj", "abij", {"a": v, "b": v, "c": v, "i": o, "j": o, "k": o}


def workload_gr_r(points=(128, 128, 128), n=4):
    """Pointwise R[a,b] = sum_{c,d} T[a,c,b,d] g[c,d] on a grid (x,y,z batch labels)."""
    ext = {"a": n, "b": n, "c": n, "d": n, "x": points[0], "y": points[1], "z": points[2]}
    return "acbdxyz", "cdxyz", "abxyz", ext


def workload_gr_s(points=(128, 128, 128), n=4):
    """Pointwise S[a,b,c] = sum_d G[a,b,d] V[d,c] on a grid."""
    ext = {"a": n, "b": n, "c": n, "d": n, "x": points[0], "y": points[1], "z": points[2]}
    return "abdxyz", "dcxyz", "abcxyz", ext


def shape_of(labels, ext):
    return tuple(ext[l] for l in labels)


def make_operands(workload_id, labA, labB, ext, kind="uniform"):
    """The two inputs of a workload, drawn with the workload's seeds."""
    sa, sb = seed_for(workload_id, 0), seed_for(workload_id, 1)
    shA, shB = shape_of(labA, ext), shape_of(labB, ext)
    if kind == "uniform":
        return uniform(shA, sa), uniform(shB, sb)
    if kind == "integers":
        return integers(shA, sa), integers(shB, sb)
    if kind == "scaled_normal":
        return scaled_normal(shA, sa), scaled_normal(shB, sb)
    raise ValueError(kind)


def random_contraction(g, rank_range=(3, 6), ext_range=(4, 64), max_elems=1 << 22,
                       p_outer=0.0, log_extents=False, allow_batch=False):
    """A random binary contraction: ranks of A and B drawn independently in
    rank_range, p contracted labels uniform in [1, min(rA, rB)] (p = 0 with
    probability p_outer), extents uniform (or log-uniform) in ext_range,
    random storage order of every tensor; rejection-sampled until each
    operand and the output hold at most max_elems entries.

    Returns (labA, labB, labC, ext) with single-character labels."""
    letters = "abcdefghijklmnopqrstuvwxyz"
    while True:
        rA = int(g.integers(rank_range[0], rank_range[1] + 1))
        rB = int(g.integers(rank_range[0], rank_range[1] + 1))
        if p_outer > 0 and g.random() < p_outer:
            p = 0
        else:
            p = int(g.integers(1, min(rA, rB) + 1))
        nb = 0
        if allow_batch and p < min(rA, rB) and g.random() < 0.2:
            nb = 1
        fa, fb = rA - p - nb, rB - p - nb
        if fa < 0 or fb < 0:
            continue
        labs = list(letters[: p + nb + fa + fb])
        g.shuffle(labs)
        con, bat = labs[:p], labs[p:p + nb]
        frA, frB = labs[p + nb:p + nb + fa], labs[p + nb + fa:]
        ext = {}
        for l in labs:
            if log_extents:
                ext[l] = int(round(np.exp(g.uniform(np.log(ext_range[0]), np.log(ext_range[1])))))
            else:
                ext[l] = int(g.integers(ext_range[0], ext_range[1] + 1))
        la = con + bat + frA
        lb = con + bat + frB
        lc = frA + frB + bat
        g.shuffle(la)
        g.shuffle(lb)
        g.shuffle(lc)
        size = lambda ls: int(np.prod([ext[l] for l in ls], dtype=np.int64)) if ls else 1
        if max(size(la), size(lb), size(lc)) > max_elems:
            continue
        return "".join(la), "".join(lb), "".join(lc), ext


def unravel_colmajor(lin, extents):
    """Column-major multi-indices (n, len(extents)) of linear indices."""
    lin = np.asarray(lin, dtype=np.int64)
    out = np.empty((lin.size, len(extents)), dtype=np.int64)
    for d, e in enumerate(extents):
        out[:, d] = lin % e
        lin = lin // e
    return out


def stratified_entries(shape, split, row_block, col_block, seed):
    """Output entries on a stratified grid: the modes of C before `split` form
    the row index, the rest the column index (each linearised column-major).
    One row is drawn uniformly inside every block of row_block consecutive
    rows, one column inside every block of col_block columns, and every
    (row, column) pair is returned, rows outermost, as an (n, len(shape))
    multi-index array.  Any tile of at least row_block x col_block aligned
    entries therefore holds a sample, and consecutive entries share a row."""
    g = rng(seed)
    nr = int(np.prod(shape[:split], dtype=np.int64))
    nc = int(np.prod(shape[split:], dtype=np.int64))

    def pick(n, block):
        starts = np.arange(0, n, block, dtype=np.int64)
        width = np.minimum(block, n - starts)
        return starts + (g.random(starts.size) * width).astype(np.int64)

    rows, cols = pick(nr, row_block), pick(nc, col_block)
    r = np.repeat(rows, cols.size)
    c = np.tile(cols, rows.size)
    return np.concatenate([unravel_colmajor(r, shape[:split]), unravel_colmajor(c, shape[split:])], axis=1)
