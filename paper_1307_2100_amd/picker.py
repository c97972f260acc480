"""Learned recipe/tile picker: timing collection, GPU training, evaluation.

The paper picks one slicing per contraction class by rule (Sec. 3.2: the
class decides between GEMM, COPY + GEMM and the BLAS-2/1 loops, and the
largest index stays unsliced).  This module adds a data-driven choice among
the library's candidates (recipe x GEMM tile, plus the rules' own plan as the
last candidate): an MLP predicts, from layout features, each candidate's time
relative to the rules' plan, and a plan created with picker="mlp" takes the
fastest prediction the shape can run.  Numerical results do not depend on the
choice: every candidate computes the same contraction.

Everything that computes runs in libtc: the features come from
tc_picker_features, the timings from tc_plan_autotune (HIP events around the
library's own kernels), and the network is trained and evaluated by the
tc_mlp_* HIP kernels.  PyTorch only holds device buffers.

Command line:
  python -m paper_1307_2100_amd.picker collect --out F --n N [--seed S]
  python -m paper_1307_2100_amd.picker train --data F [F ...] --test N --out MODEL
  python -m paper_1307_2100_amd.picker evaluate --data F --model MODEL
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import (MLP, PICKER_CANDIDATES, PICKER_FEATURES, Desc, Plan, tc_picker_candidate, tc_picker_features,
               tc_picker_install, tc_picker_uninstall, tc_version)

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "picker_model.json")
RULES = PICKER_CANDIDATES - 1  # the last candidate is the rules' own plan
HIDDEN = 64

# Caps that keep one shape's buffers and timings small (elements per tensor,
# multiply-adds per contraction).
MAX_ELEMS = 1 << 22
MAX_MADDS = 1 << 30


# --------------------------------------------------------------------- shapes
def random_shape(rng, rank_range=(2, 6), ext_range=(2, 256), max_elems=MAX_ELEMS, max_madds=MAX_MADDS):
    """A random dense contraction: labels, extents and storage order of A, B
    and C.  Ranks of A and B in rank_range; extents log-uniform in ext_range,
    then the largest extents halved until every tensor and the multiply-add
    count fit the caps; each tensor stored densely in a random mode order.
    Returns dict(a=..., b=..., c=...), each a (labels, extents, strides)."""
    lo, hi = rank_range
    while True:
        ra, rb = int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))
        nb = int(rng.integers(0, 2)) if rng.uniform() < 0.15 else 0   # batch labels (in A, B and C)
        p = int(rng.integers(1 if rng.uniform() < 0.95 else 0, min(ra, rb) - nb + 1))
        da, db = ra - nb - p, rb - nb - p
        if da < 0 or db < 0 or da + db + nb < 1:
            continue
        break
    labels = iter(range(ord("a"), ord("a") + 26))
    bat = [next(labels) for _ in range(nb)]
    con = [next(labels) for _ in range(p)]
    fa = [next(labels) for _ in range(da)]
    fb = [next(labels) for _ in range(db)]
    ext = {l: int(round(math.exp(rng.uniform(math.log(ext_range[0]), math.log(ext_range[1])))))
           for l in bat + con + fa + fb}
    la, lb, lc = bat + con + fa, bat + con + fb, bat + fa + fb
    for order in (la, lb, lc):
        rng.shuffle(order)

    def elems(ls):
        return int(np.prod([ext[l] for l in ls])) if ls else 1

    while True:
        madds = elems(bat + con + fa + fb)
        worst = max((la, lb, lc), key=elems)
        if elems(worst) <= max_elems and madds <= max_madds:
            break
        big = worst if elems(worst) > max_elems else bat + con + fa + fb
        l = max(big, key=lambda x: ext[x])
        ext[l] = max(1, ext[l] // 2)

    def desc(ls):
        # dense storage in a random mode order
        perm = list(rng.permutation(len(ls)))
        strides = [0] * len(ls)
        s = 1
        for i in perm:
            strides[i] = s
            s *= ext[ls[i]]
        return [int(x) for x in ls], [ext[l] for l in ls], strides

    return {"a": desc(la), "b": desc(lb), "c": desc(lc)}


def _descs(shape):
    return [Desc(shape[k][1], shape[k][2], shape[k][0]) for k in ("a", "b", "c")]


def _alloc(torch, spec, gen):
    labels, ext, strides = spec
    span = 1 + sum((e - 1) * s for e, s in zip(ext, strides)) if ext else 1
    base = torch.rand(max(1, span), dtype=torch.float64, device="cuda", generator=gen)
    return torch.as_strided(base, ext, strides) if ext else base[0]


def features(shape):
    """(features, the rules' candidate in the explicit table or -1)."""
    dA, dB, dC = _descs(shape)
    f, rc = tc_picker_features(dA, dB, dC)
    return f, rc


# ----------------------------------------------------------------- collection
# The sources the candidates run through (planner, FP64 execution path and
# its kernels, the C header); batches, split precision and the network are
# not among them.
CANDIDATE_SOURCES = ("api.cpp", "planner.cpp", "planner.hpp", "kernels.hpp", "gett_f64.hip", "gett_tile.hpp",
                     "permute.hip", "blas2.hip", "lanes.hpp", "batched.hip", "batched_slab.hpp")


def library_source_sha():
    """sha256 (first 16 hex digits) of CANDIDATE_SOURCES and the C header:
    the kernels and rules that candidate timings were taken with."""
    import hashlib
    root = os.path.dirname(HERE)
    paths = [os.path.join(HERE, "csrc", f) for f in CANDIDATE_SOURCES]
    paths.append(os.path.join(root, "include", "tc.h"))
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def collect(out, n, seed=0, log_every=200, seconds=None):
    """Times every candidate on n random shapes (index i uses seed + i) and
    appends one JSON line per shape to `out`; an existing file is resumed.
    With `seconds`, stops after the first shape that ends past that budget
    (run again to continue)."""
    import torch
    lib_sha = library_source_sha()
    done = 0
    if os.path.exists(out):
        with open(out) as f:
            done = sum(1 for line in f if line.strip())
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    t0 = time.time()
    with open(out, "a") as f:
        for i in range(done, n):
            rng = np.random.default_rng([seed, i])
            shape = random_shape(rng)
            feat, rc = features(shape)
            dA, dB, dC = _descs(shape)
            A = _alloc(torch, shape["a"], gen)
            B = _alloc(torch, shape["b"], gen)
            C = _alloc(torch, shape["c"], gen)
            plan = Plan(dA, dB, dC)
            best, best_ms, ms = plan.autotune(A, B, C)
            info = plan.info
            plan.close()
            rec = {"i": i, "seed": seed, "shape": shape, "features": feat, "rule_candidate": rc, "ms": ms,
                   "best": best, "flops": info.flops, "bytes": info.bytes, "paper_class": info.paper_class,
                   "lib_sha": lib_sha}
            f.write(json.dumps(rec) + "\n")
            if (i + 1) % log_every == 0:
                f.flush()
                print("collect: %d/%d shapes, %.1f s" % (i + 1, n, time.time() - t0), flush=True)
            if seconds is not None and time.time() - t0 > seconds:
                print("collect: time budget spent after %d/%d shapes; run again to resume" % (i + 1, n), flush=True)
                return
    print("collect: done, %d shapes in %s" % (n, out), flush=True)


def load_records(paths):
    """Records of one or more collection files (plain or gzip-compressed JSON lines)."""
    import gzip
    recs = []
    for p in paths:
        opener = gzip.open if p.endswith(".gz") else open
        with opener(p, "rt") as f:
            recs.extend(json.loads(line) for line in f if line.strip())
    return recs


def arrays(recs):
    """X (features), ms (candidate times, nan where illegal)."""
    X = np.array([r["features"] for r in recs], dtype=np.float32)
    ms = np.array([[t if t > 0 else np.nan for t in r["ms"]] for r in recs], dtype=np.float64)
    return X, ms


def targets(ms):
    """Targets log2(t / t_rules) and the mask of candidates that ran."""
    M = np.isfinite(ms).astype(np.float32)
    T = np.where(M > 0, np.log2(np.where(M > 0, ms, 1.0) / ms[:, RULES:RULES + 1]), 0.0).astype(np.float32)
    return T, M


# ------------------------------------------------------------------ training
def _he_init(rng, n_in, hidden, n_out):
    parts = []
    for fi, fo in ((n_in, hidden), (hidden, hidden), (hidden, n_out)):
        parts.append((rng.standard_normal(fi * fo) * math.sqrt(2.0 / fi)).astype(np.float32))
        parts.append(np.zeros(fo, dtype=np.float32))
    return np.concatenate(parts)


def normalisation(X):
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std < 1e-6] = 1.0
    return mean.astype(np.float32), std.astype(np.float32)


def train(X, T, M, epochs=100, batch=256, lr=3e-3, seed=0, log=print):
    """Trains the picker network on the GPU with the libtc kernels (Adam,
    masked MSE, learning rate decayed linearly to lr/20); returns (params,
    mean, std, history of mean training loss per epoch)."""
    import torch
    rng = np.random.default_rng(seed)
    mean, std = normalisation(X)
    Xn = (X - mean) / std
    dev = "cuda"
    Xd = torch.from_numpy(np.ascontiguousarray(Xn, dtype=np.float32)).to(dev)
    Td = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).to(dev)
    Md = torch.from_numpy(np.ascontiguousarray(M, dtype=np.float32)).to(dev)
    net = MLP(PICKER_FEATURES, HIDDEN, PICKER_CANDIDATES, batch)
    net.set_params(_he_init(rng, PICKER_FEATURES, HIDDEN, PICKER_CANDIDATES))
    n = Xd.shape[0]
    steps = epochs * ((n + batch - 1) // batch)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    history = []
    k = 0
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(n)).to(dev)
        acc, cnt = 0.0, 0
        for b0 in range(0, n, batch):
            idx = order[b0:b0 + batch]
            step_lr = lr * (1.0 - 0.95 * k / max(1, steps - 1))
            net.train_step(Xd.index_select(0, idx).contiguous(), Td.index_select(0, idx).contiguous(),
                           Md.index_select(0, idx).contiguous(), step_lr, loss=loss)
            acc += float(loss.item()) * idx.numel()
            cnt += idx.numel()
            k += 1
        history.append(acc / cnt)
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log("train: epoch %d/%d, loss %.4f" % (ep + 1, epochs, history[-1]))
    params = np.array(net.get_params(), dtype=np.float32)
    net.close()
    return params, mean, std, history


def predict(params, mean, std, X, batch=1024):
    """Predicted log2 time ratios (n, candidates), on the GPU."""
    import torch
    net = MLP(PICKER_FEATURES, HIDDEN, PICKER_CANDIDATES, batch)
    net.set_params(params)
    Xn = ((X - mean) / std).astype(np.float32)
    out = []
    for b0 in range(0, Xn.shape[0], batch):
        xb = torch.from_numpy(np.ascontiguousarray(Xn[b0:b0 + batch])).to("cuda")
        out.append(net.forward(xb).cpu().numpy())
    net.close()
    return np.concatenate(out) if out else np.zeros((0, PICKER_CANDIDATES), np.float32)


# ---------------------------------------------------------------- evaluation
def picks(pred, ms):
    """The candidate a plan takes: the fastest prediction that can run."""
    order = np.argsort(pred, axis=1, kind="stable")
    legal = np.isfinite(ms)
    return np.array([next(c for c in row if legal[i, c]) for i, row in enumerate(order)])


def evaluate(pred, ms):
    """Metrics of the picks against exhaustive timing and against the rules."""
    n = ms.shape[0]
    pick = picks(pred, ms)
    best = np.nanmin(ms, axis=1)
    t_pick = ms[np.arange(n), pick]
    t_rule = ms[:, RULES]

    def gm(x):
        return float(np.exp(np.mean(np.log(x))))

    return {
        "shapes": int(n),
        "geomean_pick_over_best": gm(t_pick / best),
        "geomean_rules_over_best": gm(t_rule / best),
        "within_5pct_pick": float(np.mean(t_pick <= 1.05 * best)),
        "within_5pct_rules": float(np.mean(t_rule <= 1.05 * best)),
        "gain_geomean_rules_over_pick": gm(t_rule / t_pick),
        "total_ms_pick": float(t_pick.sum()),
        "total_ms_rules": float(t_rule.sum()),
        "total_ms_best": float(best.sum()),
        "worst_pick_over_best": float(np.max(t_pick / best)),
        "worst_rules_over_best": float(np.max(t_rule / best)),
        "pick_histogram": np.bincount(pick, minlength=PICKER_CANDIDATES).tolist(),
        "best_histogram": np.bincount(np.nanargmin(ms, axis=1), minlength=PICKER_CANDIDATES).tolist(),
    }


# ------------------------------------------------------------- model files
def save_model(path, params, mean, std, meta):
    doc = {"format": "tc-picker-mlp", "library_version": tc_version(), "n_in": PICKER_FEATURES, "hidden": HIDDEN,
           "n_out": PICKER_CANDIDATES, "target": "log2(time / time of the rules' plan)",
           "candidates": [list(tc_picker_candidate(c)) for c in range(PICKER_CANDIDATES)],
           "params": [float(v) for v in params], "mean": [float(v) for v in mean], "std": [float(v) for v in std]}
    doc.update(meta)
    with open(path, "w") as f:
        json.dump(doc, f)


def load_model(path=DEFAULT_MODEL):
    """(params, mean, std, doc); raises ValueError on a malformed or foreign file."""
    with open(path) as f:
        doc = json.load(f)
    if doc.get("format") != "tc-picker-mlp":
        raise ValueError("not a picker model file")
    if doc.get("n_in") != PICKER_FEATURES or doc.get("n_out") != PICKER_CANDIDATES or doc.get("hidden") != HIDDEN:
        raise ValueError("model dimensions do not match this library")
    if [list(tc_picker_candidate(c)) for c in range(PICKER_CANDIDATES)] != doc.get("candidates"):
        raise ValueError("model was trained for another candidate table")
    params = np.array(doc["params"], dtype=np.float32)
    mean = np.array(doc["mean"], dtype=np.float32)
    std = np.array(doc["std"], dtype=np.float32)
    if not (np.all(np.isfinite(params)) and np.all(np.isfinite(mean)) and np.all(std > 0)):
        raise ValueError("model holds non-finite values")
    return params, mean, std, doc


def install(path=DEFAULT_MODEL):
    """Installs a model for picker="mlp" plans; returns False (plans keep the
    rules) when the file is missing or unusable."""
    try:
        params, mean, std, _ = load_model(path)
    except (OSError, ValueError, KeyError) as e:
        print("picker: no usable model (%s); plans use the rules" % e, file=sys.stderr)
        tc_picker_uninstall()
        return False
    tc_picker_install(params, HIDDEN, mean, std)
    return True


def rules_now(recs):
    """The rules of the current library against timed records.  A record's
    rules time is its measured rules plan (candidate RULES) while the rules
    still take the candidate they took at collection; when they now take
    another table candidate, that candidate's measured time."""
    t_rule, best, changed = [], [], 0
    for r in recs:
        ms = np.array([np.nan if (v is None or v < 0) else v for v in r["ms"]], dtype=np.float64)
        _, now = tc_picker_features(*_descs(r["shape"]))
        t = ms[RULES]
        if now != r["rule_candidate"] and now >= 0 and np.isfinite(ms[now]):
            changed += 1
            t = ms[now]
        t_rule.append(t)
        best.append(np.nanmin(ms))
    t_rule, best = np.array(t_rule), np.array(best)
    return {"shapes": len(recs), "rules_changed_since_collection": changed,
            "geomean_rules_over_best": float(np.exp(np.mean(np.log(t_rule / best)))),
            "within_5pct_rules": float(np.mean(t_rule <= 1.05 * best)),
            "worst_rules_over_best": float(np.max(t_rule / best)), "total_ms_rules": float(t_rule.sum())}


# ---------------------------------------------------------------------- CLI
def _split(recs, n_test):
    """Held-out shapes: the last n_test records by index (disjoint seeds)."""
    recs = sorted(recs, key=lambda r: (r["seed"], r["i"]))
    return recs[:-n_test] if n_test else recs, recs[-n_test:] if n_test else []


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1307_2100_amd.picker")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--out", required=True)
    c.add_argument("--n", type=int, required=True)
    c.add_argument("--seed", type=int, default=0)
    c.add_argument("--seconds", type=float, default=None, help="stop after this many seconds (resumable)")
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--test", type=int, default=5000)
    t.add_argument("--epochs", type=int, default=100)
    t.add_argument("--out", default=DEFAULT_MODEL)
    t.add_argument("--report", default=None)
    e = sub.add_parser("evaluate")
    e.add_argument("--data", nargs="+", required=True)
    e.add_argument("--model", default=DEFAULT_MODEL)
    r = sub.add_parser("rules", help="host only: the current rules against timed data")
    r.add_argument("--data", nargs="+", required=True)
    r.add_argument("--test", type=int, default=5000)
    a = ap.parse_args(argv)
    if a.cmd == "rules":
        tr, te = _split(load_records(a.data), a.test)
        print(json.dumps({"heldout": rules_now(te), "train": rules_now(tr)}), flush=True)
        return
    if a.cmd == "collect":
        collect(a.out, a.n, a.seed, seconds=a.seconds)
    elif a.cmd == "train":
        recs = load_records(a.data)
        tr, te = _split(recs, a.test)
        Xtr, mstr = arrays(tr)
        Ttr, Mtr = targets(mstr)
        t0 = time.time()
        params, mean, std, hist = train(Xtr, Ttr, Mtr, epochs=a.epochs)
        secs = time.time() - t0
        Xte, mste = arrays(te)
        res_te = evaluate(predict(params, mean, std, Xte), mste) if len(te) else {}
        res_tr = evaluate(predict(params, mean, std, Xtr), mstr)
        shas = sorted({r.get("lib_sha", "unrecorded") for r in recs})
        meta = {"train_shapes": len(tr), "test_shapes": len(te), "epochs": a.epochs, "train_seconds": secs,
                "final_train_loss": hist[-1], "eval_heldout": res_te, "eval_train": res_tr,
                "timings_library_source_sha": shas, "trained_with_library_source_sha": library_source_sha()}
        save_model(a.out, params, mean, std, meta)
        print(json.dumps({"heldout": res_te, "train": {k: res_tr[k] for k in res_tr if "histogram" not in k}}),
              flush=True)
        if a.report:
            with open(a.report, "w") as f:
                json.dump(meta, f, indent=1)
    else:
        recs = load_records(a.data)
        params, mean, std, _ = load_model(a.model)
        X, ms = arrays(recs)
        print(json.dumps(evaluate(predict(params, mean, std, X), ms)), flush=True)


if __name__ == "__main__":
    main()
