"""The paper's numerical experiments (Sec. 4) on one GPU, with each recipe
forced through tc_options, plus the layout advice of Sec. 3.3 measured.

    python -m paper_1307_2100_amd.experiments [--quick] [--md PATH]

Studies (inputs: seeded uniform[-1, 1] FP64 drawn on the device, stored
column-major in the listed label order):

  square   Sec. 4.1: R[a,h] = A[a,b,g] B[h,b,g] (Class 3.2) and
           R[b,h] = A[a,b,g] B[g,a,h] (Class 3.1), every extent n; recipes
           GEMM, COPY+GEMM, GEMV, GER.
  cc       Sec. 4.2, example 1: R[a,c,d] = X[i,a,j] Y[i,c,j,d] (the paper's
           R = X Y with the free index of X after j held at one value), short
           free extents, long contracted ones; recipes GEMM, COPY+GEMM, DOT,
           GER.
  gr       Sec. 4.2, example 2: the same contraction with i = j = 4 and long
           free extents.
  slices   Sec. 2.4: the square contraction run as the paper's slice loops
           (one library call per slice; GEMM, GEMV, GER and DOT slicings)
           against the fused launch.
  chain    Appendix: raising two indices of a rank-4 tensor with the metric,
           in the least-flop pairwise order and in operand order.
  layout   Sec. 3.3: a Class 3.1 layout timed as given and re-stored in the
           orders tc_suggest_layout returns (direct GEMM).

Every run is timed with HIP events on the current stream (one untimed call
first; more calls while the total stays short).  Each recipe's result is
compared with the rules' choice (`auto`) on the same inputs: the largest
difference, relative to the contracted extent K (with inputs in [-1, 1],
|A||B| <= K entrywise), is reported and must stay below 1e-12.  One JSON
object per run goes to stdout; --md writes a summary table.
"""
import argparse
import json
import sys
import time

import torch

import paper_1307_2100_amd as tc

FP64_PEAK_TFLOPS = 78.6   # MI355X, dense FP64 MFMA
HBM_PEAK_GBS = 8000.0     # MI355X, HBM3E

RECIPES = {"square": ("gemm", "copy_gemm", "gemv", "ger"),
           "cc": ("gemm", "copy_gemm", "dot", "ger"),
           "gr": ("gemm", "copy_gemm", "dot", "ger")}


def _uniform(shape, gen):
    t = tc.empty_colmajor(list(shape), device="cuda")
    t.uniform_(-1.0, 1.0, generator=gen)
    return t


def _time(plan, A, B, C, budget_ms=400.0, max_reps=20):
    ws = plan.workspace(C.device)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    plan.execute(A, B, C, stream=stream, workspace=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    first = e0.elapsed_time(e1)
    reps = int(max(0, min(max_reps, budget_ms / max(first, 1e-3))))
    if reps == 0:
        return first, 1
    e0.record(stream)
    for _ in range(reps):
        plan.execute(A, B, C, stream=stream, workspace=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, reps


def _shape(lab, ext):
    return [ext[l] for l in lab]


def run_recipes(study, la, lb, lc, ext, recipes, seed, inputs=None, keep_outputs=False):
    """One contraction under the rules and under each forced recipe.  inputs:
    optional (A, B) device tensors to use instead of seeded uniform ones;
    keep_outputs: each row also holds its result tensor under "C"."""
    if inputs is None:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        A, B = _uniform(_shape(la, ext), gen), _uniform(_shape(lb, ext), gen)
    else:
        A, B = inputs
    K = 1
    for l in la:
        if l in lb and l not in lc:
            K *= ext[l]
    ref = None
    rows = []
    for recipe in ("auto",) + tuple(recipes):
        C = tc.empty_colmajor(_shape(lc, ext), device="cuda")
        plan = tc.Plan.for_tensors(A, la, B, lb, C, lc, recipe=recipe)
        try:
            ms, reps = _time(plan, A, B, C)
            info = plan.info
        finally:
            plan.close()
        if ref is None:
            ref = C
            diff = 0.0
        else:
            diff = float((C - ref).abs().max()) / K if C.numel() else 0.0
        row = {"study": study, "contraction": "%s,%s->%s" % (la, lb, lc),
               "extents": {l: ext[l] for l in sorted(ext)}, "recipe": recipe,
               "ran": tc.RECIPE_NAMES[info.recipe], "paper_class": info.paper_class,
               "kernel": tc.KERNEL_NAMES.get(info.kernel, "?"), "ms": round(ms, 4), "reps": reps,
               "gflops": round(info.flops / ms / 1e6, 2), "max_diff_over_K": diff}
        bound_ms = max(info.flops / (FP64_PEAK_TFLOPS * 1e9), info.bytes / (HBM_PEAK_GBS * 1e6))
        row["frac_roofline"] = round(bound_ms / ms, 4) if ms > 0 else None
        print(json.dumps(row), flush=True)
        if diff > 1e-12:
            raise RuntimeError("recipe %s disagrees with the rules' result: %.3e" % (recipe, diff))
        if keep_outputs:
            row["C"] = C
        elif C is not ref:
            del C
        rows.append(row)
    del A, B, ref
    torch.cuda.empty_cache()
    return rows


def run_layout(la, lb, lc, ext, seed, inputs=None, keep_outputs=False):
    """A contraction timed in the given layout and in the suggested one
    (inputs and keep_outputs as for run_recipes; each kept result is viewed in
    the given output's label order)."""
    out, info = tc.suggest_layout(la, _shape(la, ext), lb, _shape(lb, ext), lc, _shape(lc, ext))
    if inputs is None:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        A, B = _uniform(_shape(la, ext), gen), _uniform(_shape(lb, ext), gen)
    else:
        A, B = inputs
    rows = []
    results = {}
    for which, (xa, xb, xc) in (("given", (la, lb, lc)), ("suggested", (out["A"], out["B"], out["C"]))):
        if which == "given":
            dA, dB = A, B
        else:
            # re-store the same values with the suggested mode orders
            dA = tc.empty_colmajor(_shape(xa, ext), device="cuda")
            dA.copy_(A.permute([la.index(l) for l in xa]))
            dB = tc.empty_colmajor(_shape(xb, ext), device="cuda")
            dB.copy_(B.permute([lb.index(l) for l in xb]))
        C = tc.empty_colmajor(_shape(xc, ext), device="cuda")
        plan = tc.Plan.for_tensors(dA, xa, dB, xb, C, xc)
        try:
            ms, reps = _time(plan, dA, dB, C)
            pinfo = plan.info
        finally:
            plan.close()
        results[which] = C.permute([xc.index(l) for l in lc])
        row = {"study": "layout", "contraction": "%s,%s->%s" % (xa, xb, xc), "layout": which,
               "extents": {l: ext[l] for l in sorted(ext)}, "ran": tc.RECIPE_NAMES[pinfo.recipe],
               "paper_class": pinfo.paper_class, "copy_operand": pinfo.copy_operand,
               "ms": round(ms, 4), "reps": reps, "gflops": round(pinfo.flops / ms / 1e6, 2)}
        print(json.dumps(row), flush=True)
        rows.append(row)
    K = 1
    for l in la:
        if l in lb and l not in lc:
            K *= ext[l]
    diff = float((results["given"] - results["suggested"]).abs().max()) / K
    rows[-1]["max_diff_over_K"] = diff
    if diff > 1e-12:
        raise RuntimeError("suggested layout disagrees with the given one: %.3e" % diff)
    if keep_outputs:
        rows[0]["C"], rows[1]["C"] = results["given"], results["suggested"]
    del A, B, results
    torch.cuda.empty_cache()
    return rows


def run_slicings(la, lb, lc, ext, slicings, seed):
    """The fused launch against the paper's slice loops (one library call per
    slice, Sec. 2.4) for each slicing in `slicings` (labels looped over)."""
    from . import slicing
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    A, B = _uniform(_shape(la, ext), gen), _uniform(_shape(lb, ext), gen)
    K = 1
    for l in la:
        if l in lb and l not in lc:
            K *= ext[l]
    flops = 2.0 * K
    for l in set(la) | set(lb):
        if not (l in la and l in lb and l not in lc):
            flops *= ext[l]
    ref = tc.empty_colmajor(_shape(lc, ext), device="cuda")
    plan = tc.Plan.for_tensors(A, la, B, lb, ref, lc)
    try:
        ms, reps = _time(plan, A, B, ref)
        ran = tc.RECIPE_NAMES[plan.info.recipe]
    finally:
        plan.close()
    rows = [{"study": "slices", "contraction": "%s,%s->%s" % (la, lb, lc), "extents": {l: ext[l] for l in sorted(ext)},
             "sliced": "", "calls": 1, "ran": ran, "ms": round(ms, 4), "gflops": round(flops / ms / 1e6, 2),
             "max_diff_over_K": 0.0}]
    print(json.dumps(rows[0]), flush=True)
    for sl in slicings:
        C = tc.empty_colmajor(_shape(lc, ext), device="cuda")
        slicing.run_sliced(A, la, B, lb, C, lc, sl)          # untimed first pass
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        calls = slicing.run_sliced(A, la, B, lb, C, lc, sl)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        diff = float((C - ref).abs().max()) / K
        row = {"study": "slices", "contraction": "%s,%s->%s" % (la, lb, lc), "extents": {l: ext[l] for l in sorted(ext)},
               "sliced": sl, "calls": calls, "ms": round(ms, 4), "gflops": round(flops / ms / 1e6, 2),
               "max_diff_over_K": diff}
        print(json.dumps(row), flush=True)
        if diff > 1e-12:
            raise RuntimeError("slicing %s disagrees with the fused result: %.3e" % (sl, diff))
        rows.append(row)
        del C
    del A, B, ref
    torch.cuda.empty_cache()
    return rows


def run_chain(n, seed):
    """Raising two indices of a rank-4 tensor with the metric (the appendix):
    R[e,f,c,d] = T[a,b,c,d] g[a,e] g[b,f], with the operands listed metric
    first, evaluated in the least-flop order and in operand order (which
    forms the outer product of the two metrics first)."""
    from . import chain
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    T = _uniform([n] * 4, gen)
    g = _uniform([n, n], gen)
    ops = [(g, "ae"), (g, "bf"), (T, "abcd")]
    rows, res = [], {}
    ext = {ord(c): n for c in "abcdef"}
    for order in ("optimal", "left"):
        t0 = time.perf_counter()
        ch = chain.Chain(ops, "efcd", order=order)
        plan_ms = (time.perf_counter() - t0) * 1e3
        try:
            tensors = [t for t, _ in ops]
            stream = torch.cuda.current_stream()
            ch.execute(tensors)                                # untimed first pass
            torch.cuda.synchronize()
            reps = 5
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                ch.execute(tensors)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            res[order] = ch.execute(tensors).clone()
            torch.cuda.synchronize()
        finally:
            ch.close()
        row = {"study": "chain", "contraction": "ae,bf,abcd->efcd", "extents": {"all": n}, "order": order,
               "steps": len(ch.steps), "flops": ch.flops, "ms": round(ms, 4), "plan_ms": round(plan_ms, 3),
               "gflops": round(ch.flops / ms / 1e6, 2)}
        print(json.dumps(row), flush=True)
        rows.append(row)
    diff = float((res["optimal"] - res["left"]).abs().max()) / n ** 2
    rows[-1]["max_diff_over_K"] = diff
    if diff > 1e-12:
        raise RuntimeError("chain orders disagree: %.3e" % diff)
    del T, g, res
    torch.cuda.empty_cache()
    return rows


def slicing_workloads(quick):
    # R[a,h] = A[a,b,g] B[h,b,g] (Sec. 4.1): slicing g leaves GEMMs; h and g,
    # GEMVs; b and g, GERs; a and h, DOTs over (b, g)
    for n in ((64, 128) if quick else (64, 128, 256)):
        sl = ["g", "b"] + (["hg", "bg", "ah"] if n <= 128 else [])
        yield "abg", "hbg", "ah", {l: n for l in "abgh"}, sl


def workloads(quick):
    sq = (64, 128, 256) if quick else (64, 128, 192, 256, 384, 512)
    # Fig. 4D-1: i = j up to 3000 at free extents 30, and free extents 30 to
    # 100 at i = j = 1000 (the largest input, Y, is 65 GB and 80 GB there)
    cc_ij = (500, 1000) if quick else (500, 1000, 2000, 3000)
    cc_f = (30, 45) if quick else (30, 45, 60, 80, 100)
    gr_f = (100, 200) if quick else (100, 200, 400, 600)
    for n in sq:
        yield "square", "abg", "hbg", "ah", {l: n for l in "abgh"}
        yield "square", "abg", "gah", "bh", {l: n for l in "abgh"}
    for ij in cc_ij:
        yield "cc", "iaj", "icjd", "acd", {"i": ij, "j": ij, "a": 30, "c": 30, "d": 30}
    for f in cc_f:
        yield "cc", "iaj", "icjd", "acd", {"i": 1000, "j": 1000, "a": f, "c": f, "d": f}
    for f in gr_f:
        yield "gr", "iaj", "icjd", "acd", {"i": 4, "j": 4, "a": f, "c": f, "d": f}


def layout_workloads(quick):
    n = 256 if quick else 512
    yield "abg", "gah", "bh", {l: n for l in "abgh"}
    # a coupled-cluster contraction stored with a different contracted index at
    # stride 1 in each input (Class 3.1), v = 128, o = 32
    v, o = (64, 16) if quick else (128, 32)
    yield "cdab", "dcij", "abij", {"a": v, "b": v, "c": v, "d": v, "i": o, "j": o}


def markdown(rows, cmd):
    lines = ["# The paper's experiments (Sec. 4) and its layout advice (Sec. 3.3) on one MI355X", "",
             "Command: `%s`" % cmd, "",
             "Inputs: seeded uniform[-1,1] FP64 drawn on the device, column-major in the listed label order. "
             "Times: HIP events on the current stream, mean over the calls shown (one untimed call first). "
             "`auto` is the rules' choice; every forced recipe agrees with it to < 1e-12 K. Each cell gives "
             "GFLOP/s and, in brackets, the fraction of the contraction's roofline bound: max(2 M N K L / "
             "78.6 TFLOP/s, 8 (|A| + |B| + |C|) / 8 TB/s) over the measured time (the COPY of COPY+GEMM is "
             "not counted as work).", ""]
    for study, title in (("square", "Sec. 4.1: 3-D square tensors"),
                         ("cc", "Sec. 4.2 example 1: coupled-cluster shapes (short free, long contracted)"),
                         ("gr", "Sec. 4.2 example 2: general-relativity shapes (contracted extents 4)")):
        sel = [r for r in rows if r["study"] == study]
        if not sel:
            continue
        recipes = ["auto"] + list(RECIPES[study])
        lines += ["## " + title, "",
                  "| contraction | extents | class | " + " | ".join("%s GFLOP/s" % r for r in recipes) + " |",
                  "|---|---|---|" + "---|" * len(recipes)]
        keys = []
        for r in sel:
            k = (r["contraction"], json.dumps(r["extents"], sort_keys=True))
            if k not in keys:
                keys.append(k)
        for k in keys:
            grp = {r["recipe"]: r for r in sel if (r["contraction"], json.dumps(r["extents"], sort_keys=True)) == k}
            ext = json.loads(k[1])
            extent_s = " ".join("%s=%d" % (l, e) for l, e in ext.items())
            auto = grp["auto"]
            cells = []
            for rc in recipes:
                r = grp.get(rc)
                if r is None:
                    cells.append("-")
                    continue
                txt = "%.0f" % r["gflops"] if r["gflops"] >= 10 else "%.2f" % r["gflops"]
                if r.get("frac_roofline") is not None:
                    txt += " [%.2f]" % r["frac_roofline"]
                if rc == "auto":
                    txt += " (%s)" % r["ran"]
                cells.append(txt)
            lines.append("| %s | %s | %s | %s |" % (k[0], extent_s, auto["paper_class"], " | ".join(cells)))
        lines.append("")
    sel = [r for r in rows if r["study"] == "slices"]
    if sel:
        lines += ["## Sec. 2.4: the paper's slice loops (one library call per slice) against one fused launch", "",
                  "| contraction | extents | labels looped over | calls | ms | GFLOP/s |", "|---|---|---|---|---|---|"]
        for r in sel:
            extent_s = " ".join("%s=%d" % (l, e) for l, e in r["extents"].items())
            what = r["sliced"] or "none (fused, %s)" % r.get("ran", "")
            lines.append("| %s | %s | %s | %d | %.3f | %s |" % (r["contraction"], extent_s, what, r["calls"], r["ms"],
                                                             "%.0f" % r["gflops"] if r["gflops"] >= 10 else "%.2f" % r["gflops"]))
        lines.append("")
    sel = [r for r in rows if r["study"] == "chain"]
    if sel:
        lines += ["## Appendix: raising two indices with the metric, R[e,f,c,d] = g[a,e] g[b,f] T[a,b,c,d]", "",
                  "Planned once (order, intermediates, one plan per step), then timed over 5 executions with HIP "
                  "events; planning time listed apart.", "",
                  "| n (every extent) | order | steps | GFLOP | ms | GFLOP/s | planning ms |",
                  "|---|---|---|---|---|---|---|"]
        for r in sel:
            lines.append("| %d | %s | %d | %.2f | %.3f | %.0f | %.2f |" % (
                r["extents"]["all"], r["order"], r["steps"], r["flops"] / 1e9, r["ms"], r["gflops"], r["plan_ms"]))
        lines.append("")
    sel = [r for r in rows if r["study"] == "layout"]
    if sel:
        lines += ["## Sec. 3.3: layout advice (tc_suggest_layout)", "",
                  "| layout | contraction | class | recipe run | ms | GFLOP/s |", "|---|---|---|---|---|---|"]
        for r in sel:
            lines.append("| %s | %s | %s | %s | %.3f | %.0f |" % (r["layout"], r["contraction"], r["paper_class"],
                                                                r["ran"], r["ms"], r["gflops"]))
        lines.append("")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--quick", action="store_true", help="smaller sizes (a few seconds)")
    ap.add_argument("--study", action="append", choices=["square", "cc", "gr", "slices", "chain", "layout"],
                    help="run only these studies (repeatable)")
    ap.add_argument("--md", help="write a markdown summary here")
    args = ap.parse_args(argv)
    assert torch.cuda.is_available(), "the experiments need a GPU"
    torch.cuda.set_device(0)
    studies = set(args.study or ["square", "cc", "gr", "slices", "chain", "layout"])
    rows = []
    t0 = time.time()
    for i, (study, la, lb, lc, ext) in enumerate(workloads(args.quick)):
        if study in studies:
            print("[experiments] %s %s,%s->%s %s" % (study, la, lb, lc, ext), file=sys.stderr, flush=True)
            rows += run_recipes(study, la, lb, lc, ext, RECIPES[study], 1307 * 1000 + i)
    if "slices" in studies:
        for i, (la, lb, lc, ext, sl) in enumerate(slicing_workloads(args.quick)):
            print("[experiments] slices %s,%s->%s %s %s" % (la, lb, lc, ext, sl), file=sys.stderr, flush=True)
            rows += run_slicings(la, lb, lc, ext, sl, 1307 * 3000 + i)
    if "chain" in studies:
        for i, n in enumerate((32, 64) if args.quick else (32, 64, 96)):
            print("[experiments] chain n=%d" % n, file=sys.stderr, flush=True)
            rows += run_chain(n, 1307 * 4000 + i)
    if "layout" in studies:
        for i, (la, lb, lc, ext) in enumerate(layout_workloads(args.quick)):
            print("[experiments] layout %s,%s->%s %s" % (la, lb, lc, ext), file=sys.stderr, flush=True)
            rows += run_layout(la, lb, lc, ext, 1307 * 2000 + i)
    print("[experiments] done in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)
    if args.md:
        cmd = "python -m paper_1307_2100_amd.experiments" + (" --quick" if args.quick else "") + \
              "".join(" --study " + s for s in (args.study or [])) + " --md " + args.md
        with open(args.md, "w") as f:
            f.write(markdown(rows, cmd))
    return rows


if __name__ == "__main__":
    main()
