"""Benchmark: FP64 contraction throughput on the coupled-cluster workload.

One step = one pass of the hot path over one batch of input: the two
coupled-cluster contractions at v = 128, o = 32,
  (a) C[a,b,i,j] = sum_{c,d} A[a,b,c,d] B[c,d,i,j]   (paper class 3.2, direct GEMM)
  (b) C[a,b,i,j] = sum_{k,c} A[a,k,i,c] B[k,b,c,j]   (class 3.2 with un-fusable index groups)
each through tc_execute on plans built once.  Inputs are seeded synthetic
FP64 tensors (uniform in [-1, 1], column-major) resident in HBM before the
timed region.  Prints one JSON line.

Besides the step, the JSON line carries (outside the timed region) the
split-precision runs on the same inputs, the batch workload (general-
relativity grid contractions plus 2000 random contractions in one persistent
graph-replayed launch), the memory-bound kernels' HBM rates, and the oracle
timed on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-split] [--no-batch]
                       [--precision-workload]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--v", type=int, default=128)
    ap.add_argument("--o", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the CPU sample")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision runs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch workload and memory-bound kernels")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device copy (reference for hardware byte counters)")
    ap.add_argument("--precision-workload", action="store_true",
                    help="also run the precision workload (v=192, o=48, N(0,1)*10^U(-3,3) inputs)")
    return ap.parse_args()


GETT_SOURCES = [os.path.join(ROOT, "paper_1307_2100_amd", "csrc", f) for f in ("gett_f64.hip", "gett_tile.hpp")]


def sha_of(paths):
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_srcs):
    """HBM traffic of the dominant kernel from committed counter runs, valid
    only while the kernel source is unchanged since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_gett_f64_cc_a.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha") != sha_of(kernel_srcs):
        return None
    return rec.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1307_2100_amd as tc
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        # plain copies of known size, 1 GiB read and 1 GiB written each: the
        # runtime's buffer copy, then an elementwise kernel (y = -x)
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        print("[bench] calibration copies: %d bytes read, %d bytes written each" % (x.numel() * 8, y.numel() * 8),
              file=sys.stderr, flush=True)
        del x, y
        torch.cuda.empty_cache()

    work = {}
    for name, spec, wid in (("cc_a", synth.workload_cc_a(args.v, args.o), 1),
                            ("cc_b", synth.workload_cc_b(args.v, args.o), 2)):
        labA, labB, labC, ext = spec
        t0 = time.time()
        A, B = synth.make_operands(wid, labA, labB, ext, kind="uniform")
        dA = torch.from_numpy(A).to(dev)
        dB = torch.from_numpy(B).to(dev)
        C = tc.empty_colmajor([ext[l] for l in labC], device=dev)
        C.zero_()
        tp = time.perf_counter()
        plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC)
        plan_ms = (time.perf_counter() - tp) * 1e3
        work[name] = dict(spec=spec, A=A, B=B, dA=dA, dB=dB, C=C, plan=plan, plan_ms=plan_ms,
                          ws=plan.workspace(dev), gen_s=time.time() - t0)
        print("[bench] %s ready: %s" % (name, plan.info.as_dict()), file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()

    def step(evs=None):
        for name in ("cc_a", "cc_b"):
            w = work[name]
            if evs is not None:
                evs[name][0].record(stream)
            w["plan"].execute(w["dA"], w["dB"], w["C"], 1.0, 0.0, stream=stream, workspace=w["ws"])
            if evs is not None:
                evs[name][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: exactly K steps between two device-wide synchronisations
    per = {n: [] for n in work}
    evlist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        evs = {n: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for n in work}
        step(evs)
        evlist.append(evs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for evs in evlist:
        for n in work:
            per[n].append(evs[n][0].elapsed_time(evs[n][1]))

    flops_step = sum(w["plan"].info.flops for w in work.values())
    value = flops_step * args.steps / wall / 1e9

    # accuracy on sampled outputs against the compensated oracle (outside the timed region)
    import oracle
    errs = {}
    for name, w in work.items():
        labA, labB, labC, ext = w["spec"]
        shape = [ext[l] for l in labC]
        g = np.random.default_rng(11)
        idx = np.stack([g.integers(0, e, 512) for e in shape], axis=1)
        s, a = oracle.contract_entries(w["A"], labA, w["B"], labB, labC, idx)
        got = w["C"].cpu().numpy()[tuple(idx.T)]
        errs[name] = float(np.max(np.abs(got - s) / a))

    per_contraction = {}
    for name, w in work.items():
        ms = float(np.mean(per[name]))
        info = w["plan"].info
        per_contraction[name] = {
            "ms": round(ms, 4), "tflops": round(info.flops / ms / 1e9, 3),
            "frac_fp64_peak": round(info.flops / ms / 1e9 / FP64_PEAK_TFLOPS, 4),
            "paper_class": info.paper_class, "recipe": tc.RECIPE_NAMES[info.recipe], "tile_id": info.tile_id,
            "M": info.M, "N": info.N, "K": info.K, "plan_create_ms": round(w["plan_ms"], 3),
            "max_componentwise_error_sampled": errs[name],
        }

    # dominant kernel: the GEMM launch of contraction (a)
    ia = work["cc_a"]["plan"].info
    ms_a = float(np.mean(per["cc_a"]))
    achieved = ia.flops / (ms_a * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": traffic_from_profile(GETT_SOURCES),
                "kernel": "%s (contraction a)" % ("gett_f64_dma_kernel" if ia.copy_fed else "gett_f64_kernel"),
                "algorithmic_flops_per_launch": ia.flops,
                "algorithmic_bytes_per_launch": ia.bytes}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(work["cc_a"], args.cpu_seconds)

    split = None
    if not args.no_split:
        split = split_runs(work, max(3, min(args.steps, 10)))

    batch = memory = modes = None
    if not args.no_batch:
        batch = batch_runs()
        memory = memory_bound_runs()
        modes = timing_modes_runs()

    precision_workload = None
    if args.precision_workload:
        for w in work.values():
            w["plan"].close()
            for key in ("dA", "dB", "C", "ws"):
                w[key] = None
        torch.cuda.empty_cache()
        precision_workload = precision_runs(args)

    out = {
        "metric": "contraction GFLOP/s (FP64 vs split-BF16) at stated rel. error; % MFMA peak",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded uniform[-1,1], column-major FP64)",
        "config": {"workload": "coupled-cluster contractions (a) abcd,cdij->abij and (b) akic,kbcj->abij, "
                               "v=%d o=%d, FP64" % (args.v, args.o),
                   "v": args.v, "o": args.o, "flops_per_step": flops_step},
        "frac_fp64_peak": round(value / 1e3 / FP64_PEAK_TFLOPS, 4),
        "max_componentwise_error": max(errs.values()),
        "per_contraction": per_contraction,
        "split_precision": split,
        "precision_workload": precision_workload,
        "batch_workload": batch,
        "memory_bound_kernels": memory,
        "warm_cold_graph": modes,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    for w in work.values():
        w["plan"].close()


def sampled_error(A, labA, B, labB, labC, ext, C_dev, n=512, seed=11):
    """Max componentwise error of C_dev against the compensated oracle on n
    sampled output entries (each computed in full by the oracle)."""
    import numpy as np

    import oracle
    shape = [ext[l] for l in labC]
    g = np.random.default_rng(seed)
    idx = np.stack([g.integers(0, e, n) for e in shape], axis=1)
    s, a = oracle.contract_entries(A, labA, B, labB, labC, idx)
    got = C_dev.cpu().numpy()[tuple(idx.T)]
    return float(np.max(np.abs(got - s) / a))


def time_plan(plan, dA, dB, C, reps, stream):
    import numpy as np
    import torch
    ws = plan.workspace(C.device)
    plan.execute(dA, dB, C, 1.0, 0.0, stream=stream, workspace=ws)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.execute(dA, dB, C, 1.0, 0.0, stream=stream, workspace=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.mean(ms))


def split_runs(work, reps):
    """Split-precision (BF16 and FP8 digits, INT8 residues) on the same inputs:
    time (HIP events around each tc_execute, split pass included) and sampled
    error."""
    import torch

    import paper_1307_2100_amd as tc
    stream = torch.cuda.current_stream()
    out = {}
    for prec in ("split_bf16", "split_fp8", "crt_int8"):
        res = {}
        for name, w in work.items():
            labA, labB, labC, ext = w["spec"]
            C = tc.empty_colmajor([ext[l] for l in labC], device=w["C"].device)
            plan = tc.Plan.for_tensors(w["dA"], labA, w["dB"], labB, C, labC, precision=prec)
            ms = time_plan(plan, w["dA"], w["dB"], C, reps, stream)
            err = sampled_error(w["A"], labA, w["B"], labB, labC, ext, C)
            res[name] = {"ms": round(ms, 4), "effective_tflops": round(plan.info.flops / ms / 1e9, 3),
                         "digits": plan.info.split_slices, "bits": plan.info.split_bits,
                         "max_componentwise_error_sampled": err,
                         "workspace_gb": round(plan.info.workspace_bytes / 1e9, 3)}
            plan.close()
            del C
        out[prec] = res
    return out


def precision_runs(args):
    """The precision workload: both coupled-cluster contractions at v=192,
    o=48 with N(0,1) inputs scaled per last-index slice by 10^U(-3,3), in FP64,
    split BF16, split FP8 and INT8 residues, each with its sampled error
    against the oracle."""
    import torch

    import paper_1307_2100_amd as tc
    import synth
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    for name, spec, wid in (("cc_a", synth.workload_cc_a(192, 48), 21), ("cc_b", synth.workload_cc_b(192, 48), 22)):
        labA, labB, labC, ext = spec
        A, B = synth.make_operands(wid, labA, labB, ext, kind="scaled_normal")
        dA = torch.from_numpy(A).to(dev)
        dB = torch.from_numpy(B).to(dev)
        C = tc.empty_colmajor([ext[l] for l in labC], device=dev)
        res = {}
        for prec in ("f64", "split_bf16", "split_fp8", "crt_int8"):
            plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC, precision=prec)
            ms = time_plan(plan, dA, dB, C, 3, stream)
            err = sampled_error(A, labA, B, labB, labC, ext, C, n=256)
            res[prec] = {"ms": round(ms, 3), "effective_tflops": round(plan.info.flops / ms / 1e9, 3),
                         "max_componentwise_error_sampled": err,
                         "digits": plan.info.split_slices if prec != "f64" else None,
                         "bits": plan.info.split_bits if prec != "f64" else None}
            plan.close()
            torch.cuda.empty_cache()
        res["speedup_split_bf16_vs_f64"] = round(res["f64"]["ms"] / res["split_bf16"]["ms"], 3)
        res["speedup_crt_int8_vs_f64"] = round(res["f64"]["ms"] / res["crt_int8"]["ms"], 3)
        out[name] = res
        print("[bench] precision workload %s: %s" % (name, res), file=sys.stderr, flush=True)
        del dA, dB, C
        torch.cuda.empty_cache()
    return out


def _dev_uniform(tc, torch, shape, gen):
    t = tc.empty_colmajor(list(shape), device="cuda")
    t.uniform_(-1.0, 1.0, generator=gen)
    return t


def _events_ms(fn, reps):
    """Mean time of fn() over reps back-to-back calls, HIP events on the current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batch_runs(n_random=2000, reps=10):
    """The batch workload: R[a,b] = T[a,c,b,d] g[c,d] and S[a,b,c] = G[a,b,d] V[d,c]
    on a 128^3 grid (every extent 4) plus n_random contractions of rank 3-6,
    extents uniform in [4, 64], random storage orders and contracted sets, in
    one persistent launch replayed from a graph with the autotuned tile
    configuration.  Roofline: the sum over contractions of max(flops / FP64
    peak, bytes / HBM peak) against the measured time."""
    import numpy as np
    import torch

    import oracle
    import paper_1307_2100_amd as tc
    import synth
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1307)
    g = np.random.default_rng(1307)
    specs = [synth.workload_gr_r(), synth.workload_gr_s()]
    specs += [synth.random_contraction(g, rank_range=(3, 6), ext_range=(4, 64), max_elems=1 << 20)
              for _ in range(n_random)]
    ents = []
    for la, lb, lc, ext in specs:
        A = _dev_uniform(tc, torch, synth.shape_of(la, ext), gen)
        B = _dev_uniform(tc, torch, synth.shape_of(lb, ext), gen)
        C = tc.empty_colmajor(list(synth.shape_of(lc, ext)))
        C.zero_()
        ents.append((la, lb, lc, ext, A, B, C, tc.Plan.for_tensors(A, la, B, lb, C, lc)))
    flops = sum(e[7].info.flops for e in ents)
    nbytes = sum(e[7].info.bytes for e in ents)
    ideal_ms = sum(max(e[7].info.flops / FP64_PEAK_TFLOPS / 1e9, e[7].info.bytes / HBM_PEAK_GBS / 1e6)
                   for e in ents)
    # each grid contraction alone (slab kernel)
    gr = {}
    for name, e in zip(("gr_r", "gr_s"), ents[:2]):
        ms = _events_ms(lambda: e[7].execute(e[4], e[5], e[6]), reps)
        gr[name] = {"ms": round(ms, 4), "gb_s": round(e[7].info.bytes / ms / 1e6, 1),
                    "frac_hbm_peak": round(e[7].info.bytes / ms / 1e6 / HBM_PEAK_GBS, 4),
                    "kernel": tc.KERNEL_NAMES[e[7].info.kernel]}
    print("[bench] batch workload: %d plans built" % len(ents), file=sys.stderr, flush=True)
    batch = tc.Batch([e[7] for e in ents])
    As, Bs, Cs = [e[4] for e in ents], [e[5] for e in ents], [e[6] for e in ents]
    t0 = time.perf_counter()
    best, _ = batch.autotune(As, Bs, Cs)
    tune_s = time.perf_counter() - t0
    batch.set_options(best, 1)
    batch.bind(As, Bs, Cs)
    ms = _events_ms(batch.run, reps)
    q = batch.query()
    print("[bench] batch workload: config %d, %.3f ms per execution" % (best, ms), file=sys.stderr, flush=True)
    # sampled check of a few entries of the grid contractions and of some random ones
    err = 0.0
    checked = [e for e in ents if e[2]][:12]
    for e in checked:
        la, lb, lc, ext, A, B, C = e[:7]
        shape = [ext[l] for l in lc]
        gi = np.random.default_rng(5)
        idx = np.stack([gi.integers(0, x, 64) for x in shape], axis=1)
        s, a = oracle.contract_entries(A.cpu().numpy(), la, B.cpu().numpy(), lb, lc, idx)
        got = C.cpu().numpy()[tuple(idx.T)]
        err = max(err, float(np.max(np.abs(got - s) / np.where(a > 0, a, 1.0))))
    batch.close()
    for e in ents:
        e[7].close()
    del ents, As, Bs, Cs
    torch.cuda.empty_cache()
    return {"contractions": len(specs), "tasks": q["ntasks"], "tile_config": best, "autotune_s": round(tune_s, 2),
            "ms": round(ms, 4), "gflops": round(flops / ms / 1e6, 1), "gb_s": round(nbytes / ms / 1e6, 1),
            "ideal_ms": round(ideal_ms, 4), "frac_roofline": round(ideal_ms / ms, 4),
            "max_componentwise_error_sampled": err, "grid_contractions_alone": gr}


def timing_modes_runs(reps=10, graph_reps=20):
    """The small 3-D contraction C[i,j,m] = A[i,k,m] B[k,j] (extents 64) and
    the two grid contractions, each timed three ways with HIP events on the
    current stream: warm (median of reps back-to-back-launched calls, each
    bracketed by its own events), cold (a 1 GiB buffer is written before
    each call, which evicts the 256 MB last-level cache; the call alone is
    timed) and graph replay (the call captured once in a HIP graph, mean
    over graph_reps replays).  Every replay's output is compared with the
    eager result."""
    import numpy as np
    import torch

    import paper_1307_2100_amd as tc
    import synth
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1308)
    stream = torch.cuda.current_stream()
    scratch = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    out = {}
    for name, (la, lb, lc, ext) in (("c0_3d_64", synth.workload_3d_matrix(64)), ("gr_r", synth.workload_gr_r()),
                                    ("gr_s", synth.workload_gr_s())):
        A = _dev_uniform(tc, torch, synth.shape_of(la, ext), gen)
        B = _dev_uniform(tc, torch, synth.shape_of(lb, ext), gen)
        C = tc.empty_colmajor(list(synth.shape_of(lc, ext)))
        plan = tc.Plan.for_tensors(A, la, B, lb, C, lc)
        ws = plan.workspace(C.device)
        run = lambda: plan.execute(A, B, C, stream=stream, workspace=ws)  # noqa: E731
        run()
        torch.cuda.synchronize()
        eager = C.clone()
        warm, cold = [], []
        for k in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run()
            e1.record(stream)
            torch.cuda.synchronize()
            warm.append(e0.elapsed_time(e1))
        for k in range(reps):
            scratch.fill_(float(k))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run()
            e1.record(stream)
            torch.cuda.synchronize()
            cold.append(e0.elapsed_time(e1))
        # graph: captured on a side stream, replayed on the current one
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                plan.execute(A, B, C, stream=side, workspace=ws)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        mismatch = 0.0
        for _ in range(3):
            C.zero_()
            g.replay()
            torch.cuda.synchronize()
            mismatch = max(mismatch, float((C - eager).abs().max()))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(graph_reps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        info = plan.info
        print("[bench] %s: warm %.4f ms, cold %.4f ms, graph replay %.4f ms" % (
            name, float(np.median(warm)), float(np.median(cold)), e0.elapsed_time(e1) / graph_reps),
            file=sys.stderr, flush=True)
        out[name] = {"warm_ms_median": round(float(np.median(warm)), 4),
                     "cold_ms_median": round(float(np.median(cold)), 4),
                     "graph_replay_ms": round(e0.elapsed_time(e1) / graph_reps, 4),
                     "graph_replay_max_abs_diff_vs_eager": mismatch,
                     "kernel": tc.KERNEL_NAMES[info.kernel], "flops": info.flops, "bytes": info.bytes}
        del g
        plan.close()
        del A, B, C, eager
    del scratch
    torch.cuda.empty_cache()
    return out


def memory_bound_runs(reps=20):
    """HBM rates of the memory-bound kernels on large operands: the LDS-tiled
    permute (COPY step), GEMV with lanes along the outputs and along k, DOT
    with segmented sums.  Bytes are the algorithmic ones (each operand read
    once, the output written once)."""
    import torch

    import paper_1307_2100_amd as tc
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    out = {}
    # permute: 256^3 x 8 tensor (1 GiB), its first two modes exchanged in storage
    X = _dev_uniform(tc, torch, (256, 256, 256, 8), gen)
    Y = torch.empty(X.numel(), dtype=torch.float64, device="cuda")
    strides = [256, 1, 256 * 256, 256 ** 3]
    ms = _events_ms(lambda: tc.permute(X, strides, Y), reps)
    out["permute"] = {"ms": round(ms, 4), "gb_s": round(16.0 * X.numel() / ms / 1e6, 1),
                      "frac_hbm_peak": round(16.0 * X.numel() / ms / 1e6 / HBM_PEAK_GBS, 4)}
    print("[bench] permute: %s" % out["permute"], file=sys.stderr, flush=True)
    del X, Y
    cases = {
        "gemv_lanes_over_outputs": ("ik", "k", "i", {"i": 32768, "k": 8192}),
        "gemv_lanes_over_k": ("ki", "k", "i", {"k": 32768, "i": 8192}),
        "dot": ("k", "k", "", {"k": 1 << 27}),
    }
    for name, (la, lb, lc, ext) in cases.items():
        A = _dev_uniform(tc, torch, [ext[l] for l in la], gen)
        B = _dev_uniform(tc, torch, [ext[l] for l in lb], gen)
        C = tc.empty_colmajor([ext[l] for l in lc])
        plan = tc.Plan.for_tensors(A, la, B, lb, C, lc)
        ws = plan.workspace(C.device)
        ms = _events_ms(lambda: plan.execute(A, B, C, workspace=ws), reps)
        out[name] = {"ms": round(ms, 4), "gb_s": round(plan.info.bytes / ms / 1e6, 1),
                     "frac_hbm_peak": round(plan.info.bytes / ms / 1e6 / HBM_PEAK_GBS, 4),
                     "kernel": tc.KERNEL_NAMES[plan.info.kernel]}
        plan.close()
        del A, B, C
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, target_s):
    """The oracle (plain FP64 nested loop, all host threads it uses) on a
    bounded sample of contraction (a): whole output entries, each a full
    K-long sum, timed and scaled to GFLOP/s."""
    import numpy as np

    import oracle
    labA, labB, labC, ext = w["spec"]
    shape = [ext[l] for l in labC]
    K = w["plan"].info.K
    g = np.random.default_rng(3)
    n = 64
    while True:
        idx = np.stack([g.integers(0, e, n) for e in shape], axis=1)
        t0 = time.perf_counter()
        oracle.contract_entries(w["A"], labA, w["B"], labB, labC, idx, compensated=False, with_abs=False)
        dt = time.perf_counter() - t0
        if dt >= target_s * 0.5 or n >= 1 << 22:
            break
        n = int(n * min(16.0, max(2.0, target_s / max(dt, 1e-3))))
    gflops = 2.0 * K * n / dt / 1e9
    return {"value": round(gflops, 4), "unit": "GFLOP/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "%d output entries of contraction (a) (each a %d-term sum), %.1f s" % (n, K, dt)}


if __name__ == "__main__":
    main()
