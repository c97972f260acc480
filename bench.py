"""Benchmark: FP64 and split-precision contraction throughput on the
coupled-cluster precision workload.

One step = one pass of the hot path over one batch of input: the two
coupled-cluster contractions of the paper's Sec. 4.2 at v = 192, o = 48,
  (a) C[a,b,i,j] = sum_{c,d} A[a,b,c,d] B[c,d,i,j]   (paper class 3.2, direct GEMM)
  (b) C[a,b,i,j] = sum_{k,c} A[a,k,i,c] B[k,b,c,j]   (class 3.2 with un-fusable index groups)
each through tc_execute on plans built once, in FP64 (the headline value).
Inputs are seeded synthetic FP64 tensors, N(0,1) with every slice along the
last mode scaled by 10^U(-3,3), column-major, resident in HBM before the timed
region.  The same step runs as split BF16 digits (the compared form), split
FP8 digits and INT8 residues, each timed and each result's error stated
against the compensated oracle on a stratified sample of outputs (one row
per 128-row block times one column per 10-column block, about 66k entries,
plus two full output slabs).  Prints one JSON line.

Besides the step, the JSON line carries the same contractions at v = 128,
o = 32 (uniform inputs), the batch workload (general-relativity grid
contractions plus 2000 random contractions in one persistent graph-replayed
launch), the memory-bound kernels' HBM rates, and the oracle timed on the
host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-split] [--no-batch]
                       [--no-c1] [--profile PRECISION]
"""
import argparse
import concurrent.futures
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
PRECISIONS = ("f64", "split_bf16", "split_fp8", "crt_int8")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--v", type=int, default=192)
    ap.add_argument("--o", type=int, default=48)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the CPU sample")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision runs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch workload and memory-bound kernels")
    ap.add_argument("--no-c1", action="store_true", help="skip the v=128, o=32 workload")
    ap.add_argument("--profile", choices=PRECISIONS, default=None,
                    help="only build the workload and run the timed steps in this precision (for profilers)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device copy (reference for hardware byte counters)")
    return ap.parse_args()


GETT_SOURCES = [os.path.join(ROOT, "paper_1307_2100_amd", "csrc", f) for f in ("gett_f64.hip", "gett_tile.hpp")]
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_gett_f64_dma_cc_a_v192_o48.json")


def sha_of(paths):
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_srcs, workload):
    """HBM traffic of the dominant kernel from committed counter runs, valid
    only while the kernel source is unchanged since they were taken and for
    the workload they were taken on."""
    if not os.path.exists(TRAFFIC_RECORD):
        return None
    rec = json.load(open(TRAFFIC_RECORD))
    if rec.get("kernel_source_sha") != sha_of(kernel_srcs) or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def reference_entries(A, labA, B, labB, labC, idx):
    """Compensated oracle sums and |A||B| sums of the sampled entries."""
    import oracle
    return oracle.contract_entries(A, labA, B, labB, labC, idx)


def sample_indices(shape, seed):
    """Stratified grid over C (rows: the first two modes, columns: the rest;
    one row per block of 128, one column per block of 10), then two full
    slabs C[a0, b0, :, :] of the last two modes."""
    import numpy as np

    import synth
    grid = synth.stratified_entries(shape, 2, 128, 10, seed)
    g = np.random.default_rng(seed + 1)
    slabs = []
    for _ in range(2):
        r = [int(g.integers(0, e)) for e in shape[:2]]
        cols = synth.unravel_colmajor(np.arange(int(np.prod(shape[2:]))), shape[2:])
        slabs.append(np.concatenate([np.tile(np.array(r, dtype=np.int64), (cols.shape[0], 1)), cols], axis=1))
    return np.concatenate([grid] + slabs, axis=0)


def gather(C, idx):
    """Entries of a dense (column-major) device tensor at the sampled
    multi-indices, as host FP64."""
    import numpy as np
    import torch
    off = np.zeros(idx.shape[0], dtype=np.int64)
    span = 1
    for d, (e, st) in enumerate(zip(C.shape, C.stride())):
        off += idx[:, d] * st
        span += (e - 1) * st
    assert span == C.numel(), "gather expects a dense output tensor"
    flat = torch.as_strided(C, (C.numel(),), (1,))
    return flat.index_select(0, torch.from_numpy(off).to(C.device)).cpu().numpy()


def errors(got, ref):
    """(max componentwise error, normwise error) of sampled entries against the
    compensated oracle: |got - s| / (|A||B|) per entry and max|got - s| / max|s|."""
    import numpy as np
    s, a = ref
    comp = float(np.max(np.abs(got - s) / np.where(a > 0, a, 1.0)))
    norm = float(np.max(np.abs(got - s)) / max(float(np.max(np.abs(s))), 1e-300))
    return comp, norm


def build_workload(tc, torch, synth, v, o, kind, wid_a, wid_b, dev):
    work = {}
    for name, spec, wid in (("cc_a", synth.workload_cc_a(v, o), wid_a), ("cc_b", synth.workload_cc_b(v, o), wid_b)):
        labA, labB, labC, ext = spec
        t0 = time.time()
        A, B = synth.make_operands(wid, labA, labB, ext, kind=kind)
        gen_s = time.time() - t0
        dA = torch.from_numpy(A).to(dev)
        dB = torch.from_numpy(B).to(dev)
        C = tc.empty_colmajor([ext[l] for l in labC], device=dev)
        C.zero_()
        work[name] = dict(spec=spec, A=A, B=B, dA=dA, dB=dB, C=C, gen_s=gen_s)
        log("%s v=%d o=%d inputs ready (%.1f s to generate)" % (name, v, o, gen_s))
    return work


def time_steps(work, plans, steps, warmup, stream):
    """Warm-up, then exactly `steps` steps (every contraction once) between two
    device synchronisations; HIP events around each tc_execute on `stream`.
    Returns (wall seconds, {name: [ms per execution]})."""
    import torch

    def step(evs=None):
        for name in work:
            w, pl = work[name], plans[name]
            if evs is not None:
                evs[name][0].record(stream)
            pl["plan"].execute(w["dA"], w["dB"], pl["C"], 1.0, 0.0, stream=stream, workspace=pl["ws"])
            if evs is not None:
                evs[name][1].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evlist = []
    t0 = time.perf_counter()
    for _ in range(steps):
        evs = {n: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for n in work}
        step(evs)
        evlist.append(evs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = {n: [evs[n][0].elapsed_time(evs[n][1]) for evs in evlist] for n in work}
    return wall, per


def make_plans(tc, work, precision, dev, reuse_c=False):
    plans = {}
    for name, w in work.items():
        labA, labB, labC, ext = w["spec"]
        C = w["C"] if reuse_c else tc.empty_colmajor([ext[l] for l in labC], device=dev)
        plan = tc.Plan.for_tensors(w["dA"], labA, w["dB"], labB, C, labC, precision=precision)
        plans[name] = dict(plan=plan, C=C, ws=plan.workspace(dev))
    return plans


def close_plans(plans):
    import torch
    for pl in plans.values():
        pl["plan"].close()
        pl["ws"] = pl["C"] = None
    torch.cuda.empty_cache()


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
        log("calibration copies: %d bytes read, %d bytes written each" % (x.numel() * 8, y.numel() * 8))
        del x, y
        torch.cuda.empty_cache()

    v, o = args.v, args.o
    workload = ("coupled-cluster contractions (a) abcd,cdij->abij and (b) akic,kbcj->abij, v=%d o=%d, "
                "N(0,1)*10^U(-3,3) per last-index slice" % (v, o))
    work = build_workload(tc, torch, synth, v, o, "scaled_normal", 21, 22, dev)
    stream = torch.cuda.current_stream()

    if args.profile:
        plans = make_plans(tc, work, args.profile, dev, reuse_c=True)
        wall, per = time_steps(work, plans, args.steps, args.warmup, stream)
        log("profile run %s: %s ms per step" % (args.profile, {n: round(float(np.mean(x)), 3) for n, x in per.items()}))
        close_plans(plans)
        return

    # the oracle's reference for the sampled entries runs on the host while the GPU is timed
    idx = {n: sample_indices([w["spec"][3][l] for l in w["spec"][2]], 31 + i) for i, (n, w) in enumerate(work.items())}
    pool = concurrent.futures.ThreadPoolExecutor(1)
    ref_future = {n: pool.submit(reference_entries, w["A"], w["spec"][0], w["B"], w["spec"][1], w["spec"][2], idx[n])
                  for n, w in work.items()}

    # ---- the timed region: K steps of the FP64 path
    plans = make_plans(tc, work, "f64", dev, reuse_c=True)
    for n, pl in plans.items():
        log("%s plan: %s" % (n, pl["plan"].info.as_dict()))
    wall, per = time_steps(work, plans, args.steps, args.warmup, stream)
    flops = {n: pl["plan"].info.flops for n, pl in plans.items()}
    flops_step = sum(flops.values())
    value = flops_step * args.steps / wall / 1e9
    log("FP64 step: %.3f ms, %.1f GFLOP/s" % (wall / args.steps * 1e3, value))
    results = {"f64": dict(step_ms=wall / args.steps * 1e3, per={n: float(np.mean(x)) for n, x in per.items()},
                           got={n: gather(pl["C"], idx[n]) for n, pl in plans.items()}, digits=None, bits=None)}
    ia = plans["cc_a"]["plan"].info
    infos = {n: pl["plan"].info.as_dict() for n, pl in plans.items()}
    close_plans(plans)

    # ---- split precision on the same inputs (each result timed and sampled)
    if not args.no_split:
        reps = max(3, min(args.steps, 5))
        for prec in PRECISIONS[1:]:
            plans = make_plans(tc, work, prec, dev)
            w_s, per_s = time_steps(work, plans, reps, 1, stream)
            results[prec] = dict(step_ms=sum(float(np.mean(x)) for x in per_s.values()),
                                 per={n: float(np.mean(x)) for n, x in per_s.items()},
                                 got={n: gather(pl["C"], idx[n]) for n, pl in plans.items()},
                                 digits=plans["cc_a"]["plan"].info.split_slices,
                                 bits={n: pl["plan"].info.split_bits for n, pl in plans.items()},
                                 workspace_gb={n: round(pl["plan"].info.workspace_bytes / 1e9, 3)
                                               for n, pl in plans.items()})
            log("%s step: %.3f ms" % (prec, results[prec]["step_ms"]))
            close_plans(plans)

    refs = {n: f.result() for n, f in ref_future.items()}
    pool.shutdown()
    summary = {}
    for prec, r in results.items():
        per_c = {}
        for n in work:
            comp, norm = errors(r["got"][n], refs[n])
            per_c[n] = {"ms": round(r["per"][n], 4), "effective_tflops": round(flops[n] / r["per"][n] / 1e9, 3),
                        "max_componentwise_error": comp, "normwise_error": norm}
            if prec != "f64":
                per_c[n]["bits"] = r["bits"][n]
                per_c[n]["workspace_gb"] = r["workspace_gb"][n]
        summary[prec] = {"step_ms": round(r["step_ms"], 4), "gflops": round(flops_step / r["step_ms"] / 1e6, 1),
                         "speedup_vs_f64": round(results["f64"]["step_ms"] / r["step_ms"], 3),
                         "digits_or_moduli": r["digits"],
                         "max_componentwise_error": max(c["max_componentwise_error"] for c in per_c.values()),
                         "per_contraction": per_c}
        log("%s: %s" % (prec, summary[prec]))
    fp64_err = summary["f64"]["max_componentwise_error"]

    # dominant kernel: the GEMM launch of contraction (a)
    ms_a = results["f64"]["per"]["cc_a"]
    achieved = ia.flops / (ms_a * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": traffic_from_profile(GETT_SOURCES, "cc_a v=%d o=%d" % (v, o)),
                "kernel": "%s (contraction a, v=%d o=%d)" % ("gett_f64_dma_kernel" if ia.copy_fed else "gett_f64_kernel",
                                                            v, o),
                "algorithmic_flops_per_launch": ia.flops, "algorithmic_bytes_per_launch": ia.bytes}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(work["cc_a"], ia.K, args.cpu_seconds, flops_step)

    n_samples = {n: int(idx[n].shape[0]) for n in work}
    for w in work.values():
        for key in ("dA", "dB", "C"):
            w[key] = None
    del work
    torch.cuda.empty_cache()

    c1 = None
    if not args.no_c1:
        c1 = c1_runs(args, dev, stream)
    batch = memory = modes = None
    if not args.no_batch:
        batch = batch_runs()
        memory = memory_bound_runs()
        modes = timing_modes_runs()

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
        "data": "synthetic (seeded N(0,1) scaled per last-index slice by 10^U(-3,3), column-major FP64)",
        "config": {"workload": workload, "v": v, "o": o, "flops_per_step": flops_step},
        "frac_fp64_peak": round(value / 1e3 / FP64_PEAK_TFLOPS, 4),
        "max_componentwise_error": fp64_err,
        "split_bf16_gflops": summary.get("split_bf16", {}).get("gflops"),
        "split_bf16_vs_f64": summary.get("split_bf16", {}).get("speedup_vs_f64"),
        "split_bf16_max_componentwise_error": summary.get("split_bf16", {}).get("max_componentwise_error"),
        "results": summary,
        "error_sample": {"entries_per_contraction": n_samples, "reference": "oracle, compensated (Dot2) sums",
                         "design": "one row per 128-row block x one column per 10-column block of C "
                                   "(rows = first two modes), plus two full slabs C[a0,b0,:,:]"},
        "plans": infos,
        "c1_workload": c1,
        "batch_workload": batch,
        "memory_bound_kernels": memory,
        "warm_cold_graph": modes,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def c1_runs(args, dev, stream):
    """The same two contractions at v = 128, o = 32 on uniform [-1, 1] inputs:
    FP64 step and the split forms, each with its error on 512 random outputs."""
    import numpy as np

    import oracle
    import paper_1307_2100_amd as tc
    import synth
    import torch
    work = build_workload(tc, torch, synth, 128, 32, "uniform", 1, 2, dev)
    out = {}
    flops = None
    for prec in PRECISIONS if not args.no_split else PRECISIONS[:1]:
        plans = make_plans(tc, work, prec, dev)
        flops = {n: pl["plan"].info.flops for n, pl in plans.items()}
        steps = args.steps if prec == "f64" else 5
        wall, per = time_steps(work, plans, steps, 2, stream)
        res = {"step_ms": round(sum(float(np.mean(x)) for x in per.values()), 4)}
        for n, pl in plans.items():
            labA, labB, labC, ext = work[n]["spec"]
            shape = [ext[l] for l in labC]
            g = np.random.default_rng(11)
            idx = np.stack([g.integers(0, e, 512) for e in shape], axis=1)
            ref = oracle.contract_entries(work[n]["A"], labA, work[n]["B"], labB, labC, idx)
            comp, _ = errors(gather(pl["C"], idx), ref)
            res[n] = {"ms": round(float(np.mean(per[n])), 4),
                      "effective_tflops": round(flops[n] / float(np.mean(per[n])) / 1e9, 3),
                      "max_componentwise_error_sampled": comp, "tile_id": pl["plan"].info.tile_id,
                      "copy_fed": pl["plan"].info.copy_fed}
        res["gflops"] = round(sum(flops.values()) / res["step_ms"] / 1e6, 1)
        out[prec] = res
        log("c1 %s: %s" % (prec, res))
        close_plans(plans)
    for w in work.values():
        for key in ("dA", "dB", "C"):
            w[key] = None
    torch.cuda.empty_cache()
    out["workload"] = "coupled-cluster (a)+(b), v=128 o=32, uniform[-1,1]"
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
    the two grid contractions, timed with HIP events on the current stream:
    warm (median of reps calls, each bracketed by its own events), cold (a
    1 GiB buffer is written before each call, which evicts the 256 MB
    last-level cache; the call alone is timed), device time of one eager call
    and of one replay of the call captured in a HIP graph (the stream kept
    busy before each, so the events time execution rather than submission),
    and the per-call time of graph_reps back-to-back replays.  Every replay's
    output is compared with the eager result."""
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
        # device time of one call: the stream is first kept busy by a sleep
        # kernel (about 0.2 ms), so the call is already queued when its start
        # event fires and the events bracket its execution, not its submission
        def device_ms(fn):
            ts = []
            for _ in range(reps):
                torch.cuda._sleep(500000)
                d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                d0.record(stream)
                fn()
                d1.record(stream)
                torch.cuda.synchronize()
                ts.append(d0.elapsed_time(d1))
            return float(np.median(ts))
        eager_dev = device_ms(run)
        graph_dev = device_ms(g.replay)
        # back-to-back replays: per-call time when the host submits them in a row
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(graph_reps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        info = plan.info
        print("[bench] %s: warm %.4f ms, cold %.4f ms, device time eager %.4f ms, graph replay %.4f ms, "
              "back-to-back replays %.4f ms each" % (name, float(np.median(warm)), float(np.median(cold)), eager_dev,
                                                    graph_dev, e0.elapsed_time(e1) / graph_reps),
              file=sys.stderr, flush=True)
        out[name] = {"warm_ms_median": round(float(np.median(warm)), 4),
                     "cold_ms_median": round(float(np.median(cold)), 4),
                     "device_ms_eager_median": round(eager_dev, 4),
                     "device_ms_graph_replay_median": round(graph_dev, 4),
                     "back_to_back_graph_replay_ms": round(e0.elapsed_time(e1) / graph_reps, 4),
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


def cpu_baseline(w, K, target_s, flops_step):
    """The oracle (plain FP64 nested loop, all host threads it uses) on a
    bounded sample of contraction (a): whole output entries, each a full
    K-long sum, timed and scaled to GFLOP/s; the full step's oracle time is
    extrapolated from that rate."""
    import numpy as np

    import oracle
    labA, labB, labC, ext = w["spec"]
    shape = [ext[l] for l in labC]
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
            "sample": "%d random output entries of contraction (a) (each a %d-term plain FP64 sum), %.1f s; "
                      "the whole step (a)+(b) would take %.0f s at this rate (extrapolated)"
                      % (n, K, dt, flops_step / (gflops * 1e9)),
            "extrapolated_step_s": round(flops_step / (gflops * 1e9), 1)}


if __name__ == "__main__":
    main()
