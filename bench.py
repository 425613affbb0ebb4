#!/usr/bin/env python3
"""Benchmark: DMK Stokeslet sum on one MI355X.

A step is one pass of the whole path over the benchmark input: plan (bounding
box, Morton sort, adaptive level-restricted octree, neighbour lists, device
buffers; the per-tolerance tables are cached per process) followed by one
evaluation (all far-field passes, near field, finalize), and the release of
the previous step's plan.  Inputs are resident in HBM before timing starts.
Steps are pipelined: plans are built with DMK_FLAG_CONCURRENT_PLAN, so the
host part of step k+1's plan overlaps step k's evaluation on the GPU.

Prints one JSON line (see the field list at the end of main()).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Stokeslet targets/sec at 1e6 pts, 1e-6 rel L2: FP64 vs mixed/batched"
PEAK_FP64_VECTOR_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz


def nd_bucket(deg_P: int, deg_Q: int) -> int:
    """Compiled Horner degree the near-field kernel is instantiated with."""
    d = max(deg_P, deg_Q) + 1  # coefficient count
    return 14 if d <= 14 else 18 if d <= 18 else 21 if d <= 21 else 24


def near_flops_per_pair(deg_P: int, deg_Q: int) -> int:
    """Algorithmic flops of one residual-kernel pair: 33 for the difference,
    r^2, s, y.f, the two scalar coefficients and the update, 2 d for each
    degree-d radial polynomial (Horner, one multiply-add per degree), and the
    reciprocal square root counted as one."""
    return 33 + 2 * (deg_P + deg_Q) + 1


def near_profile_ms(config: str, precision: str, kernel: str, leaf_size: int, near_lanes: int):
    """Average duration (ms) of the near-field kernel in the committed
    rocprofv3 kernel-trace summary of this workload, or None (same conditions
    as near_traffic)."""
    rec = _near_profile_record(config, precision, kernel, leaf_size, near_lanes)
    return None if rec is None or "avg_us" not in rec else rec["avg_us"] * 1e-3


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def near_traffic(config: str, tol: float, precision: str, kernel: str, leaf_size: int, near_lanes: int):
    """HBM bytes per launch of the near-field kernel from the committed
    rocprofv3 summary of this workload, or None when there is none, it was
    taken with another leaf size or lane split, or the near-field source
    section or the within-leaf reorder changed since the counters were taken."""
    if abs(tol - workloads_tol(config)) > 0:
        return None
    rec = _near_profile_record(config, precision, kernel, leaf_size, near_lanes)
    return None if rec is None else rec["hbm_bytes_per_launch"]


def _near_profile_record(config: str, precision: str, kernel: str, leaf_size: int, near_lanes: int):
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"k_near_{config}_{precision}_leaf{leaf_size}_lanes{near_lanes}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r'^\{"kernel".*\}$', open(path).read(), re.M)
    if not m:
        return None
    rec = json.loads(m.group(0))
    src = open(os.path.join(ROOT, "paper_2509_21471_amd", "csrc", "dmk_kernels.hip")).read()
    # the kernel's source and the within-leaf point order it runs on
    sec = near_source_section(src)
    if hashlib.sha256(sec.encode()).hexdigest() != rec["near_section_sha256"] or rec["kernel"] != kernel:
        return None
    if rec.get("leaf_size") != leaf_size or rec.get("near_lanes") != near_lanes:
        return None
    return rec


def near_source_section(src: str) -> str:
    """The near-field kernels and the within-leaf reorder they run on (the
    text whose hash a near-field profile records)."""
    lo = src.index("void launch_leaf_order(")
    return (src[src.index("// ---- near field"):src.index("// ---- finishing")]
            + src[src.index("// ---- compact point groups"):src.index("\n}\n", lo) + 3])


def workloads_tol(config: str) -> float:
    import workloads
    return workloads.CONFIGS[config]["tol"]


def batched_variant(dev, parity: bool) -> dict:
    """256 independent problems (N log-uniform in [1e3, 1e5], about 5.5e6
    points): one batched plan + evaluation against one plan + evaluation per
    problem, both in mixed precision and both in FP64, every plan with the same
    leaf size and lane split (the autotuner's choice for the batch); plus
    evaluation alone on the batched plan with and without hipGraph replay."""
    import torch

    import paper_2509_21471_amd as dmk
    import workloads
    probs = workloads.batch_problems()
    x = np.concatenate([p[0] for p in probs])
    f = np.concatenate([p[1] for p in probs])
    off = np.concatenate([[0], np.cumsum([p[0].shape[0] for p in probs])]).astype(np.int64)
    n = x.shape[0]
    xd = torch.from_numpy(x).to(dev)
    fd = torch.from_numpy(f).to(dev)
    out = torch.empty_like(fd)
    tol = 1e-6
    tune = dmk.autotune(xd, tol=tol, precision=dmk.PREC_MIXED, offsets=off)
    leaf, lanes = tune["leaf_size"], tune["near_lanes"]
    shape = {"stage_rows": tune["stage_rows"], "eval_points": tune["eval_points"]}
    res = {"workload": "batch_256", "n_problems": len(probs), "n": n, "tol": tol, "autotuned": tune,
           "leaf_policy": "every plan (batched and separate) uses the autotuned leaf size and lane split"}
    xs = [xd[off[b]:off[b + 1]] for b in range(len(probs))]
    fs = [fd[off[b]:off[b + 1]] for b in range(len(probs))]
    outs = [torch.empty_like(t) for t in fs]

    def batched_step(prec):
        p = dmk.Plan(xd, tol=tol, precision=prec, offsets=off, leaf_size=leaf, near_lanes=lanes, **shape)
        p.eval(fd, out)
        return p

    def separate_steps(prec):
        for b in range(len(probs)):
            p = dmk.Plan(xs[b], tol=tol, precision=prec, leaf_size=leaf, near_lanes=lanes, **shape)
            p.eval(fs[b], outs[b])
            p.close()

    u_b = {}
    for name, prec in (("mixed", dmk.PREC_MIXED), ("fp64", dmk.PREC_FP64)):
        batched_step(prec).close()
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            batched_step(prec).close()
        torch.cuda.synchronize()
        ms_b = (time.perf_counter() - t0) * 1e3 / reps
        u_b[name] = out.cpu().numpy()
        separate_steps(prec)  # warm the buffer cache and tables
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        separate_steps(prec)
        torch.cuda.synchronize()
        ms_s = (time.perf_counter() - t0) * 1e3
        res[name] = {"batched_ms_per_step": ms_b, "batched_targets_per_s": n / (ms_b * 1e-3),
                     "separate_ms": ms_s, "separate_targets_per_s": n / (ms_s * 1e-3),
                     "speedup_batched_vs_separate": ms_s / ms_b}
    res["mixed_over_fp64_batched_step"] = res["mixed"]["batched_ms_per_step"] / res["fp64"]["batched_ms_per_step"]
    # evaluation alone on one batched plan, eager and replayed
    evals = {}
    for graph in (False, True):
        p = dmk.Plan(xd, tol=tol, precision=dmk.PREC_MIXED, offsets=off, leaf_size=leaf, near_lanes=lanes,
                     graph=graph, **shape)
        for _ in range(2):
            p.eval(fd, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            p.eval(fd, out)
        torch.cuda.synchronize()
        evals["graph" if graph else "eager"] = (time.perf_counter() - t0) * 1e3 / 5
        p.close()
    res["mixed_eval_only_ms"] = evals
    if parity:
        import oracle
        for name in u_b:
            errs = []
            for b in range(0, len(probs), 8):
                xb, fb = probs[b]
                idx = workloads.sample_targets(xb.shape[0], 100, 5000 + b)
                errs.append(oracle.rel_l2(u_b[name][off[b]:off[b + 1]][idx], oracle.direct(xb, fb, idx)))
            res[name]["rel_l2_sampled_max"] = max(errs)
        res["mixed"]["rel_l2_vs_fp64"] = oracle.rel_l2(u_b["mixed"], u_b["fp64"])
        res["parity_sample"] = "100 targets in each of 32 problems (every 8th)"
    print(f"# batched: mixed {res['mixed']['batched_ms_per_step']:.1f} ms (separate {res['mixed']['separate_ms']:.1f}), "
          f"fp64 {res['fp64']['batched_ms_per_step']:.1f} ms (separate {res['fp64']['separate_ms']:.1f}) "
          f"for {len(probs)} problems", file=sys.stderr, flush=True)
    del xd, fd, out
    torch.cuda.empty_cache()
    return res


def copy_calibration(mib: int):
    """Three launches of a plain copy of `mib` MiB between two device buffers:
    each reads and writes exactly that many bytes of HBM."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 8, "launches": 3}), flush=True)


def multi_rhs_variant(args, dev, parity: bool) -> dict:
    """One plan on 2e6 uniform points with 32 force vectors, in mixed
    precision and in FP64: evaluation rate in target-vectors per second with
    the near field batched over 8 vectors, and the same plan with one vector
    per near-field pass."""
    import torch

    import paper_2509_21471_amd as dmk
    import workloads
    name = "uniform_2e6_rhs32"
    cfg = workloads.CONFIGS[name]
    x, f = workloads.config(name)
    n, k = x.shape[0], f.shape[0]
    xd = torch.from_numpy(x).to(dev)
    fd = torch.from_numpy(f).to(dev)
    out = torch.empty_like(fd)
    res = {"workload": name, "n": n, "n_rhs": k, "tol": cfg["tol"]}
    idx = workloads.sample_targets(n, 200, cfg["seed"])
    u_last = {}
    for pname, prec in (("mixed", dmk.PREC_MIXED), ("fp64", dmk.PREC_FP64)):
        r = {}
        for batch in (8, 1):
            plan = dmk.Plan(xd, tol=cfg["tol"], rhs_batch=batch, precision=prec)
            plan.eval(fd, out)
            torch.cuda.synchronize()
            reps = 2
            t0 = time.perf_counter()
            for _ in range(reps):
                plan.eval(fd, out)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            r[f"rhs_batch_{batch}"] = {"eval_ms": ms, "target_rhs_per_s": n * k / (ms * 1e-3)}
            plan.close()
        r["batching_speedup"] = r["rhs_batch_1"]["eval_ms"] / r["rhs_batch_8"]["eval_ms"]
        u_last[pname] = out[k - 1].cpu().numpy()
        res[pname] = r
    res["mixed_over_fp64_eval"] = res["mixed"]["rhs_batch_8"]["eval_ms"] / res["fp64"]["rhs_batch_8"]["eval_ms"]
    if parity:
        import oracle
        ref = oracle.direct(x, f[k - 1], idx)
        for pname in u_last:
            res[pname]["rel_l2_sampled_last_rhs"] = oracle.rel_l2(u_last[pname][idx], ref)
        res["mixed"]["rel_l2_vs_fp64_last_rhs"] = oracle.rel_l2(u_last["mixed"], u_last["fp64"])
        res["parity_sample"] = f"{idx.size} targets of the last vector"
    print(f"# multi-rhs: mixed {res['mixed']['rhs_batch_8']['eval_ms']:.1f} ms, fp64 "
          f"{res['fp64']['rhs_batch_8']['eval_ms']:.1f} ms for {k} vectors (unbatched fp64 "
          f"{res['fp64']['rhs_batch_1']['eval_ms']:.1f} ms)", file=sys.stderr, flush=True)
    del fd, out
    torch.cuda.empty_cache()
    return res


def uniform_1e4_variant(args, dev, parity: bool) -> dict:
    """10^4 uniform points at 1e-6 (a small problem, where launches rather
    than kernels set the evaluation time): plan + eval per step, evaluation
    alone with eager launches and with hipGraph replay, and the error against
    the direct sum at every target."""
    import torch

    import paper_2509_21471_amd as dmk
    import workloads
    name = "uniform_1e4"
    cfg = workloads.CONFIGS[name]
    x, f = workloads.config(name)
    n = x.shape[0]
    xd = torch.from_numpy(x).to(dev)
    fd = torch.from_numpy(f).to(dev)
    out = torch.empty_like(fd)
    reps = 50
    res = {"workload": name, "n": n, "tol": cfg["tol"], "precision": "fp64"}
    for _ in range(3):
        dmk.Plan(xd, tol=cfg["tol"]).eval(fd, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        p = dmk.Plan(xd, tol=cfg["tol"])
        p.eval(fd, out)
        p.close()
    torch.cuda.synchronize()
    res["ms_per_step"] = (time.perf_counter() - t0) * 1e3 / reps
    res["targets_per_s"] = n / (res["ms_per_step"] * 1e-3)
    for graph in (False, True):
        p = dmk.Plan(xd, tol=cfg["tol"], graph=graph)
        for _ in range(3):
            p.eval(fd, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            p.eval(fd, out)
        torch.cuda.synchronize()
        res["eval_graph_ms" if graph else "eval_eager_ms"] = (time.perf_counter() - t0) * 1e3 / reps
        u = out.cpu().numpy()
        p.close()
    res["graph_speedup"] = res["eval_eager_ms"] / res["eval_graph_ms"]
    if parity:
        import oracle
        res["rel_l2_all_targets"] = oracle.rel_l2(u, oracle.direct(x, f))
    print(f"# uniform_1e4: {res['ms_per_step']:.2f} ms/step, eval eager {res['eval_eager_ms']:.3f} ms, "
          f"graph {res['eval_graph_ms']:.3f} ms", file=sys.stderr, flush=True)
    del xd, fd, out
    torch.cuda.empty_cache()
    return res


def clusters_4e6_variant(args, dev, parity: bool) -> dict:
    """4e6 clustered points (sigma 0.01) at 1e-6: plan + eval steps and
    evaluation alone in FP64 and in mixed precision, with errors against the
    stored direct sums at 10,000 sampled targets and mixed against FP64."""
    import torch

    import paper_2509_21471_amd as dmk
    import workloads
    name = "clusters_4e6"
    cfg = workloads.CONFIGS[name]
    x, f = workloads.config(name)
    n = x.shape[0]
    xd = torch.from_numpy(x).to(dev)
    fd = torch.from_numpy(f).to(dev)
    out = torch.empty_like(fd)
    steps = max(2, min(args.steps, 5))
    res = {"workload": name, "n": n, "tol": cfg["tol"], "steps": steps}
    u = {}
    for pname, prec in (("fp64", dmk.PREC_FP64), ("mixed", dmk.PREC_MIXED)):
        def plan():
            return dmk.Plan(xd, tol=cfg["tol"], precision=prec, timing=True)
        p = plan()
        p.eval(fd, out)
        torch.cuda.synchronize()
        p.close()
        t0 = time.perf_counter()
        for i in range(steps):
            p = plan()
            p.eval(fd, out)
            torch.cuda.synchronize()
            if i < steps - 1:
                p.close()
        step_ms = (time.perf_counter() - t0) * 1e3 / steps
        t0 = time.perf_counter()
        for _ in range(steps):
            p.eval(fd, out)
        torch.cuda.synchronize()
        eval_ms = (time.perf_counter() - t0) * 1e3 / steps
        info = p.info()
        res[pname] = {"ms_per_step": step_ms, "targets_per_s": n / (step_ms * 1e-3), "eval_only_ms": eval_ms,
                      "eval_only_targets_per_s": n / (eval_ms * 1e-3), "levels": info["levels"],
                      "leaf_size": info["leaf_size"], "phases_ms": p.phase_ms()}
        u[pname] = out.cpu().numpy()
        p.close()
    res["mixed_speedup_step"] = res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"]
    res["mixed_speedup_eval"] = res["fp64"]["eval_only_ms"] / res["mixed"]["eval_only_ms"]
    if parity:
        import oracle
        g = np.load(os.path.join(ROOT, "tests", "golden", "clusters_4e6_direct.npz"))
        for pname in u:
            res[pname]["rel_l2_sampled"] = oracle.rel_l2(u[pname][g["idx"]], g["u"])
        res["mixed"]["rel_l2_vs_fp64"] = oracle.rel_l2(u["mixed"], u["fp64"])
        res["parity_sample"] = f"{g['idx'].size} stored direct-sum targets"
    print(f"# clusters_4e6: fp64 {res['fp64']['ms_per_step']:.1f} ms/step, mixed {res['mixed']['ms_per_step']:.1f} "
          f"ms/step", file=sys.stderr, flush=True)
    del xd, fd, out
    torch.cuda.empty_cache()
    return res


def ewald_variant(args, dev, parity: bool) -> dict:
    """The 2e6-point periodic workload at 1e-9 by the single-level spectral
    Ewald method (split level swept over 3, 4, 5 through the leaf size) against
    the multilevel DMK on the same points: plan + eval per step and eval alone."""
    import torch

    import paper_2509_21471_amd as dmk
    import workloads
    name = "periodic_2e6"
    cfg = workloads.CONFIGS[name]
    x, f = workloads.config(name)
    n = x.shape[0]
    xd = torch.from_numpy(x).to(dev)
    fd = torch.from_numpy(f).to(dev)
    out = torch.empty_like(fd)
    steps = max(2, args.steps)

    def run(method, leaf):
        def plan():
            return dmk.Plan(xd, periodic=True, tol=cfg["tol"], leaf_size=leaf, method=method, timing=True)
        p = plan()
        p.eval(fd, out)
        torch.cuda.synchronize()
        p.close()
        t0 = time.perf_counter()
        for _ in range(steps):
            p = plan()
            p.eval(fd, out)
            torch.cuda.synchronize()
            if _ < steps - 1:
                p.close()
        step_ms = (time.perf_counter() - t0) * 1e3 / steps
        t0 = time.perf_counter()
        for _ in range(steps):
            p.eval(fd, out)
        torch.cuda.synchronize()
        eval_ms = (time.perf_counter() - t0) * 1e3 / steps
        info = p.info()
        ph = p.phase_ms()
        u = out.cpu().numpy()
        p.close()
        return {"ms_per_step": step_ms, "eval_only_ms": eval_ms, "levels": info["levels"],
                "grid": info["ewald_grid"], "modes": info["ewald_modes"], "phases_ms": ph}, u

    res = {"workload": name, "n": n, "tol": cfg["tol"], "precision": "fp64"}
    res["dmk"], u_dmk = run(dmk.METHOD_DMK, 0)
    best = None
    for leaf in (4000, 2000, 400):
        r, u = run(dmk.METHOD_EWALD, leaf)
        r["leaf_size"] = leaf
        res[f"ewald_L{r['levels'] - 1}"] = r
        if best is None or r["ms_per_step"] < best[0]["ms_per_step"]:
            best = (r, u)
    res["ewald_best_split_level"] = best[0]["levels"] - 1
    res["ewald_over_dmk_step"] = best[0]["ms_per_step"] / res["dmk"]["ms_per_step"]
    res["ewald_over_dmk_eval"] = best[0]["eval_only_ms"] / res["dmk"]["eval_only_ms"]
    if parity:
        import oracle
        g = np.load(os.path.join(ROOT, "tests", "golden", "periodic_2e6_ewald.npz"))
        res["dmk"]["rel_l2_sampled"] = oracle.rel_l2(u_dmk[g["idx"]], g["u"])
        res["ewald_rel_l2_sampled"] = oracle.rel_l2(best[1][g["idx"]], g["u"])
    print(f"# periodic 2e6 1e-9: DMK {res['dmk']['ms_per_step']:.1f} ms/step (eval {res['dmk']['eval_only_ms']:.1f}), "
          f"spectral Ewald L={res['ewald_best_split_level']} {best[0]['ms_per_step']:.1f} ms/step "
          f"(eval {best[0]['eval_only_ms']:.1f})", file=sys.stderr, flush=True)
    del fd, out
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="clusters_1e6")
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="precision of the main timed steps (the benchmark line is FP64; mixed is for profiling)")
    ap.add_argument("--leaf-size", type=int, default=0)
    ap.add_argument("--near-lanes", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=12000)
    ap.add_argument("--parity-sample", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the tolerance's default leaf size and lane split instead of the autotuner's")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the multi-right-hand-side (and other) variant measurements")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes three times (the "
                         "reference kernel for scaling HBM byte counters) and exit")
    ap.add_argument("--only", choices=["spectral_ewald", "multi_rhs", "batched", "clusters_4e6", "uniform_1e4"],
                    default=None,
                    help="run only this variant and print its JSON record (for profiling; not the benchmark line)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.only:
        import torch
        dev = torch.device("cuda:0")
        fn = {"spectral_ewald": lambda: ewald_variant(args, dev, not args.no_parity),
              "multi_rhs": lambda: multi_rhs_variant(args, dev, not args.no_parity),
              "batched": lambda: batched_variant(dev, not args.no_parity),
              "clusters_4e6": lambda: clusters_4e6_variant(args, dev, not args.no_parity),
              "uniform_1e4": lambda: uniform_1e4_variant(args, dev, not args.no_parity)}[args.only]
        print(json.dumps({"variant": args.only, **fn()}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    import paper_2509_21471_amd as dmk
    import workloads

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    dev = torch.device("cuda:0")
    cfg = workloads.CONFIGS[args.config]
    tol = args.tol if args.tol is not None else cfg["tol"]
    periodic = bool(cfg["periodic"])
    x, f = workloads.make(cfg["kind"], cfg["n"], cfg["seed"], cfg["sigma"])
    n = x.shape[0]
    xd = torch.from_numpy(x).to(dev)
    fd = torch.from_numpy(f).to(dev)
    out = torch.empty_like(fd)
    torch.cuda.synchronize()
    print(f"# input ready: {args.config} n={n} tol={tol}", file=sys.stderr, flush=True)

    leaf, lanes = args.leaf_size, args.near_lanes
    rows, pts = 0, 0
    tuned = None
    if not args.no_autotune and leaf == 0 and lanes == 0:
        # outside the timed region: picks the leaf size, near-field lane split and tile shapes
        tuned = dmk.autotune(xd, periodic=periodic, tol=tol)
        leaf, lanes = tuned["leaf_size"], tuned["near_lanes"]
        rows, pts = tuned["stage_rows"], tuned["eval_points"]
        print(f"# autotuned: leaf {leaf}, lanes {lanes}, stage rows {rows}, eval points {pts} ({tuned['ms']:.1f} ms)",
              file=sys.stderr, flush=True)

    nvd = None  # stresslet orientation vectors, made when the stresslet variant runs

    def make_plan(prec, window=0, leaf_size=None, near_lanes=None, kernel=0, ptol=None):
        # the tuned tile shapes go with the tuned leaf size and tolerance only
        tuned_shape = leaf_size is None and ptol is None and window == 0 and kernel == 0
        return dmk.Plan(xd, periodic=periodic, tol=tol if ptol is None else ptol,
                        leaf_size=leaf if leaf_size is None else leaf_size,
                        timing=True, near_lanes=lanes if near_lanes is None else near_lanes, precision=prec,
                        concurrent=True, window=window, kernel=kernel,
                        stage_rows=rows if tuned_shape else 0, eval_points=pts if tuned_shape else 0)

    def run(p, kernel):
        if kernel == dmk.KERNEL_STRESSLET:
            p.eval_stresslet(fd, nvd, out)
        else:
            p.eval(fd, out)

    def timed_steps(prec, window=0, leaf_size=None, near_lanes=None, kernel=0, ptol=None):
        """Warmup, K timed plan+eval steps, then K eval-only repetitions on the
        last plan.  Returns the measurements and the last plan (open)."""
        for _ in range(args.warmup):
            p = make_plan(prec, window, leaf_size, near_lanes, kernel, ptol)
            run(p, kernel)
            torch.cuda.synchronize()
            p.close()
        near_ms, phases_acc = [], []
        prev = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            p = make_plan(prec, window, leaf_size, near_lanes, kernel, ptol)
            run(p, kernel)  # queued behind the previous evaluation: the device never waits for the host
            if prev is not None:
                ph = prev.phase_ms()
                phases_acc.append(ph)
                near_ms.append(ph["near"])
                prev.close()
            prev = p
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ph = prev.phase_ms()
        phases_acc.append(ph)
        near_ms.append(ph["near"])
        ms_step = (t1 - t0) * 1e3 / args.steps
        for _ in range(2):
            run(prev, kernel)
        torch.cuda.synchronize()
        te0 = time.perf_counter()
        for _ in range(args.steps):
            run(prev, kernel)
        torch.cuda.synchronize()
        ms_eval = (time.perf_counter() - te0) * 1e3 / args.steps
        phases = {k: float(np.mean([a[k] for a in phases_acc])) for k in phases_acc[0]}
        return ms_step, ms_eval, phases, float(np.mean(near_ms)), prev

    main_prec = dmk.PREC_MIXED if args.precision == "mixed" else dmk.PREC_FP64
    ms_per_step, eval_ms, phases, near_mean, plan = timed_steps(main_prec)
    info = plan.info()
    print(f"# timed: {ms_per_step:.2f} ms/step, eval {eval_ms:.2f} ms", file=sys.stderr, flush=True)
    stats = plan.near_stats()
    fpp = near_flops_per_pair(info["deg_P"], info["deg_Q"])
    t_near = near_mean * 1e-3
    achieved = stats["in_support"] * fpp / t_near / 1e12

    nd = nd_bucket(info['deg_P'], info['deg_Q'])
    refine = "false" if (nd == 14 and tol >= 1e-6 * (1 - 1e-9)) else "true"
    nz = "true" if info["no_coincident"] else "false"
    near_kernel = f"dmk::k_near<{nd}, {info['near_lanes']}, 1, 0, {refine}, {nz}>"
    traffic = near_traffic(args.config, tol, args.precision, near_kernel, info["leaf_size"], info["near_lanes"])
    result = {
        "metric": METRIC,
        "value": n / (ms_per_step * 1e-3),
        "unit": "targets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.config, "n": n, "kind": cfg["kind"], "sigma": cfg["sigma"],
                   "periodic": periodic, "tol": tol, "precision": args.precision, "step": "plan+eval",
                   "leaf_size": info["leaf_size"], "near_lanes": info["near_lanes"],
                   "stage_rows": rows, "eval_points": pts, "autotuned": tuned is not None},
        "roofline": {"bound": "alu", "kernel": "k_near", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
                     "traffic": traffic, "traffic_unit": "bytes/launch",
                     "near_ms": t_near * 1e3, "pairs_in_support": stats["in_support"],
                     "pairs_evaluated": stats["evaluated"], "pairs_listed": stats["listed"],
                     "flops_per_pair": fpp,
                     # the same flops per pair over every evaluated pair (the kernel's issue
                     # efficiency) and the in-support share of evaluated pairs
                     "frac_evaluated": stats["evaluated"] * fpp / t_near / 1e12 / PEAK_FP64_VECTOR_TFLOPS,
                     "useful_fraction": stats["in_support"] / max(stats["evaluated"], 1)},
        "eval_only_ms": eval_ms,
        "eval_only_targets_per_s": n / (eval_ms * 1e-3),
        "phases_ms": phases,
        "tree": {k: info[k] for k in ("levels", "n_boxes", "n_nonempty_leaves", "n_senders", "n_receivers",
                                      "device_bytes", "plan_ms", "plan_phase_ms", "p", "n1", "deg_P",
                                      "deg_Q")},
    }

    u64 = out.cpu().numpy()
    plan.close()
    if not args.no_variants:
        mixed = {}
        m_step, m_eval, m_phases, m_near, mplan = timed_steps(dmk.PREC_MIXED)
        mixed = {"precision": "mixed (FP32 far-field storage, FP64 arithmetic)", "workload": args.config,
                 "ms_per_step": m_step, "targets_per_s": n / (m_step * 1e-3), "eval_only_ms": m_eval,
                 "eval_only_targets_per_s": n / (m_eval * 1e-3), "phases_ms": m_phases,
                 "device_bytes": mplan.info()["device_bytes"],
                 "speedup_vs_fp64_step": ms_per_step / m_step, "speedup_vs_fp64_eval": eval_ms / m_eval}
        u32 = out.cpu().numpy()
        mplan.close()
        print(f"# mixed: {m_step:.2f} ms/step, eval {m_eval:.2f} ms", file=sys.stderr, flush=True)
        # the same method with the Gaussian (Hasimoto) window and its parameter columns
        # (its leaf size is swept here: 0.75, 1 and 1.35 times the default)
        best = None
        for fac in (0.75, 1.0, 1.35):
            lf = int(round(1200 * fac)) if args.leaf_size == 0 else args.leaf_size
            st_ms, ev_ms, g_phases, _, gplan = timed_steps(dmk.PREC_FP64, 1, lf, lanes)
            ginfo = gplan.info()
            u_g = out.cpu().numpy()
            gplan.close()
            if best is None or st_ms < best[0]:
                best = (st_ms, ev_ms, g_phases, ginfo, lf, u_g)
            if args.leaf_size != 0:
                break
        gaussian = {"window": "gaussian", "workload": args.config, "precision": "fp64", "leaf_size": best[4],
                    "q": best[3]["q"], "p": best[3]["p"], "n1": best[3]["n1"], "ms_per_step": best[0],
                    "eval_only_ms": best[1], "phases_ms": best[2],
                    "gaussian_over_prolate_step": best[0] / ms_per_step}
        u_gauss = best[5]
        print(f"# gaussian window: {best[0]:.2f} ms/step, eval {best[1]:.2f} ms (leaf {best[4]})", file=sys.stderr,
              flush=True)
        # the same FP64 Stokeslet steps at the tighter tolerance 1e-9 (leaf size
        # swept over 1 and 1.35 times that row's default)
        tight = None
        if not periodic and tol > 1e-9:
            best = None
            for fac in (1.0, 1.35):
                lf = int(round(2000 * fac)) if args.leaf_size == 0 else args.leaf_size
                st_ms, ev_ms, t_phases, t_near, tplan = timed_steps(dmk.PREC_FP64, 0, lf, lanes, 0, 1e-9)
                if best is None or st_ms < best[0]:
                    if best is not None:
                        best[4].close()
                    best = (st_ms, ev_ms, t_phases, t_near, tplan, lf, out.cpu().numpy())
                else:
                    tplan.close()
                if args.leaf_size != 0:
                    break
            tinfo = best[4].info()
            tst = best[4].near_stats()
            tfpp = near_flops_per_pair(tinfo["deg_P"], tinfo["deg_Q"])
            tach = tst["in_support"] * tfpp / (best[3] * 1e-3) / 1e12
            tight = {"tol": 1e-9, "workload": args.config, "precision": "fp64", "leaf_size": best[5],
                     "p": tinfo["p"], "n1": tinfo["n1"], "ms_per_step": best[0],
                     "targets_per_s": n / (best[0] * 1e-3), "eval_only_ms": best[1], "phases_ms": best[2],
                     "near_roofline": {"achieved": tach, "peak": PEAK_FP64_VECTOR_TFLOPS,
                                       "frac": tach / PEAK_FP64_VECTOR_TFLOPS, "flops_per_pair": tfpp,
                                       "useful_fraction": tst["in_support"] / max(tst["evaluated"], 1)}}
            u_tight = best[6]
            best[4].close()
            print(f"# tol 1e-9: {best[0]:.2f} ms/step, eval {best[1]:.2f} ms (leaf {best[5]})", file=sys.stderr,
                  flush=True)
        # the stresslet (double-layer) sum on the same points, f the same forces
        # and n seeded unit vectors; its leaf size swept over 1, 1.35 and 1.8
        # times the Stokeslet's (its far field carries 6 density components)
        stress = None
        if not periodic:
            nv = workloads.normals(x, cfg["seed"], "sphere" if cfg["kind"] == "sphere" else "random")
            nvd = torch.from_numpy(nv).to(dev)
            best = None
            for fac in (1.0, 1.35, 1.8):
                lf = int(round(leaf * fac)) if leaf else int(round(1200 * fac))
                st_ms, ev_ms, s_phases, _, splan = timed_steps(dmk.PREC_FP64, 0, lf, lanes, dmk.KERNEL_STRESSLET)
                sinfo = splan.info()
                u_s = out.cpu().numpy()
                splan.close()
                if best is None or st_ms < best[0]:
                    best = (st_ms, ev_ms, s_phases, sinfo, lf, u_s)
            stress = {"kernel": "stresslet", "workload": args.config, "precision": "fp64", "leaf_size": best[4],
                      "q": best[3]["q"], "p": best[3]["p"], "ms_per_step": best[0],
                      "targets_per_s": n / (best[0] * 1e-3), "eval_only_ms": best[1], "phases_ms": best[2],
                      "stresslet_over_stokeslet_step": best[0] / ms_per_step}
            u_stress = best[5]
            print(f"# stresslet: {best[0]:.2f} ms/step, eval {best[1]:.2f} ms (leaf {best[4]})", file=sys.stderr,
                  flush=True)
        result["variants"] = {"mixed": mixed, "gaussian_window": gaussian,
                              "multi_rhs": multi_rhs_variant(args, dev, not args.no_parity),
                              "batched": batched_variant(dev, not args.no_parity),
                              "clusters_4e6": clusters_4e6_variant(args, dev, not args.no_parity),
                              "uniform_1e4": uniform_1e4_variant(args, dev, not args.no_parity),
                              "spectral_ewald": ewald_variant(args, dev, not args.no_parity)}
        if stress is not None:
            result["variants"]["stresslet"] = stress
        if tight is not None:
            result["variants"]["tol_1e-9"] = tight

    if not args.no_parity:
        import oracle
        idx = workloads.sample_targets(n, args.parity_sample, cfg["seed"])
        if periodic:
            from oracle.ewald import ewald
            ref = ewald(x, f, idx, E=25.0)
        else:
            ref = oracle.direct(x, f, idx)
        result["rel_l2_sampled"] = oracle.rel_l2(u64[idx], ref)
        result["parity_sample"] = int(idx.size)
        if "variants" in result:
            result["variants"]["mixed"]["rel_l2_sampled"] = oracle.rel_l2(u32[idx], ref)
            result["variants"]["mixed"]["rel_l2_vs_fp64"] = oracle.rel_l2(u32, u64)
            result["variants"]["gaussian_window"]["rel_l2_sampled"] = oracle.rel_l2(u_gauss[idx], ref)
            if "tol_1e-9" in result["variants"]:
                result["variants"]["tol_1e-9"]["rel_l2_sampled"] = oracle.rel_l2(u_tight[idx], ref)
            if "stresslet" in result["variants"]:
                ref_s = oracle.stresslet_direct(x, f, nv, idx)
                result["variants"]["stresslet"]["rel_l2_sampled"] = oracle.rel_l2(u_stress[idx], ref_s)

    if not args.no_cpu_baseline and not periodic:
        import oracle
        idx = workloads.sample_targets(n, args.cpu_sample, cfg["seed"] + 1)
        cores = oracle.num_threads()
        tc0 = time.perf_counter()
        oracle.direct(x, f, idx)
        tc = time.perf_counter() - tc0
        # the same sum on one core, over the first sixteenth of the sample
        idx1 = idx[:max(1, idx.size // 16)]
        oracle.set_num_threads(1)
        t10 = time.perf_counter()
        oracle.direct(x, f, idx1)
        t1 = time.perf_counter() - t10
        oracle.set_num_threads(cores)
        result["cpu_baseline"] = {"value": idx.size / tc, "unit": "targets/s", "cores": cores,
                                  "kind": "oracle", "cpu_model": cpu_model(),
                                  "value_1_core": idx1.size / t1,
                                  "sample": f"{idx.size} seeded targets of the {n}-point input, each summing "
                                            f"all {n} sources (direct O(N^2) FP64 sum), {tc:.1f} s on {cores} "
                                            f"threads; {idx1.size} of them on 1 thread, {t1:.1f} s"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
