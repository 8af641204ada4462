"""Benchmark: Lagrange-FMM force evaluation on one MI355X.

One step = one dfmm_fmm_forces call (points, P2M, M2M, M2L, L2L, L2P + near
field, force assembly) over the whole synthetic loop ensemble, inputs resident
in HBM.  The tree is built once before timing (reported separately), the M2L
operators are precomputed once (reported separately).

Prints ONE JSON line (see the keys below).  Default workload: 1M segments
(25,000 hexagonal loops), cubic medium (C11, C12, C44) = (1, 0.6, 0.5),
order p = 6, depth D = 7, mixed precision.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FMM force-eval time & segments/s at N_s=1M, rel err vs FP64 direct <=1e-4"
PEAK_FP32_VALU = 157.3e12  # MI355X fp32 vector (256 CUs x 2.4 GHz x 256 flop/clk)
PEAK_FP64_VALU = 78.6e12
PEAK_HBM = 8.0e12
# Smallest interpolation order whose force error on the workload is <= 1e-4
# (measured: cubic1m p=6 1.15e-4, p=7 3.0e-5 against the FP64 direct sum).
BAR_ORDER = {"cubic1m": 7, "cubic10m": 7, "iso200k": 6, "cubic100k": 6}
def traffic_file(kernel):
    return os.path.join(ROOT, "profiles", "%s_cubic1m_p7_traffic.json" % kernel)


def kernel_source_sha(kernel):
    """SHA-256 of a kernel's definition in fmm.hip (from its __global__
    line to the brace that closes its body), so that a traffic figure goes
    stale exactly when that kernel's code changes."""
    import hashlib
    import re

    src = open(os.path.join(ROOT, "paper_1712_07739_amd", "csrc", "fmm.hip")).read()
    m = re.search(r"__global__[^;{]*?\b%s\s*\(" % re.escape(kernel), src)
    if m is None:
        return None
    i = src.index("{", m.end())
    depth = 0
    for j in range(i, len(src)):
        depth += {"{": 1, "}": -1}.get(src[j], 0)
        if depth == 0:
            return hashlib.sha256(src[m.start():j + 1].encode()).hexdigest()
    return None


def hadamard_traffic(order, kernel="k_hadamard", workload="cubic1m"):
    """HBM bytes per step of the Hadamard kernel's launches, from the
    committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, if it was taken on the
    current source of that kernel, the same workload and the same order;
    else None."""
    path = traffic_file(kernel)
    if workload != "cubic1m" or not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_sha256") is None or d.get("kernel_sha256") != kernel_source_sha(kernel) or d.get("order") != order:
        return None
    return d["hbm_bytes_per_step"]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def hadamard_flops(tree_info, nf):
    """Algorithmic flops of the M2L Hadamard stage: per interaction pair and
    frequency a 6x9 complex matrix times a 9-vector (54 complex MACs = 432 flop)."""
    return tree_info["m2l_pairs"] * nf * 54 * 8


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cubic1m")
    ap.add_argument("--precision", default="mixed16", choices=["mixed", "mixed16", "fp64"],
                    help="mixed: f32 evaluation; mixed16: f32 with f16 operands in the M2L product; fp64")
    ap.add_argument("--order", type=int, default=0,
                    help="interpolation order p (default: the smallest order meeting the 1e-4 bar, "
                         "7 for cubic1m; its configured p=6 measures 1.15e-4)")
    ap.add_argument("--depth", type=int, default=0, help="override the workload's leaf depth D")
    ap.add_argument("--leaf-max", type=int, default=0,
                    help="adaptive tree: split cells holding more than this many quadrature points, down to "
                         "the depth (0: uniform tree)")
    ap.add_argument("--m2l-mode", default="sym", choices=["fft", "sym"],
                    help="M2L operator store: 158 offset spectra (fft) or 16 symmetry classes (sym)")
    ap.add_argument("--err-sample", type=int, default=2000,
                    help="target segments checked against the GPU FP64 direct sum over all sources")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="cubic media: skip training the anisotropic-kernel network (it is used where its gate passes)")
    ap.add_argument("--cpu-sample", type=int, default=3, help="target segments timed on the CPU oracle")
    ap.add_argument("--surrogate-tol", type=float, default=1e-5,
                    help="residual gate of the anisotropic-kernel network (bins below it use the network)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run 3 plain device copies of MIB MiB (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calib:
        import torch

        x = torch.ones(args.copy_calib * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_mib": args.copy_calib, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported "
              "(sharding one ensemble over several GPUs is not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1712_07739_amd as pk
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batch64":
        return bench_batch(args)
    seg, burg, prm = synth.make_workload(args.workload)
    configured_order = prm["order"]
    if args.order:
        prm["order"] = args.order
    elif args.workload in BAR_ORDER:
        prm["order"] = BAR_ORDER[args.workload]
    if args.depth:
        prm["depth"] = args.depth
    ns = seg.shape[0]
    log("workload %s: %d segments" % (args.workload, ns))
    prec = {"mixed": pk.DFMM_MIXED, "mixed16": pk.DFMM_MIXED_F16, "fp64": pk.DFMM_FP64}[args.precision]

    def make_plan(precision):
        p = pk.make_params(prm["order"], prm["depth"], prm["c11"], prm["c12"], prm["c44"], prm["core_a"],
                           prm["box_lo"], prm["box_size"], precision=precision,
                           m2l_mode=pk.DFMM_M2L_FFT_SYM if args.m2l_mode == "sym" else pk.DFMM_M2L_FFT,
                           leaf_max=args.leaf_max)
        return pk.Plan(p)

    t0 = time.perf_counter()
    plan = make_plan(prec)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = plan.info()
    log("setup %.2f s %s" % (setup_s, info))
    sur = None
    cubic = abs(2 * prm["c44"] - (prm["c11"] - prm["c12"])) > 1e-12
    if cubic and prec != pk.DFMM_FP64 and not args.no_surrogate and not args.leaf_max:
        # the learned surrogate of the anisotropic kernel: 2M samples, residual gate 1e-5,
        # the exact quadrature wherever a direction bin fails the gate
        t0 = time.perf_counter()
        sinfo = plan.surrogate_train(n_samples=1 << 21, tol=args.surrogate_tol, seed=5)
        plan.surrogate_use(True)
        torch.cuda.synchronize()
        sur = {k: sinfo[k] for k in ("n_params", "n_samples", "epochs", "bins", "tol", "pass_frac",
                                      "median_bin_err", "max_bin_err", "train_ms")}
        sur["loss_first_last"] = [sinfo["loss"][0], sinfo["loss"][-1]]
        sur["setup_s"] = time.perf_counter() - t0
        log("surrogate: %s" % sur)
    tseg = torch.tensor(seg, device=dev)
    tb = torch.tensor(burg, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree = pk.Tree(plan, tseg)
    torch.cuda.synchronize()
    tree_s = time.perf_counter() - t0
    tinfo = tree.info()
    log("tree %.3f s: m2l pairs %d, near pairs %d, leaves %d, w/x pairs %d, spectrum chunks %d, workspace %.1f GB" % (
        tree_s, tinfo["m2l_pairs"], tinfo["near_pairs"], tinfo["leaves"], tinfo["w_pairs"], tinfo["freq_chunks"],
        tinfo["workspace_bytes"] / 1e9))
    out = torch.empty((ns, 2, 3), dtype=torch.float64, device=dev)
    for i in range(args.warmup):
        pk.fmm_forces(plan, tree, tseg, tb, out=out)
        torch.cuda.synchronize()
        log("warmup %d done" % i)
    # timed region: K calls as a user makes them (near field beside the far field)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        pk.fmm_forces(plan, tree, tseg, tb, out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = 1e3 * el / args.steps
    # per-stage breakdown: K more calls with HIP events around every stage (stages then run one by one)
    tree.set_timing(True)
    for i in range(args.steps):
        pk.fmm_forces(plan, tree, tseg, tb, out=out)
    torch.cuda.synchronize()
    stage_ms, ncalls = tree.stage_times()
    tree.set_timing(False)
    log("timed %d steps: %.3f ms/step; stages, run one by one (ms/step): %s (sum %.3f)" % (
        args.steps, ms_step, {pk.STAGES[i]: round(stage_ms[i] / ncalls, 3) for i in range(pk.N_STAGES)},
        sum(stage_ms) / ncalls))

    # accuracy: relative error vs the GPU FP64 direct sum on a seeded segment subset
    sub = synth.segment_subset(ns, args.err_sample, 10000 + ns % 1000)
    tsub = torch.tensor(sub, device=dev)
    ref = pk.direct_forces(plan, tseg, tb, targets=tsub, fp32=False).cpu().numpy()
    f = out.cpu().numpy()[sub]
    err = float(np.linalg.norm(f - ref) / np.linalg.norm(ref))
    log("rel err vs FP64 direct on %d segments: %.3e" % (len(sub), err))

    # roofline of the dominant kernel (M2L Hadamard product)
    nf = info["n_freq"]
    had_flops = hadamard_flops(tinfo, nf)
    had_ms = stage_ms[3] / ncalls
    achieved = had_flops / (had_ms * 1e-3)
    peak = PEAK_FP32_VALU if prec != pk.DFMM_FP64 else PEAK_FP64_VALU
    kname = {pk.DFMM_MIXED_F16: "k_hadamard16 (M2L in frequency space, f16 operands)",
             pk.DFMM_MIXED: "k_hadamard (M2L in frequency space, f32 operands)",
             pk.DFMM_FP64: "k_hadamard64 (FP64 M2L in frequency space)"}[prec]
    roof = {"kernel": kname + ", all levels of one step", "bound": "alu",
            "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": hadamard_traffic(prm["order"], {pk.DFMM_MIXED_F16: "k_hadamard16", pk.DFMM_MIXED: "k_hadamard",
                                                       pk.DFMM_FP64: "k_hadamard64"}[prec], args.workload),
            "flop_per_step": had_flops, "ms_per_step": had_ms}
    result = {
        "metric": METRIC, "value": ns / (ms_step * 1e-3), "unit": "segments/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {pk.DFMM_MIXED: "f32", pk.DFMM_MIXED_F16: "f16/f32", pk.DFMM_FP64: "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "n_seg": ns, "order": prm["order"], "depth": prm["depth"],
                   "C": [prm["c11"], prm["c12"], prm["c44"]], "core_a": prm["core_a"],
                   "precision": args.precision, "configured_order": configured_order, "m2l_mode": args.m2l_mode,
                   "tree": "adaptive, leaves of at most %d points" % args.leaf_max if args.leaf_max else "uniform",
                   "freq_chunks": tinfo["freq_chunks"]},
        "rel_err_vs_fp64_direct": err, "err_sample_segments": int(len(sub)),
        "stage_ms": {pk.STAGES[i]: stage_ms[i] / ncalls for i in range(pk.N_STAGES)},
        "stage_ms_note": "separate pass with HIP events around each stage, stages one by one (in the timed "
                         "region the near field runs on a second stream beside the far field)",
        "setup_s": setup_s, "build_tree_s": tree_s,
        "plan": {k: info[k] for k in ("n_freq", "n_circle", "n_circle_float", "float_rule_err", "spectra_bytes",
                                      "stored_offsets", "generator_fp64_bytes_per_level",
                                      "mem_unif_fp64_bytes_per_level") if k in info},
        "surrogate": sur, "m2l_pairs": tinfo["m2l_pairs"],
        "near_pairs": tinfo["near_pairs"], "roofline": roof,
    }
    del tree
    def other_path(precision, kernel, peak, kshort):
        """Time and error of the same workload in another precision (same
        tree shape, its own plan): K calls as issued, then K with stage events."""
        plan2 = make_plan(precision)
        tree2 = pk.Tree(plan2, tseg)
        out2 = pk.fmm_forces(plan2, tree2, tseg, tb)
        torch.cuda.synchronize()
        n2 = max(1, min(args.steps, 3))
        t0 = time.perf_counter()
        for i in range(n2):
            pk.fmm_forces(plan2, tree2, tseg, tb, out=out2)
        torch.cuda.synchronize()
        ms2 = 1e3 * (time.perf_counter() - t0) / n2
        f2 = out2.cpu().numpy()[sub]
        tree2.set_timing(True)
        for i in range(n2):
            pk.fmm_forces(plan2, tree2, tseg, tb, out=out2)
        torch.cuda.synchronize()
        st2, nc2 = tree2.stage_times()
        tree2.set_timing(False)
        had2_ms = st2[3] / nc2
        ach2 = had_flops / (had2_ms * 1e-3)
        res = {
            "ms_per_step": ms2, "rel_err_vs_fp64_direct": float(np.linalg.norm(f2 - ref) / np.linalg.norm(ref)),
            "speedup_of_headline": ms2 / ms_step,
            "stage_ms": {pk.STAGES[i]: st2[i] / nc2 for i in range(pk.N_STAGES)},
            "roofline": {"kernel": kernel + ", all levels of one step", "bound": "alu", "achieved": ach2 / 1e12,
                         "peak": peak / 1e12, "unit": "TFLOP/s", "frac": ach2 / peak,
                         "traffic": hadamard_traffic(prm["order"], kshort, args.workload),
                         "flop_per_step": had_flops, "ms_per_step": had2_ms}}
        log("%s path: %.3f ms/step (headline speedup %.2fx), error %.3e; Hadamard %.1f ms = %.1f TFLOP/s"
            % (kernel, ms2, ms2 / ms_step, res["rel_err_vs_fp64_direct"], had2_ms, ach2 / 1e12))
        del tree2, plan2
        return res

    if not args.no_fp64_compare and prec != pk.DFMM_FP64:
        if prec == pk.DFMM_MIXED_F16:
            result["mixed_f32_path"] = other_path(pk.DFMM_MIXED, "k_hadamard (f32 operands)", PEAK_FP32_VALU,
                                                  "k_hadamard")
        result["fp64_path"] = other_path(pk.DFMM_FP64, "k_hadamard64 (FP64 M2L in frequency space)", PEAK_FP64_VALU,
                                         "k_hadamard64")
    if not args.no_cpu_baseline:
        import oracle

        med = oracle.medium_from_params(prm)
        k = max(1, args.cpu_sample)
        tgt = synth.segment_subset(ns, k, 77)
        t0 = time.perf_counter()
        f_or = oracle.direct_forces(seg, burg, med, targets=tgt)
        cpu_s = time.perf_counter() - t0
        # the GPU FP64 direct sum that the error sample uses, checked against
        # the oracle on the same targets in this run
        f_gd = pk.direct_forces(plan, tseg, tb, targets=torch.tensor(tgt, device=dev), fp32=False).cpu().numpy()
        e_gd = float(np.linalg.norm(f_gd - f_or) / np.linalg.norm(f_or))
        result["cpu_baseline"] = {
            "value": k / cpu_s, "unit": "segments/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "%d target segment(s) x all %d source segments (direct FP64 sum, Neumaier), %.1f s"
                      % (k, ns, cpu_s)}
        result["gpu_direct_vs_oracle_rel_err"] = e_gd
        log("cpu oracle: %d segment(s) in %.1f s on %d threads (%s); GPU FP64 direct vs oracle %.2e"
            % (k, cpu_s, oracle.num_threads(), cpu_model(), e_gd))
    print(json.dumps(result), flush=True)


def bench_batch(args):
    """64 independent isotropic ensembles (5k..150k segments, log-uniform), one
    graph launch per step; depth per ensemble from the App. B autotuner."""
    import numpy as np
    import torch

    import paper_1712_07739_amd as pk
    import synth

    dev = torch.device("cuda:0")
    C = synth.loops.ISO
    order = args.order or 5
    t0 = time.perf_counter()
    ens = synth.make_batch(64, 4)
    sizes = [s.shape[0] for s, _ in ens]
    log("batch: %d ensembles, %d segments in total (generated in %.1f s)" % (len(ens), sum(sizes),
                                                                            time.perf_counter() - t0))
    segs = [torch.tensor(s, device=dev) for s, _ in ens]
    burgs = [torch.tensor(b, device=dev) for _, b in ens]
    # autotune on the median ensemble: optimal leaf density, then D_i for all
    med = int(np.argsort(sizes)[len(sizes) // 2])
    prm = pk.make_params(order, 5, *C, synth.loops.CORE_A, synth.loops.BOX_LO, synth.loops.BOX_SIZE,
                         precision=pk.DFMM_MIXED)
    d_med, pred, meas = pk.autotune_depth(prm, segs[med], burgs[med], 3, 7)
    dens = sizes[med] / 8.0 ** d_med
    depths = [int(min(7, max(3, round(np.log(n / dens) / np.log(8.0))))) for n in sizes]
    log("autotuner: median ensemble %d segments -> depth %d (predicted ms %s, measured ms %s); depths used %s"
        % (sizes[med], d_med, {k: round(v, 2) for k, v in pred.items()}, {k: round(v, 2) for k, v in meas.items()},
           {d: depths.count(d) for d in sorted(set(depths))}))
    plans = {d: pk.Plan(pk.make_params(order, d, *C, synth.loops.CORE_A, synth.loops.BOX_LO,
                                       synth.loops.BOX_SIZE, precision=pk.DFMM_MIXED_F16,
                                       m2l_mode=pk.DFMM_M2L_FFT_SYM)) for d in set(depths)}
    trees = [pk.Tree(plans[d], s) for d, s in zip(depths, segs)]
    outs = [torch.empty((n, 2, 3), dtype=torch.float64, device=dev) for n in sizes]
    lanes, lane_ms = pk.autotune_batch_lanes([plans[d] for d in depths], trees, segs, burgs, outs, reps=2)
    log("batch branches -> ms per replay %s: %d branches" % ({k: round(v, 2) for k, v in lane_ms.items()}, lanes))
    batch = pk.Batch([plans[d] for d in depths], trees, segs, burgs, outs, lanes=lanes)
    for _ in range(args.warmup):
        batch.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run()
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    lat = np.array(batch.latencies_ms())
    # accuracy on three ensembles against the GPU FP64 direct sum (40-segment samples)
    errs = []
    for i in (int(np.argmin(sizes)), med, int(np.argmax(sizes))):
        sub = synth.segment_subset(sizes[i], 40, 20000 + i)
        ref = pk.direct_forces(plans[depths[i]], segs[i], burgs[i], targets=torch.tensor(sub, device=dev)).cpu()
        f = outs[i].cpu().numpy()[sub]
        errs.append(float(np.linalg.norm(f - ref.numpy()) / np.linalg.norm(ref.numpy())))
    result = {
        "metric": "batched FMM force evaluation throughput, 64 ensembles of 5k-150k segments",
        "value": sum(sizes) / (ms_step * 1e-3), "unit": "segments/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16/f32", "data": "synthetic",
        "config": {"workload": "batch64", "n_ensembles": 64, "n_seg_total": int(sum(sizes)), "order": order,
                   "medium": "isotropic", "depths": {str(d): depths.count(d) for d in sorted(set(depths))},
                   "graph_lanes": lanes, "graph_lanes_ms": {str(k): v for k, v in lane_ms.items()}},
        "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
        "latency_ms_max": float(lat.max()), "rel_err_vs_fp64_direct_max": max(errs),
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
