"""Throughput of the kinetic DG time step on one MI355X.

One step = transport of every kinetic function (all subdomain iterations of
the downwind sweep) + relaxation, over the whole seeded workload, with the
state resident in HBM.  Prints ONE JSON line:

  value        cell-DOF-velocity updates per second (U / t_step), FP32 path
  roofline     dominant kernel vs the HBM roofline (algorithmic bytes / time)
  cpu_baseline the FP64 CPU oracle on a bounded sample of the same workload
  extra        the plain FP64 GPU sweep (the reference GPU path) and speedup;
               for the degree-3 workload (cfg4) also the front schedule's dense
               cell GEMM on matrix cores in FP32 and the FP16 / BF16 split forms

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg2]
       (--workload: cfg1..cfg4, maxwell, batch = 48 uneven problems together)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-DOF-velocity updates/s per step, FP32-MFMA batched vs plain FP64 sweep"
HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {"line": "k_sweep_line", "plain": "k_sweep_plain", "front": "k_sweep_front",
                "relax": "k_relax"}
MFMA_PEAK_TFS = {"fp32": 157.3, "fp32_split_f16": 2500.0, "fp32_split_bf16": 2500.0}
KERNEL_SOURCES = ["paper_2212_11010_amd/csrc/" + f for f in (
    "kds_internal.h", "kds_device.h", "kds_line.h", "kds_line_f32.hip", "kds_line_f64.hip",
    "kds_kernels.hip", "kds_front.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    return h.hexdigest()[:16]


def workload(name, cells=0, sub=0):
    from paper_2212_11010_amd import workloads as wl
    cfg = {"cfg1": 1, "cfg2": 2, "cfg3": 3, "cfg4": 4, "maxwell": 6}[name]
    kw = {}
    if cells:
        d = 2 if cfg in (1, 2) else 3
        kw["n_cells"] = [cells] * d
        kw["sub_cells"] = [sub or cells] * d
    return wl.make_workload(cfg, **kw)


def device_copy_gbs(nbytes=1 << 30, reps=10):
    """Practical streaming reference: torch device-to-device copy of nbytes,
    timed with events (read + written bytes per second)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def time_problem(spec, W0, prec, sched, steps, warmup, tune=False):
    import torch
    from paper_2212_11010_amd import kds
    pb = kds.Problem(spec, precision=prec, schedule=sched)
    pb.set_state(torch.from_numpy(W0).cuda())
    if tune:
        pb.tune(3)   # autotuner (setup, outside the timed region); restores the state
    info = pb.info()
    pb.step(warmup)
    pb.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pb.step(steps)
    pb.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_graph = (t1 - t0) * 1e3 / steps
    # per-kernel durations: HIP events recorded by the library on its stream
    # around `steps` back-to-back launches of each kernel (state restored)
    kms = pb.time_kernels(steps)
    ok = pb.check_finite()
    pb.close()
    return ms_graph, kms, info, ok


def traffic_record(kernel, wname, prec):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, if they were
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_%s.json" % (kernel, wname, prec))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def _pmc_per_dispatch(csv_path, name_part, last=0):
    """Average counter value (KiB per dispatch) of the kernels whose name
    contains name_part, from a rocprofv3 --pmc counter_collection.csv; with
    last > 0 only the last `last` dispatches (those after the autotuner)."""
    import csv
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(csv_path))
            if name_part in r["Kernel_Name"]]
    if last:
        vals = vals[-last:]
    return sum(vals) / len(vals), len(vals)


def pmc_summary(args):
    """Write profiles/traffic_<kernel>_<workload>_fp32.json from four rocprofv3
    --pmc runs (FETCH_SIZE and WRITE_SIZE of the workload, and of the plain
    1 GiB copy of --copy-probe, whose true bytes calibrate the counters)."""
    fetch_csv, write_csv, cfetch_csv, cwrite_csv = args.pmc_summary
    kname = KERNEL_NAMES[args.schedule if args.schedule != "auto" else "line"]
    # the counter runs use --steps 3 --warmup 1: 1 + 3 graph + 3 timed dispatches
    f_kib, nf = _pmc_per_dispatch(fetch_csv, kname, last=7)
    w_kib, nw = _pmc_per_dispatch(write_csv, kname, last=7)
    cf_kib, _ = _pmc_per_dispatch(cfetch_csv, "copyBuffer")
    cw_kib, _ = _pmc_per_dispatch(cwrite_csv, "copyBuffer")
    true_copy = float(1 << 30)
    rd_scale = true_copy / (cf_kib * 1024)
    wr_scale = true_copy / (cw_kib * 1024)
    rd = f_kib * 1024 * rd_scale
    wr = w_kib * 1024 * wr_scale
    spec, _ = workload(args.workload)
    from paper_2212_11010_amd import workloads as wl
    U = wl.unknowns(spec)
    rec = {"kernel": kname, "workload": args.workload, "precision": "fp32",
           "kernel_source_hash": kernel_source_hash(),
           "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib,
           "dispatches": [nf, nw],
           "copy_probe_fetch_kib": cf_kib, "copy_probe_write_kib": cw_kib,
           "read_scale": rd_scale, "write_scale": wr_scale,
           "hbm_bytes_per_launch": rd + wr, "hbm_read_bytes": rd, "hbm_write_bytes": wr,
           "algorithmic_bytes_per_launch": 8.0 * U,
           "ratio_to_algorithmic": (rd + wr) / (8.0 * U)}
    out = os.path.join(ROOT, "profiles", "traffic_%s_%s_fp32.json" % (kname, args.workload))
    json.dump(rec, open(out, "w"), indent=1)
    print(json.dumps(rec))


def gemm_variants(spec, W0, U, steps=2):
    """The front schedule (one dense cell GEMM per front on the matrix cores)
    in FP32 and the FP16 / BF16 split three-product forms, each against the
    FP64 front schedule (FMA; parity-tested against the FP64 oracle at 1e-12)
    after the same `steps` steps from the same state: ms per step, kernel ms,
    executed TFLOP/s against the variant's matrix peak, relative error of F."""
    import torch
    from paper_2212_11010_amd import kds

    def run(prec):
        pb = kds.Problem(spec, precision=prec, schedule="front")
        pb.set_state(torch.from_numpy(W0).cuda())
        pb.step(steps)
        F = torch.empty(pb.f_shape, dtype=torch.float64, device="cuda")
        pb.get_kinetic(F)
        pb.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb.step(steps)
        pb.synchronize()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        kms = pb.time_kernels(2)
        pb.close()
        return F, ms, kms

    Fref, ms64, k64 = run("fp64")
    scale = float(Fref.abs().max())
    P = spec["degree"] + 1
    nn = P ** spec["dim"]
    Kd = nn + 3 * (nn // P)
    out = {"steps_compared": steps, "fp64_front_ms_per_step": ms64,
           "fp64_front_sweep_ms": k64[0]}
    for prec in ("fp32", "fp32_split_f16", "fp32_split_bf16"):
        F, ms, kms = run(prec)
        err = float((F - Fref).abs().max()) / scale
        del F
        flops = 2.0 * Kd * U * (3 if "split" in prec else 1)
        tf = flops / (kms[0] * 1e-3) / 1e12
        out[prec] = {"ms_per_step": ms, "sweep_ms": kms[0], "executed_tflops": tf,
                     "peak_tflops": MFMA_PEAK_TFS[prec], "frac": tf / MFMA_PEAK_TFS[prec],
                     "rel_err_vs_fp64_front": err}
        log("front %s: %.3f ms/step, sweep %.3f ms, %.1f TFLOP/s, rel err %.2e"
            % (prec, ms, kms[0], tf, err))
    del Fref
    return out


def cpu_baseline(spec, W0, budget_s=12.0):
    from oracle import oracle
    cfg = oracle.Config(spec)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
    F = oracle.init(cfg, W0)
    t0 = time.perf_counter()
    F = oracle.step(cfg, F, 1, threads)
    t1 = time.perf_counter()
    one = t1 - t0
    n = max(1, min(20, int(budget_s / max(one, 1e-3))))
    t2 = time.perf_counter()
    F = oracle.step(cfg, F, n, threads)
    t3 = time.perf_counter()
    from paper_2212_11010_amd import workloads as wl
    U = wl.unknowns(spec)
    return {"value": U * n / (t3 - t2), "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d full time steps of the same workload (after 1 untimed), FP64 oracle, "
                      "OpenMP over (velocity, component) transports" % n}


def bench_batch(args):
    """The many-problem workloads, advanced together by kds_batch_step (grouped
    launches, one captured graph per step): "batch" = 48 seeded uneven
    problems (3.4e9 unknowns); "batch_small" = 256 small ones (acoustics
    32^2..64^2, Euler 8^3..16^3), each too small to fill the GPU alone."""
    import torch
    from paper_2212_11010_amd import kds
    from paper_2212_11010_amd import workloads as wl
    if args.workload == "batch_small":
        specs = wl.make_batch_workload(n_problems=256, max_unknowns=4e9, acoustics_n=(32, 48, 64),
                                       euler_n=(8, 12, 16), seed=wl.SEED_BASE + 55)
    else:
        specs = wl.make_batch_workload()
    U = sum(wl.unknowns(s) for s in specs)
    log("batch of %d problems, U=%d" % (len(specs), U))

    states = {}   # host copies of the seeded initial states (sampled once)

    def build(prec, sched, tune):
        members = []
        for s in specs:
            if s["name"] not in states:
                states[s["name"]] = wl.batch_member_state(s)
                log("  sampled %s (%d unknowns)" % (s["name"], wl.unknowns(s)))
            pb = kds.Problem(s, precision=prec, schedule=sched)
            pb.set_state(torch.from_numpy(states[s["name"]]).cuda())
            if tune:
                pb.tune(3)
            members.append(pb)
        return members

    members = build(args.precision, args.schedule, not args.no_tune)
    scheds = [{1: "plain", 2: "line", 3: "front"}[pb.info()["schedule"]] for pb in members]
    log("schedules: %s" % {k: scheds.count(k) for k in set(scheds)})
    b = kds.Batch(members)
    b.step(args.warmup)
    b.synchronize()
    torch.cuda.synchronize()
    ms_total = b.step_timed(args.steps)        # HIP events on the batch stream
    ms32 = ms_total / args.steps
    kms = b.time_kernels(args.steps)          # grouped sweep / relax launches per step
    # the same members stepped one problem at a time (each on its own
    # stream, with its own graphs: concurrent up to the hardware queues), and
    # step by step in turn, the order one stream would impose
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pb in members:
        pb.step(args.steps)
    for pb in members:
        pb.synchronize()
    ms_single = (time.perf_counter() - t0) * 1e3 / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for pb in members:
            pb.step(1)
            pb.synchronize()
    ms_serial = (time.perf_counter() - t0) * 1e3 / args.steps
    # and their own kernels' durations (line members; HIP events per problem)
    single_k = [0.0, 0.0]
    for pb, sc in zip(members, scheds):
        if sc == "line":
            k = pb.time_kernels(max(2, args.steps // 2))
            single_k[0] += k[0]
            single_k[1] += k[1]
    ok = all(pb.check_finite() for pb in members)
    log("batched %.3f ms/step (sweeps %.3f, relax %.3f), one by one %.3f ms/step"
        % (ms32, kms[0], kms[1], ms_single))
    b.close()
    U_line = sum(wl.unknowns(s) for s, sc in zip(specs, scheds) if sc == "line")
    for pb in members:
        pb.close()
    extra = {"schedules": {k: scheds.count(k) for k in set(scheds)},
             "grouped_kernel_ms": {"sweep": kms[0], "relax": kms[1]},
             "one_by_one_ms_per_step": ms_single,
             "serial_ms_per_step": ms_serial,
             "speedup_batched_vs_serial": ms_serial / ms32,
             "one_by_one_line_member_kernel_ms": {"sweep": single_k[0], "relax": single_k[1]},
             "speedup_batched_vs_one_by_one": ms_single / ms32,
             "state_finite": ok}
    if not args.no_fp64:
        m64 = build("fp64", "plain", False)
        n64 = max(2, args.steps // 10)
        b64 = kds.Batch(m64)
        b64.step(1)
        ms64 = b64.step_timed(n64) / n64
        b64.close()
        for pb in m64:
            pb.close()
        log("fp64 plain batch: %.3f ms/step" % ms64)
        extra.update({"fp64_plain_value": U / (ms64 * 1e-3), "fp64_plain_ms_per_step": ms64,
                      "speedup_fp32_vs_fp64_plain": ms64 / ms32})
    alg_bytes = 8.0 * U_line
    dur_s = kms[0] * 1e-3
    achieved = alg_bytes / dur_s / 1e9 if dur_s > 0 else 0.0
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_sweep_line_batch",
            "algorithmic_bytes_per_launch": alg_bytes, "avg_launch_ms": kms[0],
            "note": "sum over the grouped line-sweep launches of one step"}
    out = {
        "metric": METRIC, "value": U / (ms32 * 1e-3), "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms32,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("batch256_small_acoustics2d_euler3d" if args.workload == "batch_small"
                                else "batch48_acoustics2d_euler3d_mixed"), "problems": len(specs),
                   "unknowns": U, "n_iter": specs[0]["n_iter"]},
        "roofline": roof, "extra": extra,
    }
    if not args.no_cpu_baseline:
        from oracle import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
        u_done, t_done, names = 0, 0.0, []
        for s in sorted(specs, key=wl.unknowns):
            cfg = oracle.Config(s)
            F = oracle.init(cfg, states[s["name"]])
            t0 = time.perf_counter()
            oracle.step(cfg, F, 1, threads)
            t_done += time.perf_counter() - t0
            u_done += wl.unknowns(s)
            names.append(s["name"])
            if t_done > 12.0:
                break
        out["cpu_baseline"] = {"value": u_done / t_done, "unit": "updates/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "one time step of each of the %d smallest members "
                                         "(%d unknowns), FP64 oracle" % (len(names), u_done)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--schedule", default="auto")
    ap.add_argument("--cells", type=int, default=0, help="cells per axis (default: the workload's)")
    ap.add_argument("--sub", type=int, default=0, help="subdomain cells per axis with --cells")
    ap.add_argument("--precision", default="fp32", help="fp32 | fp32_split_f16 | fp32_split_bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-plan autotuner")
    ap.add_argument("--no-gemm-variants", action="store_true",
                    help="cfg4: skip the front-schedule GEMM variants (FP32 / FP16 / BF16 split)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates HBM counters)")
    ap.add_argument("--pmc-summary", nargs=4, metavar="CSV",
                    help="fetch.csv write.csv copy_fetch.csv copy_write.csv -> profiles/traffic_*.json")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args)
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                          "launches": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(subdomain sharding across GPUs is a design note, not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2212_11010_amd import workloads as wl

    if args.workload in ("batch", "batch_small"):
        bench_batch(args)
        return
    spec, W0 = workload(args.workload, args.cells, args.sub)
    U = wl.unknowns(spec)
    log("workload %s U=%d dt=%.5g nu=%.3f" % (spec["name"], U, spec["dt"], spec["kinetic_courant"]))

    ms32, k32, info32, ok32 = time_problem(spec, W0, args.precision, args.schedule, args.steps,
                                           args.warmup, tune=not args.no_tune)
    sched = {1: "plain", 2: "line", 3: "front"}[info32["schedule"]]
    log("fp32 %s: %.4f ms/step (graph), kernels %s ms" % (sched, ms32, k32))
    extra = {"fp32_schedule": sched, "fp32_kernel_ms": {"sweep": k32[0], "relax": k32[1]},
             "fp32_state_finite": ok32, "line_plan": {"cells_per_lane": info32["line_Q"][:spec["dim"]],
                                                      "columns_per_workgroup": info32["line_bw"][:spec["dim"]],
                                                      "autotuned": bool(info32["tuned"]),
                                                      "x_direct": bool(info32["line_xdirect"]),
                                                      "lds_bytes_per_workgroup": info32["line_lds_bytes"],
                                                      "step_launch": "enqueued" if info32["step_eager"] else "graph",
                                                      "relax_16byte_access": bool(info32["relax_vec"])}}
    if not args.no_fp64:
        base = "front" if sched == "front" else "plain"
        # (its step launch mode tuned too, so that both sides launch their best way)
        ms64, k64, info64, ok64 = time_problem(spec, W0, "fp64", base, max(5, args.steps // 5), 2,
                                               tune=not args.no_tune)
        log("fp64 plain: %.4f ms/step, kernels %s ms" % (ms64, k64))
        extra.update({"fp64_plain_value": U / (ms64 * 1e-3), "fp64_plain_ms_per_step": ms64,
                      "fp64_plain_kernel_ms": {"sweep": k64[0], "relax": k64[1]},
                      "speedup_fp32_vs_fp64_plain": ms64 / ms32})

    # dominant kernel and its algorithmic bytes: one read + one write of the
    # FP32 state per launch (sweep) -- see the design doc for the per-unknown figures
    dom = "sweep" if k32[0] >= k32[1] else "relax"
    kname = KERNEL_NAMES[sched] if dom == "sweep" else KERNEL_NAMES["relax"]
    bytes_per_unknown = 8.0
    alg_bytes = U * bytes_per_unknown
    dur_s = (k32[0] if dom == "sweep" else k32[1]) * 1e-3
    achieved = alg_bytes / dur_s / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_record(kname, args.workload, "fp32"),
            "kernel": kname, "algorithmic_bytes_per_launch": alg_bytes,
            "avg_launch_ms": dur_s * 1e3}

    roof["device_copy_gbs"] = device_copy_gbs()  # context: what a plain copy reaches
    # whole-step traffic: this schedule's algorithmic bytes per unknown, and
    # the literal scheme's (K sweeps each reading the state and its traces,
    # the last one writing it, then the relaxation: 32 B/U in FP32 at K = 3)
    step_bpu = {"line": 16.0, "plain": 4.0 * spec["n_iter"] + 4.0 + 8.0,
                "front": 8.0 * spec["n_iter"] + 8.0}[sched]
    literal_bpu = 8.0 * spec["n_iter"] + 8.0
    extra["step_hbm"] = {"bytes_per_unknown": step_bpu,
                         "frac": step_bpu * U / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "literal_scheme_bytes_per_unknown": literal_bpu,
                         "literal_scheme_frac": literal_bpu * U / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if sched == "front":
        # dense cell solves: 2 Kd flop per unknown per launch (one subdomain
        # iteration), Kd = nn + 3 nf; the split forms execute three products
        P = spec["degree"] + 1
        nn = P ** spec["dim"]
        Kd = nn + 3 * (nn // P)
        flops = 2.0 * Kd * U * (3 if "split" in args.precision else 1)
        sweep_s = k32[0] * 1e-3
        extra["front_mfma"] = {"executed_tflops": flops / sweep_s / 1e12,
                               "peak_tflops": MFMA_PEAK_TFS[args.precision],
                               "frac": flops / sweep_s / 1e12 / MFMA_PEAK_TFS[args.precision],
                               "hbm_gbs_algorithmic": 8.0 * U / sweep_s / 1e9}
    if args.workload == "cfg4" and sched != "front" and not args.no_gemm_variants:
        extra["front_gemm_variants"] = gemm_variants(spec, W0, U)
    out = {
        "metric": METRIC, "value": U / (ms32 * 1e-3), "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms32,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp32_split_f16": "f32 (f16x3 products)",
                  "fp32_split_bf16": "f32 (bf16x3 products)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": spec["name"], "n_cells": spec["n_cells"][:spec["dim"]],
                   "sub_cells": spec["sub_cells"][:spec["dim"]], "degree": spec["degree"],
                   "m": spec["m"], "n_vel": spec["n_vel"], "n_iter": spec["n_iter"],
                   "omega": spec["omega"], "cfl": spec["beta"], "unknowns": U},
        "roofline": roof,
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, W0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
