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

# The FP32 form measured on the axis-aligned D2Q4 / D3Q6 workloads is the line
# schedule (no dense cell operator: no matrix cores); the matrix-core front
# form of the same step is timed beside it in extra.fp32_mfma_front.
METRIC = ("cell-DOF-velocity updates/s per step, FP32 line-schedule sweep "
          "(FP32-MFMA front form in extra) vs plain FP64 sweep")
INFINITY_CACHE_BYTES = 256 << 20   # MI355X last-level (Infinity) cache
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


def time_problem(spec, W0, prec, sched, steps, warmup, tune=False, plan=None, front_kernel=0):
    """Returns (ms per step, [sweep, relax] ms per launch, info, state finite,
    launch plan)."""
    import torch
    from paper_2212_11010_amd import kds
    pb = kds.Problem(spec, precision=prec, schedule=sched)
    pb.set_state(torch.from_numpy(W0).cuda())
    if plan is not None:
        pb.set_plan(plan)
    elif tune:
        # autotuner (setup, outside the timed region); restores the state.  It
        # needs room for a copy of the state: without it the defaults stay
        try:
            pb.tune(3)
        except kds.KdsError as e:
            if e.status != kds.KDS_E_NOMEM:
                raise
            print("  (no device memory for the tuner's state copy: default launch plan)",
                  file=sys.stderr, flush=True)
    if front_kernel:
        # a forced front kernel (1: workgroup per subdomain, 2: wave per task)
        fp = pb.get_plan()
        fp["front_kernel"] = front_kernel
        pb.set_plan(fp)
    info = pb.info()
    plan = pb.get_plan()
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
    # the subdomain iteration's residual at the state reached (Sec. 5.1):
    # change of the outflow traces between the last two iterates
    try:
        d, v = pb.trace_residual()
        info["trace_residual"] = {"max_abs_change": d, "max_abs_trace": v,
                                  "relative": d / v if v > 0 else 0.0, "n_iter": spec["n_iter"]}
    except kds.KdsError as e:
        if e.status != kds.KDS_E_UNSUPPORTED:
            raise
    pb.close()
    return ms_graph, kms, info, ok, plan


def gpu_state_after(spec, W0, prec, sched, plan, n_steps):
    """(W, F) after n_steps from W0 with the given launch plan (host FP64)."""
    import torch
    from paper_2212_11010_amd import kds
    with kds.Problem(spec, precision=prec, schedule=sched) as pb:
        pb.set_plan(plan)
        pb.set_state(torch.from_numpy(W0).cuda())
        pb.step(n_steps)
        return pb.moments(), pb.get_kinetic()


def rel_errors(W, Wref, F, Fref):
    """max |x - x_oracle| / max |x_oracle| over all values (W and F), and the
    same per component of W / per (velocity, component) plane of F, each on
    its own scale; F in the C ABI layout [k][cell][node][c]."""
    def planes(a, b, red):
        # (a plane below 1e-6 of the largest is zero in exact arithmetic:
        # measured on the global scale)
        num = np.max(np.abs(a - b), axis=red)
        pmax, gmax = np.max(np.abs(b), axis=red), np.max(np.abs(b))
        return float(np.max(num / np.where(pmax >= 1e-6 * gmax, pmax, gmax)))
    g = lambda a, b: float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    return {"W": g(W, Wref), "F": g(F, Fref), "W_per_component": planes(W, Wref, (0, 1)),
            "F_per_plane": planes(F, Fref, (1, 2))}


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


def host_cpu():
    """nproc (affinity), os.cpu_count() and the CPU model of this host."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return {"nproc": nproc, "cpu_count": os.cpu_count(), "model": model}


def cpu_baseline(spec, W0, budget_s=10.0):
    """The FP64 oracle on this host, one thread and all threads (OpenMP over
    its independent (velocity, component) transports, so at most n_vel * m of
    them are busy).  Each leg: one untimed step, then about budget_s seconds
    of full steps.  Returns (record, oracle F after the all-thread leg
    [k][c][cell][node], steps it took)."""
    from oracle import oracle
    from paper_2212_11010_amd import workloads as wl
    cfg = oracle.Config(spec)
    U = wl.unknowns(spec)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
    tasks = spec["n_vel"] * spec["m"]
    F0 = oracle.init(cfg, W0)

    def leg(nt):
        F = oracle.step(cfg, F0, 1, nt)
        t0 = time.perf_counter()
        F = oracle.step(cfg, F, 1, nt)
        one = time.perf_counter() - t0
        n = max(1, min(20, int(budget_s / max(one, 1e-3))))
        t0 = time.perf_counter()
        F = oracle.step(cfg, F, n, nt)
        dt = time.perf_counter() - t0
        return U * (n + 1) / (dt + one), F, n + 2

    v1, _, n1 = leg(1)
    vt, F, nt_steps = leg(threads)
    busy = min(threads, tasks)
    rec = {"value": vt, "unit": "updates/s", "cores": busy, "kind": "oracle",
           "threads_requested": threads, "parallel_tasks": tasks,
           "single_thread_value": v1, "host": host_cpu(),
           "sample": "%d and %d full time steps of the same workload (one untimed first) on 1 "
                     "and on %d threads; FP64 oracle (g++ -O2), OpenMP over its %d independent "
                     "(velocity, component) transports, so at most %d threads busy"
                     % (n1 - 1, nt_steps - 1, threads, tasks, busy)}
    return rec, F, nt_steps


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
    # the batch's own launch shape (bundle widths of its line members)
    tune_ms = b.tune(3) if not args.no_tune else None
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
             "batch_tune_ms_per_step": tune_ms,
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
    ap.add_argument("--fp64-front-kernel", type=int, default=0, choices=(0, 1, 2),
                    help="front schedule, FP64 leg: 1 workgroup kernel, 2 wave kernel "
                         "(default: the library's choice)")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-plan autotuner")
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="skip the K = 1 and matrix-core front timings")
    ap.add_argument("--no-hbm-leg", action="store_true",
                    help="cfg2: skip the 128^3 Euler (HBM-bound) leg")
    ap.add_argument("--no-front-leg", action="store_true",
                    help="cfg2: skip the 64^3 D3Q4 Maxwell front-schedule leg")
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

    ms32, k32, info32, ok32, plan32 = time_problem(spec, W0, args.precision, args.schedule,
                                                   args.steps, args.warmup, tune=not args.no_tune)
    sched = {1: "plain", 2: "line", 3: "front"}[info32["schedule"]]
    log("fp32 %s: %.4f ms/step, kernels %s ms" % (sched, ms32, k32))
    extra = {"fp32_schedule": sched, "fp32_kernel_ms": {"sweep": k32[0], "relax": k32[1]},
             "fp32_state_finite": ok32, "fp32_plan": plan32,
             "line_plan": {"cells_per_lane": info32["line_Q"][:spec["dim"]],
                           "columns_per_workgroup": info32["line_bw"][:spec["dim"]],
                           "autotuned": bool(info32["tuned"]),
                           "x_direct": bool(info32["line_xdirect"]),
                           "lds_bytes_per_workgroup": info32["line_lds_bytes"],
                           "step_launch": "enqueued" if info32["step_eager"] else "graph",
                           "relax_16byte_access": bool(info32["relax_vec"])}}
    if "trace_residual" in info32:
        extra["trace_residual"] = info32["trace_residual"]
    if sched == "line":
        # the line kernel resolves all n_iter subdomain iterations in one launch
        extra["fp32_sweep_ms_per_iteration_equivalent"] = k32[0] / max(1, spec["n_iter"])
    plan64 = None
    if not args.no_fp64:
        base = "front" if sched == "front" else "plain"
        # (its step launch mode tuned too, so that both sides launch their best way)
        ms64, k64, info64, ok64, plan64 = time_problem(spec, W0, "fp64", base,
                                                       max(5, args.steps // 5), 2,
                                                       tune=not args.no_tune,
                                                       front_kernel=args.fp64_front_kernel)
        log("fp64 %s: %.4f ms/step, kernels %s ms" % (base, ms64, k64))
        extra.update({"fp64_plain_value": U / (ms64 * 1e-3), "fp64_plain_ms_per_step": ms64,
                      "fp64_plain_kernel_ms": {"sweep_per_iteration": k64[0], "relax": k64[1]},
                      "fp64_plain_launch": {
                          "step_launch": "enqueued" if info64["step_eager"] else "graph",
                          "relax_16byte_access": bool(info64["relax_vec"])},
                      "fp64_plain_state_finite": ok64,
                      "fp64_front_kernel": plan64.get("front_kernel", 0),
                      "speedup_fp32_vs_fp64_plain": ms64 / ms32})
    if sched == "line" and not args.no_extra_legs:
        # one subdomain iteration per step (K = 1): the step time the lag of
        # interface data alone costs
        spec1 = dict(spec, n_iter=1)
        ms1, k1, _, ok1, _ = time_problem(spec1, W0, args.precision, "auto", args.steps,
                                          args.warmup, tune=not args.no_tune)
        extra["k1_step"] = {"ms_per_step": ms1, "value": U / (ms1 * 1e-3), "sweep_ms": k1[0],
                            "relax_ms": k1[1], "state_finite": ok1}
        log("fp32 K=1: %.4f ms/step" % ms1)
        if spec["dim"] == 2 or U < 2e8:
            # the same step in the matrix-core form: fronts of the cell graph,
            # one dense GEMM (FP32 MFMA) per front, one launch per iteration
            msf, kf, _, okf, _ = time_problem(spec, W0, "fp32", "front", max(5, args.steps // 5),
                                              2, tune=not args.no_tune)
            P = spec["degree"] + 1
            nn = P ** spec["dim"]
            Kd = nn + 3 * (nn // P)
            tf = 2.0 * Kd * U / (kf[0] * 1e-3) / 1e12
            extra["fp32_mfma_front"] = {
                "ms_per_step": msf, "value": U / (msf * 1e-3), "sweep_ms_per_iteration": kf[0],
                "relax_ms": kf[1], "executed_tflops": tf, "peak_tflops": MFMA_PEAK_TFS["fp32"],
                "frac": tf / MFMA_PEAK_TFS["fp32"], "state_finite": okf,
                "note": "executed flops 2 (nn + 3 nf) per unknown and iteration (dense cell "
                        "operator); the axis-aligned velocities need ~2(p+1)+4 per unknown"}
            log("fp32 MFMA front: %.4f ms/step" % msf)

    # dominant kernel and its algorithmic bytes: one read + one write of the
    # FP32 state per launch (sweep) -- see the design doc for the per-unknown figures
    dom = "sweep" if k32[0] >= k32[1] else "relax"
    kname = KERNEL_NAMES[sched] if dom == "sweep" else KERNEL_NAMES["relax"]
    bytes_per_unknown = 8.0
    alg_bytes = U * bytes_per_unknown
    dur_s = (k32[0] if dom == "sweep" else k32[1]) * 1e-3
    achieved = alg_bytes / dur_s / 1e9
    state_bytes = info32["state_bytes"]
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_record(kname, args.workload, "fp32"),
            "kernel": kname, "algorithmic_bytes_per_launch": alg_bytes,
            "avg_launch_ms": dur_s * 1e3, "state_bytes": state_bytes,
            "cache_resident": state_bytes <= INFINITY_CACHE_BYTES}
    if roof["cache_resident"]:
        roof["note"] = ("the %.1f MB state fits the 256 MB Infinity Cache: the fraction is of the "
                        "HBM peak, the bytes mostly come from the cache (extra.hbm_leg_cfg3 is the "
                        "HBM-bound case)" % (state_bytes / 1e6))

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
    if args.workload == "cfg2" and not args.no_hbm_leg and args.cells == 0:
        extra["hbm_leg_cfg3"] = hbm_leg(args)
    if args.workload == "cfg2" and not args.no_front_leg and args.cells == 0:
        extra["front_leg_maxwell64"] = front_leg(args)
    out = {
        "metric": METRIC, "value": U / (ms32 * 1e-3), "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms32,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp32_split_f16": "f32 (f16x3 products)",
                  "fp32_split_bf16": "f32 (bf16x3 products)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": spec["name"], "schedule": sched, "n_cells": spec["n_cells"][:spec["dim"]],
                   "sub_cells": spec["sub_cells"][:spec["dim"]], "degree": spec["degree"],
                   "m": spec["m"], "n_vel": spec["n_vel"], "n_iter": spec["n_iter"],
                   "omega": spec["omega"], "cfl": spec["beta"], "unknowns": U},
        "roofline": roof,
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        rec, Forc, n_orc = cpu_baseline(spec, W0)
        out["cpu_baseline"] = rec
        # the measured paths against the oracle's state after the same steps
        # (the all-thread leg's): the FP32 path with the timed plan, and the
        # FP64 plain leg
        from oracle import oracle
        Wo = oracle.moments(oracle.Config(spec), Forc)
        Fo = np.ascontiguousarray(Forc.transpose(0, 2, 3, 1))
        del Forc
        err = {"steps": n_orc}
        Wg, Fg = gpu_state_after(spec, W0, args.precision, args.schedule, plan32, n_orc)
        err["fp32"] = rel_errors(Wg, Wo, Fg, Fo)
        if plan64 is not None:
            base = "front" if sched == "front" else "plain"
            Wg, Fg = gpu_state_after(spec, W0, "fp64", base, plan64, n_orc)
            err["fp64_plain"] = rel_errors(Wg, Wo, Fg, Fo)
        err["tolerance"] = {"fp32": 1e-5, "fp64": 1e-12}
        extra["error_vs_fp64_oracle"] = err
        log("error vs oracle after %d steps: %s" % (n_orc, err))
    print(json.dumps(out), flush=True)


def hbm_leg(args):
    """The 128^3 Euler p = 2 workload (6.8 GB FP32 state, HBM-bound): the
    FP32 step with the tuned plan, its kernels and their HBM fractions."""
    from paper_2212_11010_amd import workloads as wl
    t0 = time.perf_counter()
    spec, W0 = workload("cfg3")
    log("cfg3 state sampled in %.1f s" % (time.perf_counter() - t0))
    U = wl.unknowns(spec)
    ms, k, info, ok, plan = time_problem(spec, W0, "fp32", "auto", args.steps, args.warmup,
                                         tune=not args.no_tune)
    del W0
    sched = {1: "plain", 2: "line", 3: "front"}[info["schedule"]]
    log("cfg3 fp32 %s: %.3f ms/step, kernels %s ms" % (sched, ms, k))
    gbs = lambda b, ms_: b / (ms_ * 1e-3) / 1e9
    return {"workload": spec["name"], "n_cells": spec["n_cells"], "sub_cells": spec["sub_cells"],
            "degree": spec["degree"], "unknowns": U, "schedule": sched, "plan": plan,
            "ms_per_step": ms, "value": U / (ms * 1e-3), "sweep_ms": k[0], "relax_ms": k[1],
            "sweep_hbm_frac": gbs(8.0 * U, k[0]) / HBM_PEAK_GBS,
            "relax_hbm_frac": gbs(8.0 * U, k[1]) / HBM_PEAK_GBS,
            "step_hbm_frac": gbs(16.0 * U, ms) / HBM_PEAK_GBS,
            "literal_scheme_step_frac": gbs(32.0 * U, ms) / HBM_PEAK_GBS,
            "state_bytes": info["state_bytes"], "state_finite": ok}


def front_leg(args):
    """The paper's own velocity set: D3Q4 Maxwell, 64^3 cells, 8^3-cell
    subdomains, p = 2, FP32 front schedule (one launch per subdomain
    iteration, dense cell GEMMs on the matrix cores).  Algorithmic figures
    per launch: one read and one write of the state (8 B per unknown) and
    2 n_n (n_n + 3 n_f) flop per cell column of every (velocity, component)."""
    from paper_2212_11010_amd import workloads as wl
    spec, W0 = workload("maxwell", 64, 8)
    U = wl.unknowns(spec)
    ms, k, info, ok, plan = time_problem(spec, W0, "fp32", "front", max(5, args.steps // 4), 2,
                                         tune=False)
    log("maxwell 64^3 fp32 front: %.3f ms/step, kernels %s ms" % (ms, k))
    nn = (spec["degree"] + 1) ** 3
    nf = (spec["degree"] + 1) ** 2
    cols = U // nn                               # cell columns over all (velocity, component)
    flops = 2.0 * nn * (nn + 3 * nf) * cols
    sweep_s = k[0] * 1e-3
    return {"workload": spec["name"], "n_cells": spec["n_cells"], "sub_cells": spec["sub_cells"],
            "degree": spec["degree"], "unknowns": U, "front_kernel": plan.get("front_kernel"),
            "ms_per_step": ms, "value": U / (ms * 1e-3), "sweep_ms_per_iteration": k[0],
            "relax_ms": k[1], "sweep_hbm_frac": 8.0 * U / sweep_s / 1e9 / HBM_PEAK_GBS,
            "sweep_algorithmic_tflops": flops / sweep_s / 1e12,
            "sweep_mfma_frac": flops / sweep_s / 1e12 / MFMA_PEAK_TFS["fp32"],
            "state_finite": ok}


if __name__ == "__main__":
    main()
