#!/usr/bin/env python3
"""Benchmark: supernodal LDL^T + selected inversion of a 3D Laplacian on one GPU.

A step is one pass of the whole hot path on device-resident input: numeric
factorization (assemble, diagonal LDL^T, panels with the normalised L_hat,
Schur updates) followed by the root-to-leaf selected inversion (gathered
GEMMs, diagonal blocks) and the export of the selected values.  The default
workload is the 64^3 variable-coefficient Laplacian with supernodes capped
at 256 columns.

Prints ONE JSON line.  `value` is algorithmic FP64 GFLOP/s of the step
(fundamental-supernode flop counts of factor + selected inversion divided by
the step time).  `roofline` covers the kernel kind with the largest share of
device time, timed live with HIP events stamped in each dispatch during a
second pass over the same K steps (the stamps cost time of their own, so
`ms_per_step` comes from the pass without them); `peaks` holds the device's
measured FP64 MFMA and copy ceilings beside the published ones.
`cpu_baseline` times the CPU oracle (test infrastructure, untuned) on a
bounded sample of the same workload.  More parts of the metric ride on the
same line: `backward` (the reverse sweep's time over the forward step's,
same matrix, without and with checkpointing of the inverse panels),
`deterministic` (the atomic-free mode's step), `extra_workloads` (the 40^3
grid and the molecular matrix) and `batched` (256 independent 2D grids: the
batch on the persistent per-level kernels replayed from a HIP graph, against
a loop of per-matrix runs with per-level launches, same kernels, same GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "selinv FP64 GFLOP/s + % MFMA peak (3D Laplacian); batched speedup; bwd/fwd"
PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 matrix peak; the FP64 vector peak is the same
# (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz)
PEAK_HBM_GBS = 8000.0
WORKLOADS = {
    "lap3d_40": "3D 7-point Laplacian, 40^3 grid (n=64000), edge conductivities U[0.5,2] seed 2, shift 1e-2, "
                "nested dissection, fundamental supernodes capped at 128",
    "lap3d_64": "3D 7-point Laplacian, 64^3 grid (n=262144), conductivities log-uniform [0.1,10] seed 5, "
                "shift 1e-3, nested dissection, supernodes capped at 256",
    "lap2d_32": "2D 5-point Laplacian, 32x32 grid (n=1024), shift 0.1, supernodes capped at 128",
    "molecular_16": "block-sparse SPD matrix on a jittered 16^3 atom lattice, 8 unknowns per atom (n=32768), "
                    "8x8 N(0,1) blocks within 1.8 lattice spacings, diagonal shift, seed 4, supernodes capped at 128",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def native_sources_sha256():
    """Hash of the native sources (kernels, schedule, host code): the work of
    a launch depends on all of them."""
    import hashlib
    d = os.path.join(ROOT, "paper_1404_0447_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".cpp", ".hpp")):
            h.update(name.encode())
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, kind):
    """HBM bytes per dispatch of a kernel kind (FETCH_SIZE + WRITE_SIZE, each
    scaled by the same counter's reading for a plain 1 GiB copy), from the
    rocprofv3 summary under profiles/; None when there is none for this
    workload or the native sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    rec, sha = {}, None
    for line in open(path):
        f = line.split()
        if len(f) == 5 and f[0] == "traffic":
            rec[f[1]] = float(f[3]) + float(f[4])
        elif len(f) == 2 and f[0] == "sources_sha256_16":
            sha = f[1]
    now = native_sources_sha256()[:16]
    if sha != now or kind not in rec:
        return None
    return round(rec[kind], 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lap3d_64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fuse", action="store_true", help="run fundamental supernodes unamalgamated")
    ap.add_argument("--no-bwd", action="store_true", help="skip the backward (adjoint) timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-speedup measurement")
    ap.add_argument("--no-extra", action="store_true", help="skip the 40^3 and molecular side measurements")
    ap.add_argument("--no-det", action="store_true", help="skip the deterministic-mode step")
    ap.add_argument("--no-poles", action="store_true", help="skip the complex pole-batch measurement")
    ap.add_argument("--no-pivot", action="store_true", help="skip the symmetric indefinite (2x2 pivots) measurement")
    ap.add_argument("--checkpoint-every", type=int, default=4,
                    help="checkpoint interval of the second backward measurement (0: skip it)")
    ap.add_argument("--batch-reps", type=int, default=10, help="timed replays of the batched graph")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched measurement, printed as its own JSON line (for profiling it)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain device copy of 1 GiB (read 1 GiB, write 1 GiB) three times: the "
                         "reference dispatch for scaling FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the multi-GPU "
              "design is described but not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calib:
        n = 1 << 27  # doubles: 1 GiB
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0.0, out=dst)  # one elementwise kernel: reads src, writes dst
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read": n * 8, "copy_calib_bytes_written": n * 8, "dispatches": 3}))
        return
    if args.batch_only:
        print(json.dumps({"batched": measure_batched(args, dev)}))
        return
    t0 = time.time()
    m = W.make(args.workload)
    cap = W.CONFIGS[args.workload]["cap"]
    log(f"[bench] generated {args.workload}: n={m.n} nnzA={m.nnz} ({time.time() - t0:.1f}s)")
    t0 = time.time()
    plan = S.Plan.from_matrix(m, max_super=cap, fuse_chains=not args.no_fuse)
    info = plan.info
    log(f"[bench] analyze: nsuper={info['nsuper']} depth={info['depth']} blocks={info['nblocks']} "
        f"exec_depth={info['exec_depth']} nnzL={info['nnzL']} ({time.time() - t0:.1f}s)")
    plan.bind(device=dev)
    vals = torch.as_tensor(m.vals, dtype=torch.float64, device=dev)
    out = torch.empty(int(info["nnzL"]), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        plan.factor(vals)
        plan.invert(out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.sync_status()
    log(f"[bench] warmup done ({args.warmup} steps)")

    # timed region: K steps, nothing but the launches of the path
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        step()
    stop.record(stream)
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(stop)
    ms_step = ms_total / args.steps
    plan.sync_status()
    log(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step")
    # the same K steps again with a HIP event pair stamped around every
    # dispatch (on the stream it runs on): per-kernel durations for the
    # roofline; the stamps cost time of their own, so the step time above
    # comes from the run without them
    plan.profile(True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        step()
    stop.record(stream)
    torch.cuda.synchronize()
    plan.profile(False)
    ms_step_prof = start.elapsed_time(stop) / args.steps
    prof = plan.profile_read()
    plan.sync_status()
    log(f"[bench] profiled {args.steps} steps: {ms_step_prof:.3f} ms/step")
    # the same K steps once more, an event pair around each: the spread
    # of single steps (mean, std, median)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    plan.sync_status()
    per_step = np.array([a.elapsed_time(b) for a, b in evs])

    work = plan.kernel_work()
    flops_step = info["flops_factor"] + info["flops_selinv"]
    value = flops_step / (ms_step * 1e-3) / 1e9
    kern_ms = {k: prof[k][0] / args.steps for k in prof}
    dom = max(kern_ms, key=lambda k: kern_ms[k])
    per_launch = {k: (prof[k][0] / prof[k][1] if prof[k][1] else 0.0) for k in prof}
    launches_per_step = {k: prof[k][1] / args.steps for k in prof}
    hbm_kinds = ("assemble", "export")
    alu_kinds = ("ldlt",)  # FP64 vector Gauss-Jordan sweep: s dependent pivot steps per block
    if dom in hbm_kinds:
        achieved = work[dom][1] / (kern_ms[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None}
    elif dom in alu_kinds:
        achieved = work[dom][0] / (kern_ms[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None}
    else:
        achieved = work[dom][0] / (kern_ms[dom] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None}
    roof["traffic"] = measured_traffic(args.workload, dom)  # HBM bytes per launch
    roof["traffic_unit"] = "bytes per launch"
    roof.update({"kernel": dom, "avg_launch_ms": round(per_launch[dom], 5),
                 "launches_per_step": launches_per_step[dom],
                 "algorithmic_per_step": work[dom][0] if roof["unit"] == "TFLOP/s" else work[dom][1]})
    # GEMM phase (steps 3-4 of the selected inversion): the tiled kernels and
    # the small-block kernel that runs both steps for blocks with s <= 16
    gemm_phase_ms = kern_ms["gemm"] + kern_ms["sdiag"] + kern_ms["sbinvert"]
    gemm_phase_tf = info["flops_gemm"] / (gemm_phase_ms * 1e-3) / 1e12 if gemm_phase_ms > 0 else 0.0
    invert_ms = gemm_phase_ms + kern_ms["export"]
    factor_ms = sum(kern_ms[k] for k in ("assemble", "ldlt", "panel", "schur", "sbfactor"))

    log("[bench] device ceilings: FP64 MFMA loop and copy ...")
    mf_tf, copy_gbs = S.measure_peaks(device=dev)
    roof["measured_peak"] = round(mf_tf if roof["unit"] == "TFLOP/s" else copy_gbs, 2)
    roof["frac_of_measured_peak"] = round(roof["achieved"] / roof["measured_peak"], 4) if roof["measured_peak"] else None
    log(f"[bench] measured FP64 MFMA {mf_tf:.1f} TFLOP/s, copy {copy_gbs:.0f} GB/s")

    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "n": m.n, "nnzA": m.nnz,
                   "nnzL": info["nnzL"], "nsuper": info["nsuper"], "depth": info["depth"],
                   "exec_blocks": info["nblocks"], "exec_depth": info["exec_depth"],
                   "flops_factor": info["flops_factor"], "flops_selinv": info["flops_selinv"],
                   "fuse_chains": not args.no_fuse},
        "roofline": roof,
        "ms_per_step_profiled": round(ms_step_prof, 4),
        "phases_ms": {"factor_kernels": round(factor_ms, 4), "invert_kernels": round(invert_ms, 4),
                      **{k: round(v, 4) for k, v in kern_ms.items()}},
        "gemm_phase": {"tflops": round(gemm_phase_tf, 4), "frac_of_fp64_peak": round(gemm_phase_tf / PEAK_FP64_TFLOPS, 4),
                       "flops": info["flops_gemm"], "ms": round(gemm_phase_ms, 4)},
        # measured HBM bytes per launch (rocprof counters, when they match
        # the sources) over the average launch time: the gather-GEMM's
        # gather and the export's copy, against 8 TB/s
        "hbm_gbs": {k: (round(measured_traffic(args.workload, k) / (per_launch[k] * 1e-3) / 1e9, 1)
                        if measured_traffic(args.workload, k) and per_launch.get(k) else None)
                    for k in ("gemm", "export")},
        "factor_gflops": round(info["flops_factor"] / (factor_ms * 1e-3) / 1e9, 2) if factor_ms > 0 else None,
        "invert_gflops": round(info["flops_selinv"] / (invert_ms * 1e-3) / 1e9, 2) if invert_ms > 0 else None,
        "step_ms": {"mean": round(float(per_step.mean()), 4), "std": round(float(per_step.std()), 4),
                    "median": round(float(np.median(per_step)), 4), "runs": int(per_step.size)},
        "peaks": {"fp64_mfma_tflops_measured": round(mf_tf, 2), "fp64_mfma_tflops_published": PEAK_FP64_TFLOPS,
                  "copy_gbs_measured": round(copy_gbs, 1), "hbm_gbs_published": PEAK_HBM_GBS,
                  "gemm_phase_frac_of_measured": round(gemm_phase_tf / mf_tf, 4) if mf_tf > 0 else None},
        "cpu_baseline": None,
    }

    if not args.no_bwd:
        result["backward"] = measure_backward(plan, vals, out, ms_step, args, dev)
        if args.checkpoint_every > 1:
            del plan  # its workspace is not needed any more
            torch.cuda.empty_cache()
            result["backward"]["checkpointed"] = measure_checkpointed(m, cap, args, dev, ms_step,
                                                                      result["backward"].get("grad_probe"))
    if not args.no_det:
        result["deterministic"] = measure_deterministic(m, cap, args, dev, ms_step, out)
    if not args.no_extra:
        result["extra_workloads"] = {w: measure_extra(w, args, dev) for w in ("lap3d_40", "molecular_16")
                                     if w != args.workload}
    if not args.no_batch:
        result["batched"] = measure_batched(args, dev)
    if not args.no_poles:
        result["poles"] = measure_poles(args, dev)
    if not args.no_pivot:
        result["pivoting"] = measure_pivoting(args, dev)

    if not args.no_cpu:
        result["cpu_baseline"], err = cpu_baseline(m, args.workload, cap, flops_step, value, out)
        if err is not None:
            result["max_err_vs_oracle"] = err
    if "backward" in result:
        result["backward"].pop("grad_probe", None)
    print(json.dumps(result), flush=True)


def _time(fn, reps, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(reps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps


def sub_box(m, dims, box_hi):
    """Principal submatrix of a grid matrix on the points [0, box_hi) (x, y,
    z), as a grid matrix of its own.  When the box is a subtree of the
    nested dissection of the full grid, its factorization is that subtree's
    part of the full factorization."""
    import numpy as np
    from paper_1404_0447_amd import workloads as W
    nx, ny, nz = dims
    idx = np.arange(m.n)
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    keep = (x < box_hi[0]) & (y < box_hi[1]) & (z < box_hi[2])
    new = np.full(m.n, -1, np.int64)
    new[keep] = x[keep] + box_hi[0] * (y[keep] + box_hi[1] * z[keep])
    cols = np.repeat(np.arange(m.n), np.diff(m.colptr))
    r, c = m.rowind.astype(np.int64), cols
    sel = keep[r] & keep[c]
    rr, cc, vv = new[r[sel]], new[c[sel]], m.vals[sel]
    n = int(keep.sum())
    colptr = np.zeros(n + 1, np.int64)
    np.add.at(colptr, cc + 1, 1)
    colptr = np.cumsum(colptr)
    order = np.lexsort((rr, cc))
    return W.Matrix(n, colptr, rr[order].astype(np.int32), vv[order], ndim=3, dims=tuple(box_hi), dofs=1)


def cpu_baseline(m, workload, cap, flops_step, gpu_gflops, out):
    """The oracle (its factor + selected inversion, symbolic phase excluded)
    on the host cores: the whole matrix when it is small, else the half box
    [0,32) x [0,64) x [0,64) of the 64^3 grid, which is the subtree its nested
    dissection orders first (n = 131,072, about 7 s of CPU work a run on 16
    threads).  The figure is the median of three runs; one single-thread run
    on the 32^3 corner box (the whole matrix when it is small) sits beside it."""
    import numpy as np
    from oracle import oracle as O
    if workload == "lap3d_64":
        sample_m = sub_box(m, m.dims, (32, 64, 64))
        # the sub-box, in its own nested-dissection order, is exactly the
        # first subtree of the full grid's order
        i = np.arange(sample_m.n)
        to_full = (i % 32) + 64 * ((i // 32) % 64) + 4096 * (i // 2048)
        full = O.nd_order(3, m.dims)
        assert np.array_equal(full[:sample_m.n], to_full[O.nd_order(3, (32, 64, 64))])
        sample = ("principal submatrix of the 64^3 matrix on the half box [0,32)x[0,64)x[0,64), the first "
                  "subtree of its nested dissection (n=131072), cap 256")
        single_m = sub_box(m, m.dims, (32, 32, 32))
        single = "principal submatrix of the 64^3 matrix on the corner box [0,32)^3 (n=32768), cap 256"
    else:
        sample_m, sample = m, f"the whole {workload} matrix"
        single_m, single = m, sample
    log(f"[bench] cpu baseline: oracle symbolic on {sample_m.n} unknowns ...")
    osym = O.symbolic(sample_m, cap=cap)
    fl = osym.sym.factor_flops + selinv_flops(osym.sym)
    log("[bench] cpu baseline: oracle factor + selected inversion, three runs ...")
    runs, ref = [], None
    t0 = time.time()
    for _ in range(3):
        ref, _, st, _, tf, ts = osym.factor_selinv(sample_m.vals)
        assert st == 0
        runs.append(tf + ts)
    wall = time.time() - t0
    t_med = float(np.median(runs))
    cpu_gflops = fl / t_med / 1e9
    err = None
    if sample_m is m:
        got = out.cpu().numpy()
        cp, ri = osym.sym.colptrL, osym.sym.rowindL
        d = ref[cp[:-1]]
        cols = np.repeat(np.arange(m.n), np.diff(cp))
        err = float(np.max(np.abs(got - ref) / np.sqrt(np.abs(d[ri] * d[cols]))))
    cores = O.threads()
    # one thread, smaller sample
    osym1 = O.symbolic(single_m, cap=cap)
    fl1 = osym1.sym.factor_flops + selinv_flops(osym1.sym)
    O.set_threads(1)
    try:
        _, _, st, _, tf1, ts1 = osym1.factor_selinv(single_m.vals)
    finally:
        O.set_threads(cores)
    assert st == 0
    cpu_model = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
                      if ln.startswith("model name")), "unknown")
    res = {"value": round(cpu_gflops, 3), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model, "nproc": os.cpu_count(),
           "sample": f"{sample}: factor + selected inversion (symbolic excluded), {fl:.3e} flops, median of "
                     f"3 runs ({', '.join(f'{r:.2f}' for r in runs)} s)",
           "runs_s": [round(r, 3) for r in runs],
           "single_thread": {"value": round(fl1 / (tf1 + ts1) / 1e9, 3), "unit": "GFLOP/s", "cores": 1,
                             "sample": f"{single}: {fl1:.3e} flops in {tf1 + ts1:.2f}s, one run"},
           "speedup_gpu_over_cpu": round(gpu_gflops / cpu_gflops, 2)}
    log(f"[bench] oracle median {t_med:.2f}s of 3 ({wall:.1f}s wall) = {cpu_gflops:.2f} GFLOP/s on {cores} threads; "
        f"1 thread {res['single_thread']['value']:.2f} GFLOP/s on n={single_m.n}")
    return res, err


def selinv_flops(sym):
    """Sum of 2c^2 s + 3cs^2 + 2s^3/3 over the oracle's supernodes."""
    import numpy as np
    s = np.diff(sym.xsuper).astype(np.float64)
    c = np.diff(sym.cptr).astype(np.float64)
    return float(np.sum(2 * c * c * s + 3 * c * s * s + 2.0 / 3.0 * s ** 3))


def time_forward(plan, vals, out, steps, warmup, stream, profile=False):
    """(ms per factor + invert step, per-kind profile or None)."""
    import torch

    def step():
        plan.factor(vals)
        plan.invert(out)
    for _ in range(warmup):
        step()
    plan.sync_status()
    ms = _time(step, steps, stream)
    prof = None
    if profile:
        plan.profile(True)
        _time(step, steps, stream)
        plan.profile(False)
        prof = plan.profile_read()
    plan.sync_status()
    return ms, prof


def measure_checkpointed(m, cap, args, dev, fwd_ms, grad_probe):
    """Backward with checkpointing: the inverse panels of every k-th level
    are copied to the persistent store by the forward, the transient memory
    (inverse panels and adjoint arenas) is released between forward and
    backward, and the backward restores the checkpoints and recomputes the
    other levels before the reverse sweep."""
    import numpy as np
    import torch
    from paper_1404_0447_amd import selinv as S
    k = args.checkpoint_every
    stream = torch.cuda.current_stream()
    p = S.Plan.from_matrix(m, max_super=cap, checkpoint_every=k).bind(device=dev)
    vals = torch.as_tensor(m.vals, dtype=torch.float64, device=dev)
    out = torch.empty(int(p.info["nnzL"]), dtype=torch.float64, device=dev)
    fwd_k, _ = time_forward(p, vals, out, args.steps, args.warmup, stream)
    g = torch.as_tensor(np.random.default_rng(0).standard_normal(int(p.info["nnzL"])), device=dev)
    gA = torch.empty(int(p.info["nnzA"]), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    p.factor(vals)
    p.invert(out)
    p.release_transient()
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated(dev)
    torch.cuda.reset_peak_memory_stats(dev)
    p.backward(g, out=gA)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated(dev)
    for _ in range(max(1, args.warmup) - 1):
        p.backward(g, out=gA)
    bwd = _time(lambda: p.backward(g, out=gA), args.steps, stream)
    p.profile(True)
    _time(lambda: p.backward(g, out=gA), args.steps, stream)
    p.profile(False)
    prof = p.profile_read()
    p.sync_status()
    res = {"checkpoint_every": k, "fwd_ms": round(fwd_k, 4), "bwd_ms": round(bwd, 4),
           "bwd_over_fwd": round(bwd / fwd_ms, 3), "bwd_over_own_fwd": round(bwd / fwd_k, 3),
           "recompute_ms": round((prof["gemm"][0] + prof["sdiag"][0] + prof["sbinvert"][0]) / args.steps, 4),
           "checkpoint_copy_ms": round(prof["checkpoint"][0] / args.steps, 4),
           "persistent_bytes": p.persistent_bytes, "transient_bytes": p.transient_bytes,
           "checkpoint_store_bytes": int(p.kernel_work()["checkpoint"][1] / 2),
           "device_bytes_held_between_fwd_and_bwd": int(held),
           "device_bytes_held_without_checkpointing": int(held + p.transient_bytes),
           "device_peak_bytes_in_backward": int(peak)}
    if grad_probe is not None:
        gk = gA[: len(grad_probe)].cpu().numpy()
        res["grad_max_rel_diff_vs_full"] = float(np.abs(gk - grad_probe).max() / max(np.abs(grad_probe).max(), 1e-300))
    log(f"[bench] backward with checkpoint_every={k}: {bwd:.3f} ms ({bwd / fwd_ms:.2f}x forward), "
        f"held {held / 1e9:.2f} GB between forward and backward (vs {(held + p.transient_bytes) / 1e9:.2f} GB)")
    del p
    torch.cuda.empty_cache()
    return res


def measure_deterministic(m, cap, args, dev, fwd_ms, out_ref):
    """The atomic-free mode on the same matrix: step time, and two runs
    compared bit for bit."""
    import numpy as np
    import torch
    from paper_1404_0447_amd import selinv as S
    stream = torch.cuda.current_stream()
    p = S.Plan.from_matrix(m, max_super=cap, deterministic=True).bind(device=dev)
    vals = torch.as_tensor(m.vals, dtype=torch.float64, device=dev)
    out = torch.empty(int(p.info["nnzL"]), dtype=torch.float64, device=dev)
    ms, prof = time_forward(p, vals, out, args.steps, args.warmup, stream)
    a = out.clone()
    p.factor(vals)
    p.invert(out)
    p.sync_status()
    same = bool(torch.equal(a, out))
    diff = float((out - out_ref).abs().max().item())
    log(f"[bench] deterministic step {ms:.3f} ms ({ms / fwd_ms:.2f}x), bitwise repeatable: {same}")
    del p
    torch.cuda.empty_cache()
    return {"ms_per_step": round(ms, 4), "over_default": round(ms / fwd_ms, 3), "bitwise_repeatable": same,
            "max_abs_diff_vs_default": diff}


def measure_extra(workload, args, dev):
    """Forward step (and for the molecular matrix the backward) of another
    configuration, with the GEMM phase from stamped kernel times."""
    import numpy as np
    import torch
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    stream = torch.cuda.current_stream()
    t0 = time.time()
    m = W.make(workload)
    cap = W.CONFIGS[workload]["cap"]
    p = S.Plan.from_matrix(m, max_super=cap).bind(device=dev)
    info = p.info
    vals = torch.as_tensor(m.vals, dtype=torch.float64, device=dev)
    out = torch.empty(int(info["nnzL"]), dtype=torch.float64, device=dev)
    ms, prof = time_forward(p, vals, out, args.steps, args.warmup, stream, profile=True)
    kern = {k: prof[k][0] / args.steps for k in prof}
    gp = kern["gemm"] + kern["sdiag"] + kern["sbinvert"]
    gtf = info["flops_gemm"] / (gp * 1e-3) / 1e12 if gp > 0 else 0.0
    res = {"workload": WORKLOADS[workload], "ms_per_step": round(ms, 4),
           "gflops": round((info["flops_factor"] + info["flops_selinv"]) / (ms * 1e-3) / 1e9, 2),
           "gemm_phase_tflops": round(gtf, 3), "gemm_phase_frac_of_fp64_peak": round(gtf / PEAK_FP64_TFLOPS, 4),
           "ldlt_ms": round(kern["ldlt"], 4), "dominant_kernel": max(kern, key=lambda k: kern[k])}
    if workload == "molecular_16":
        g = torch.as_tensor(np.random.default_rng(0).standard_normal(int(info["nnzL"])), device=dev)
        gA = torch.empty(int(info["nnzA"]), dtype=torch.float64, device=dev)
        p.factor(vals)
        p.invert(out)
        p.backward(g, out=gA)
        bwd = _time(lambda: p.backward(g, out=gA), args.steps, stream)
        res["bwd_ms"] = round(bwd, 4)
        res["bwd_over_fwd"] = round(bwd / ms, 3)
    p.sync_status()
    log(f"[bench] {workload}: {ms:.3f} ms/step, GEMM phase {gtf:.1f} TFLOP/s ({time.time() - t0:.1f}s)")
    del p
    torch.cuda.empty_cache()
    return res


def measure_pivoting(args, dev):
    """Symmetric indefinite saddle-point matrix on the 16^3-atom molecular
    pattern (seed 8, 8 unknowns per atom, n = 32768), factored with 1x1/2x2
    Bunch-Kaufman pivots inside the diagonal blocks, against the SPD
    molecular matrix of the same pattern (same seed, shifted) on the default
    path: the cost of pivoting."""
    import torch
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    stream = torch.cuda.current_stream()
    t0 = time.time()
    mi = W.indefinite_molecular(side=16, dofs=8, seed=8)
    ms_spd = W.molecular(side=16, dofs=8, seed=8)
    res = {"workload": "saddle-point blocks [[0, I], [I, 0]] per atom on a jittered 16^3-atom lattice x 8 (n=32768), "
                       "other entries 0.08 x N(0,1) blocks, seed 8, supernodes capped at 128"}
    for key, m, kw in (("pivoted", mi, {"pivoting": True}), ("spd_same_pattern", ms_spd, {})):
        p = S.Plan.from_matrix(m, max_super=128, **kw).bind(device=dev)
        vals = torch.as_tensor(m.vals, dtype=torch.float64, device=dev)
        out = torch.empty(int(p.info["nnzL"]), dtype=torch.float64, device=dev)
        ms, prof = time_forward(p, vals, out, args.steps, args.warmup, stream, profile=True)
        res[key] = {"ms_per_step": round(ms, 4), "ldlt_ms": round(prof["ldlt"][0] / args.steps, 4),
                    "gflops": round((p.info["flops_factor"] + p.info["flops_selinv"]) / (ms * 1e-3) / 1e9, 2)}
        del p
        torch.cuda.empty_cache()
    res["pivoted_over_spd"] = round(res["pivoted"]["ms_per_step"] / res["spd_same_pattern"]["ms_per_step"], 3)
    log(f"[bench] pivoting: indefinite {res['pivoted']['ms_per_step']:.3f} ms/step (diagonal blocks "
        f"{res['pivoted']['ldlt_ms']:.3f} ms), SPD on the same pattern {res['spd_same_pattern']['ms_per_step']:.3f} ms "
        f"({time.time() - t0:.1f}s)")
    return res


def measure_poles(args, dev):
    """Complex symmetric A(z_k) = H - z_k S on a jittered 10^3-atom lattice
    (8 unknowns per atom, n = 8000) for 32 poles on a half circle: one
    analysis for all poles, factor + selected inversion of the whole batch
    (one launch per level and kernel), against the same poles one after the
    other on a single-matrix plan.  Flops are counted as real flops (a
    complex multiply-add is 8 of them: 4x the real formulas)."""
    import numpy as np
    import torch
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    stream = torch.cuda.current_stream()
    t0 = time.time()
    H, Sm = W.hamiltonian_overlap(side=10, dofs=8, seed=6)
    z = W.poles(32, 0.0, 40.0)
    batch = S.Plan.poles(H, len(z)).bind(device=dev)
    vals = torch.as_tensor(np.concatenate([W.pencil_values(H, Sm, zk) for zk in z]), device=dev)
    out = torch.empty(int(batch.info["nnzL"]), dtype=torch.complex128, device=dev)
    log(f"[bench] poles: {len(z)} x n={H.n}, nnzL={batch.info['nnzL']} ({time.time() - t0:.1f}s)")

    def run_batch():
        batch.factor_complex(vals)
        batch.invert_complex(out)
    run_batch()
    batch.sync_status()
    ms_batch = _time(run_batch, max(1, args.steps // 2), stream)
    one = S.Plan.poles(H, 1).bind(device=dev)
    pv = [vals[int(batch.nnzA_off[k]):int(batch.nnzA_off[k + 1])] for k in range(len(z))]
    po = torch.empty(int(one.info["nnzL"]), dtype=torch.complex128, device=dev)

    def run_loop():
        for v in pv:
            one.factor_complex(v)
            one.invert_complex(po)
    run_loop()
    one.sync_status()
    ms_loop = _time(run_loop, max(1, args.steps // 5), stream)
    flops = 4.0 * (batch.info["flops_factor"] + batch.info["flops_selinv"])
    res = {"workload": "A(z) = H - z S, jittered 10^3-atom lattice x 8 (n=8000), 32 poles on a half circle "
                       "(center 0, radius 40), complex FP64",
           "poles": len(z), "n_per_pole": H.n, "nnzL_total": batch.info["nnzL"],
           "ms_batch": round(ms_batch, 4), "ms_per_pole_batched": round(ms_batch / len(z), 4),
           "ms_loop_one_pole_at_a_time": round(ms_loop, 4), "batch_speedup": round(ms_loop / ms_batch, 2),
           "gflops_real_equivalent": round(flops / (ms_batch * 1e-3) / 1e9, 2),
           "frac_of_fp64_peak": round(flops / (ms_batch * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)}
    log(f"[bench] poles: batch {ms_batch:.3f} ms ({ms_batch / len(z):.3f} ms/pole), one at a time {ms_loop:.3f} ms")
    del batch, one
    torch.cuda.empty_cache()
    return res


def measure_backward(plan, vals, out, fwd_ms, args, dev):
    """Reverse sweep (adjoint of factor + selected inversion) on the bench
    matrix for a seeded weight vector, timed against the forward step."""
    import numpy as np
    import torch
    from paper_1404_0447_amd import selinv as S
    if plan.blocks()["s"].max() > 128:
        return {"skipped": "execution blocks wider than 128 columns"}
    rng = np.random.default_rng(0)
    g = torch.as_tensor(rng.standard_normal(int(plan.info["nnzL"])), device=dev)
    gA = torch.empty(int(plan.info["nnzA"]), dtype=torch.float64, device=dev)
    plan.factor(vals)
    plan.invert(out)
    stream = torch.cuda.current_stream()
    for _ in range(max(1, args.warmup)):
        plan.backward(g, out=gA)
    bwd_ms = _time(lambda: plan.backward(g, out=gA), args.steps, stream)
    plan.profile(True)  # kernel split from a second, stamped run
    _time(lambda: plan.backward(g, out=gA), args.steps, stream)
    plan.profile(False)
    prof = plan.profile_read()
    plan.sync_status()
    log(f"[bench] backward {bwd_ms:.3f} ms/step ({bwd_ms / fwd_ms:.2f}x forward)")
    return {"fwd_ms": round(fwd_ms, 4), "bwd_ms": round(bwd_ms, 4), "bwd_over_fwd": round(bwd_ms / fwd_ms, 3),
            "kernels_ms": {k: round(prof[k][0] / args.steps, 4) for k in ("revsel", "revfac")},
            "target": "<= 3", "grad_probe": gA[:100000].cpu().numpy()}


def measure_batched(args, dev):
    """256 2D 5-point grids, sides U{32..96}, shifts U[0.01,1] (seed 3):
    batched persistent kernels replayed from a graph vs a loop of per-matrix
    plans launching per level.  Every matrix is checked against the oracle."""
    import numpy as np
    import torch
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    stream = torch.cuda.current_stream()
    t0 = time.time()
    ms = W.batch_2d()
    batch = S.Plan.batch(ms).bind(device=dev)
    vals = torch.as_tensor(np.concatenate([m.vals for m in ms]), device=dev)
    out = torch.empty(int(batch.info["nnzL"]), dtype=torch.float64, device=dev)
    log(f"[bench] batch: {len(ms)} matrices n={batch.info['n']} nnzL={batch.info['nnzL']} "
        f"blocks={batch.info['nblocks']} levels={batch.info['exec_depth']} ({time.time() - t0:.1f}s)")
    sched, tune_ms, _ = batch.tune(vals, out=out)
    log(f"[bench] batch tuned: {sched} {tune_ms:.3f} ms")
    for _ in range(max(1, args.warmup)):
        batch.run(vals, out=out, graph=True)
    batch.sync_status()
    reps = args.batch_reps
    ms_graph = _time(lambda: batch.run(vals, out=out, graph=True), reps, stream)
    ms_direct = _time(lambda: batch.run(vals, out=out), reps, stream)
    def union_levels():
        batch.factor(vals)
        batch.invert(out)
    union_levels()
    ms_union = _time(union_levels, reps, stream)
    batch.run(vals, out=out, graph=True)
    batch.sync_status()
    got = out.cpu().numpy()
    # per-matrix plans, per-level launches: the loop the batch replaces
    t0 = time.time()
    plans = [S.Plan.from_matrix(m).bind(device=dev) for m in ms]
    pv = [vals[int(batch.nnzA_off[k]):int(batch.nnzA_off[k + 1])] for k in range(len(ms))]
    po = [torch.empty(int(p.info["nnzL"]), dtype=torch.float64, device=dev) for p in plans]
    log(f"[bench] per-matrix plans ready ({time.time() - t0:.1f}s)")

    def loop():
        for p, v, o in zip(plans, pv, po):
            p.factor(v)
            p.invert(o)
    loop()
    for p in plans:
        p.sync_status()
    ms_loop = _time(loop, max(1, reps // 5), stream)
    # the largest member alone: a lower bound for any schedule of the batch
    # is the time of its longest dependency chain, which lies in the largest
    # grids (their top separators are the deepest chains of blocks)
    big = int(np.argmax([p.info["flops_factor"] + p.info["flops_selinv"] for p in plans]))
    pb, vb, ob = plans[big], pv[big], po[big]

    def one_member():
        pb.factor(vb)
        pb.invert(ob)
    one_member()
    ms_big = _time(one_member, reps, stream)
    pb.run(vb, out=ob, graph=True)
    ms_big_graph = _time(lambda: pb.run(vb, out=ob, graph=True), reps, stream)
    pb.sync_status()
    flops = batch.info["flops_factor"] + batch.info["flops_selinv"]
    res = {"workload": "256 2D 5-point grids, side U{32..96}, shift U[0.01,1], seed 3",
           "count": len(ms), "n": batch.info["n"], "nnzL": batch.info["nnzL"], "blocks": batch.info["nblocks"],
           "levels": batch.info["exec_depth"], "schedule": sched,
           "ms_graph": round(ms_graph, 4), "ms_persistent_direct": round(ms_direct, 4),
           "ms_union_per_level_launches": round(ms_union, 4), "ms_loop_per_matrix": round(ms_loop, 4),
           "speedup_vs_loop": round(ms_loop / ms_graph, 2),
           "speedup_graph_vs_union_per_level": round(ms_union / ms_graph, 3),
           "largest_member": {"n": int(pb.n), "ms_per_level": round(ms_big, 4),
                              "ms_persistent_graph": round(ms_big_graph, 4),
                              "batch_graph_over_largest": round(ms_graph / min(ms_big, ms_big_graph), 3)},
           "gflops_graph": round(flops / (ms_graph * 1e-3) / 1e9, 3)}
    log(f"[bench] batched graph {ms_graph:.3f} ms, direct {ms_direct:.3f} ms, union per-level {ms_union:.3f} ms, "
        f"loop {ms_loop:.3f} ms: speedup {ms_loop / ms_graph:.1f}x")
    log(f"[bench] largest member alone (n={pb.n}): per-level {ms_big:.3f} ms, persistent graph {ms_big_graph:.3f} ms")
    if not args.no_cpu:
        from oracle import oracle as O
        worst, cpu_s = 0.0, 0.0
        for k, m in enumerate(ms):
            o = O.symbolic(m, cap=128)
            ref, _, st, _, tf, ts = o.factor_selinv(m.vals)
            cpu_s += tf + ts
            l0, l1 = int(batch.nnzL_off[k]), int(batch.nnzL_off[k + 1])
            cp, ri = o.sym.colptrL, o.sym.rowindL
            d = ref[cp[:-1]]
            cols = np.repeat(np.arange(m.n), np.diff(cp))
            worst = max(worst, float(np.max(np.abs(got[l0:l1] - ref) / np.sqrt(np.abs(d[ri] * d[cols])))))
        res["max_err_vs_oracle"] = worst
        res["cpu_oracle_ms"] = round(cpu_s * 1e3, 2)
        res["cpu_oracle_cores"] = O.threads()
        log(f"[bench] batch vs oracle: max err {worst:.2e}; oracle {cpu_s:.2f}s")
    del plans
    return res


if __name__ == "__main__":
    main()
