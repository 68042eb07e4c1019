#!/usr/bin/env python3
"""Benchmark of the NPF hot path on one MI355X.

One step = one pass of the whole hot path over the workload: plan (Alg. 1 block sizing),
upper-index contraction, the lower-index chain, divisor / division, reduction to P_M
for every order, and the NPF assembly (Alg. 2), with inputs already resident in HBM.

Prints ONE JSON line: modal tensor entries per second (sum over orders of n * U_M
symmetric-unique entries per step / step time) for the selected precision, the same for
the plain FP64 GPU path, the error of both against the CPU FP64 oracle, the roofline of
the dominant kernel (timed live with HIP events on its launch stream) and the oracle's
own rate on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "modal tensor entries/s + MFMA util, split-BF16 vs FP64 GPU at ≤1e-6 rel err"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}   # dense MFMA, MI355X
PEAK_VALU_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 157.3}
HBM_GBPS = 8000.0
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16"}
SPLIT_PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Workspace cap per workload and precision (the memory limit of Alg. 1, applied to HBM);
# 0 = none.  The n=200 workload needs 5.4 GB (FP32 operands) or 10.8 GB (FP64) of chain
# buffers per output mode: 176 GB gives 7 blocks of 29 modes (FP32 operands), 192 GB 13
# blocks of 16 (FP64); the device holds 288 GB.
WORKLOAD_BUDGET = {"n128-o4-dense-resonant": {"*": 64 << 30},
                   "n200-o4-dense-hash": {"*": 176 << 30, "fp64": 192 << 30}}


def budget_for(workload, precision):
    b = WORKLOAD_BUDGET.get(workload, {})
    return b.get(precision, b.get("*", 0))


# Workloads whose oracle reference is stored (the oracle takes minutes per mode there).
STORED_REFERENCE = {"n200-o4-dense-hash": os.path.join(ROOT, "tests", "golden",
                                                       "hash200_modes.json")}


def reference_modes(s):
    """Output modes whose P rows and NPF columns the oracle computes: all of them for small
    systems, else the mode nearest an order-2 resonance and one fixed mode (each mode's
    chain is independent, so these rows are exact checks)."""
    import numpy as np
    if s.n <= 64:
        return list(range(s.n))
    lam = s.lam
    d2 = np.abs(lam[None, :, None] + lam[None, None, :] - lam[:, None, None]).reshape(s.n, -1)
    return sorted({int(np.argmin(d2.min(1))), 5})


def kernel_source_digest():
    """Digest of the HIP sources: counter summaries are valid only for the kernels they were
    taken on."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2509_08968_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic_<workload>_<precision>.json), or None when there is none or the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_digest") != kernel_source_digest():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


def kernel_work(name, sysm, plan):
    """(algorithmic flops, algorithmic HBM bytes, bound, uses MFMA) of ONE launch of a
    kernel, from the shapes (a complex multiply-add counts 8 flops, real x complex 4)."""
    n, J, U = sysm.n, plan.block_modes, plan.unique_tuples
    if name == "finalize":
        return 8.0 * n * n, 16.0 * 4 * n * n, "hbm", False
    M = int(name[1])
    what = name.split("_", 1)[1]
    if what == "psi_a":
        t = sysm.tensors[M - 2]
        if t.kind == 2:                      # generated on the device: no A traffic
            return 4.0 * n * J * U[M], 8.0 * J * U[M], "alu", False
        if t.kind == 1:
            nnz = int(t.desc.nnz)
            return 4.0 * nnz * J, 8.0 * nnz + 8.0 * J * U[M], "alu", False
        return 4.0 * n * J * U[M], 8.0 * n * U[M], "alu", False
    if what == "tucker_support":
        return 0.0, 0.0, "alu", False
    if what == "tucker_w":
        # W: about s^M complex multiply-adds per (p, k), s = support bound
        sm = sysm_support(sysm)
        return (8.0 * sm ** M * U[M - 1] * n, 16.0 * U[M - 1] * n * sm, "alu", False)
    if what == "tucker_psi":
        sm = sysm_support(sysm)
        return (8.0 * U[M - 1] * n * J * sm, 8.0 * U[M - 1] * n * J, "hbm", False)
    if what.startswith("stage"):
        i = int(what[5:])
        return (8.0 * J * n * U[i] * U[M - i], 8.0 * J * (U[i - 1] * U[M - i + 1] + U[i] * U[M - i]),
                "mfma", True)
    if what == "last_to_c":
        return 8.0 * J * n * U[M], 8.0 * J * (U[M - 1] * n) + 16.0 * J * U[M], "alu", False
    if what == "normal_form":
        return 20.0 * J * U[M], 32.0 * J * U[M], "hbm", False
    if what == "assemble":
        return 8.0 * J * n * U[M], 16.0 * J * U[M], "alu", False
    if what == "fused":
        return 16.0 * J * n * U[M], 8.0 * J * U[M - 1] * n, "mfma", True
    return 0.0, 0.0, "alu", False


def sysm_support(sysm):
    return getattr(sysm, "support_max", 0) or 8


def time_path(sysm, s, precision, steps, warmup, device, profile, budget=0, progress=False):
    """Time `steps` steps on a dedicated stream (graph replay after the first call), then,
    if `profile`, run the same steps eagerly with HIP events around every kernel launch.
    With `progress` (multi-second steps) every step is synchronised and logged."""
    import torch
    from paper_2509_08968_amd import binding as B

    n, N = s.n, s.order_max
    P = torch.empty((N - 1, n, n), dtype=torch.complex128, device=device)
    npf = torch.empty((n, n), dtype=torch.complex128, device=device)
    mk = lambda: B.Plan(n, N, precision, s.eps, s.tau, s.delta, budget_bytes=budget,
                        support_max=s.support_max)
    plan0 = mk()
    ws = plan0.workspace(device)
    stream = torch.cuda.Stream(device=device)       # default priority

    def step(plan):
        plan.run(sysm.tensors, sysm.U, sysm.V, sysm.lam, ws, P, npf, stream)

    torch.cuda.synchronize()
    for w in range(warmup):
        p = mk()
        step(p)
        p.close()
        if progress:
            torch.cuda.synchronize()
            log(f"[bench] {precision} warmup step {w + 1}/{warmup} done")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for i in range(steps):
        p = mk()                       # Alg. 1 block sizing is part of every step
        step(p)
        p.close()
        if progress:
            torch.cuda.synchronize()
            log(f"[bench] {precision} step {i + 1}/{steps} done")
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    out = {"ms_per_step": ms, "wall_ms_per_step": 1e3 * wall / steps, "kernels": {},
           "P": {M: P[M - 2].cpu().numpy() for M in range(2, N + 1)}, "npf": npf.cpu().numpy(),
           "plan": plan0}
    if profile:
        plans = []
        e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e2.record(stream)
        for i in range(steps):
            p = mk()
            p.profile(True)            # eager launches, an event pair around each kernel
            step(p)
            plans.append(p)
            if progress:
                torch.cuda.synchronize()
                log(f"[bench] {precision} profiled step {i + 1}/{steps} done")
        e3.record(stream)
        torch.cuda.synchronize()
        out["eager_ms_per_step"] = e2.elapsed_time(e3) / steps
        for p in plans:
            for k, (cnt, tot) in p.kernel_times().items():
                c0, t_ = out["kernels"].get(k, (0, 0.0))
                out["kernels"][k] = (c0 + cnt, t_ + tot)
            p.close()
    return out


def rel(a, b):
    import numpy as np
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def cpu_baseline(s, entries, target_s=10.0):
    """The oracle as it stands, timed on this host's cores over a bounded sample: the full
    workload repeated until about target_s seconds have passed (small systems), or one
    output mode of every order (large systems), scaled to modal entries per second."""
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    if s.n > 64:
        t0 = time.perf_counter()
        for M in s.orders:
            oracle.sym(s, M, modes=[0], nthreads=cores)
        el = time.perf_counter() - t0
        done = sum(math.comb(s.n + M - 1, M) for M in s.orders)
        return {"value": done / el, "unit": "modal entries/s", "cores": cores, "kind": "oracle",
                "sample": f"one output mode (mode 0) of orders {s.orders}: {done} entries in "
                          f"{el:.1f} s, packed-symmetric FP64 oracle with {cores} OpenMP threads"}
    reps, t0 = 0, time.perf_counter()
    while True:
        for M in s.orders:
            oracle.sym(s, M, nthreads=cores)
        reps += 1
        el = time.perf_counter() - t0
        if el >= target_s or reps >= 1000:
            break
    return {"value": entries * reps / el, "unit": "modal entries/s", "cores": cores,
            "kind": "oracle",
            "sample": f"full workload (all output modes, orders {s.orders}) x {reps} repeats, "
                      f"{el:.1f} s, packed-symmetric FP64 oracle with {cores} OpenMP threads"}


BATCH_WORKLOAD = "batch256-o3-blocksparse"
BATCH_BUDGET = 128 << 30


def copy_probe(args, device):
    """One device copy of --copy-probe-mib MiB before the workload: the reference that the
    HBM counter summaries scale every dispatch by."""
    import torch
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=device)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst


def bench_batch(args):
    """256 block-sparse systems (n uniform over even values in [32, 160], orders 2-3) in one
    batched call per step, replayed as a graph; per-system solo rates beside it."""
    import numpy as np
    import torch

    import oracle
    from paper_2509_08968_amd import binding as B
    from paper_2509_08968_amd import inputs as I

    device = "cuda:0"
    torch.cuda.set_device(0)
    B.lib()
    copy_probe(args, device)
    t0 = time.perf_counter()
    ss = I.workload_batch()
    devs = [B.upload_system(s, device) for s in ss]
    log(f"[bench] {len(ss)} systems generated and uploaded in {time.perf_counter() - t0:.1f} s")
    b = B.Batch(ss, BATCH_BUDGET)
    ws = b.workspace(device)
    P = [torch.empty((s.order_max - 1, s.n, s.n), dtype=torch.complex128, device=device) for s in ss]
    N = [torch.empty((s.n, s.n), dtype=torch.complex128, device=device) for s in ss]
    st = torch.cuda.Stream(device=device)
    tuned = None
    if not args.no_tune:
        tuned = b.tune(devs, ws, P, N, st)
    for _ in range(max(1, args.warmup)):
        b.run(devs, ws, P, N, st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        b.run(devs, ws, P, N, st)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    entries = b.report["modal_entries"]
    value = entries / (ms * 1e-3)
    log(f"[bench] batch: {ms:.3f} ms/step, {value:.3e} entries/s")

    # Oracle on sampled systems and modes.
    order = np.argsort([s.n for s in ss], kind="stable")
    rng = np.random.default_rng(I.BASE_SEED + 3 + 1000)
    picks = sorted({int(order[0]), int(order[-1]), *[int(x) for x in rng.choice(len(ss), 3, replace=False)]})
    errs = {}
    for q in picks:
        s = ss[q]
        modes = sorted({0, s.n // 2 + 1, s.n - 1})
        for M in s.orders:
            ref = oracle.sym(s, M, modes=modes)["P"]
            got = P[q][M - 2].cpu().numpy()[modes]
            errs[f"P{M}"] = max(errs.get(f"P{M}", 0.0), rel(got, ref))

    roof = None
    if not args.no_profile:
        launches = b.time_launches(devs, ws, P, N, st)
        tot = sum(L["ms"] for L in launches)
        L = max(launches, key=lambda x: x["ms"])
        achieved = L["flops"] / (L["ms"] * 1e-3) / 1e12
        name = (f"w{L['wave']}_np{L['npad']}_o{L['order']}_" +
                (f"stage{L['stage']}" if L["kind"] == 0 else "fused"))
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["bf16x3"],
                "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["bf16x3"],
                "traffic": measured_traffic(BATCH_WORKLOAD, "bf16x3", name),
                "kernel": name, "systems_in_launch": L["systems"],
                "workgroups": L["workgroups"], "avg_launch_ms": L["ms"],
                "algorithmic_flops": L["flops"],
                "share_of_step": L["ms"] / ms, "shared_launches_ms": tot,
                "executed_mfma_frac": achieved * SPLIT_PRODUCTS["bf16x3"] / PEAK_TFLOPS["bf16x3"],
                "timing": "HIP events around every shared launch, one eager run"}

    # Per-system rates: each system alone through npf_run (eager launches), same precision.
    solo = None
    if not args.no_solo:
        big = max(B.Plan(s.n, s.order_max, "bf16x3", support_max=s.support_max).workspace_bytes
                  for s in ss)
        del ws
        torch.cuda.empty_cache()
        wsolo = torch.empty(big, dtype=torch.uint8, device=device)
        rates, total = [], 0.0
        for q, s in enumerate(ss):
            plan = B.Plan(s.n, s.order_max, "bf16x3", s.eps, s.tau, s.delta,
                          support_max=s.support_max, graph=False)
            plan.run(devs[q].tensors, devs[q].U, devs[q].V, devs[q].lam, wsolo, P[q], N[q], st)
            a, c = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
            for _ in range(3):
                plan.run(devs[q].tensors, devs[q].U, devs[q].V, devs[q].lam, wsolo, P[q], N[q], st)
            c.record(st)
            torch.cuda.synchronize()
            t = a.elapsed_time(c) / 3
            total += t
            rates.append(plan.modal_entries / (t * 1e-3))
            plan.close()
        rates = np.asarray(rates)
        solo = {"launches": "eager (no graph)", "sum_ms": total, "batching_speedup": total / ms,
                "entries_per_s_min": float(rates.min()), "entries_per_s_median": float(np.median(rates)),
                "entries_per_s_max": float(rates.max())}
        log(f"[bench] solo: sum {total:.3f} ms, batching speedup {total / ms:.2f}x")

    cpu = None
    if not args.no_cpu_baseline:
        cores = max(1, min(len(os.sched_getaffinity(0)), 16))
        small = [ss[int(i)] for i in order[:24]]
        t0 = time.perf_counter()
        done = 0
        for s in small:
            for M in s.orders:
                oracle.sym(s, M, nthreads=cores)
                done += s.n * math.comb(s.n + M - 1, M)
        el = time.perf_counter() - t0
        cpu = {"value": done / el, "unit": "modal entries/s", "cores": cores, "kind": "oracle",
               "sample": f"the 24 smallest systems of the batch in full (orders 2-3, all modes): "
                         f"{done} entries in {el:.1f} s, packed-symmetric FP64 oracle with "
                         f"{cores} OpenMP threads"}

    line = {
        "metric": METRIC, "value": value, "unit": "modal entries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": BATCH_WORKLOAD, "systems": len(ss),
                   "n_range": [min(s.n for s in ss), max(s.n for s in ss)], "orders": [2, 3],
                   "precision": "bf16x3", "modal_entries_per_step": entries,
                   "waves": b.report["waves"], "workspace_bytes": b.report["workspace_bytes"],
                   "budget_bytes": BATCH_BUDGET, "launches_per_step": b.report["launches"],
                   "shared_launches": b.report["shared_launches"],
                   "autotuned_workgroups": tuned, "oracle_checked_systems": picks},
        "rel_err_vs_oracle": errs,
        "per_system_solo": solo,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="n64-o3-blocksparse")
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="timed steps of the FP64 comparison (default: --steps)")
    ap.add_argument("--fp64-warmup", type=int, default=None,
                    help="warmup steps of the FP64 comparison (default: --warmup)")
    ap.add_argument("--no-tune", action="store_true", help="batch workload: skip the autotuner")
    ap.add_argument("--no-solo", action="store_true", help="batch workload: skip per-system runs")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hot path is not sharded across GPUs "
              "(it would shard by output-mode block; each GPU's share runs as here).",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == BATCH_WORKLOAD:
        return bench_batch(args)

    import numpy as np
    import torch

    import oracle
    from paper_2509_08968_amd import binding as B
    from paper_2509_08968_amd import inputs as I

    device = "cuda:0"
    torch.cuda.set_device(0)
    B.lib()
    copy_probe(args, device)
    s = I.WORKLOADS[args.workload]()
    sysm = B.upload_system(s, device)
    log(f"[bench] workload {args.workload}: n={s.n} orders={s.orders}")

    # Oracle reference (outside every timed region): P rows and NPF columns of the modes.
    t0 = time.perf_counter()
    if args.workload in STORED_REFERENCE:
        g = json.load(open(STORED_REFERENCE[args.workload]))
        cplx = lambda a: np.asarray(a)[..., 0] + 1j * np.asarray(a)[..., 1]
        modes = g["modes"]
        refP = {M: cplx(g["P"][str(M)]) for M in s.orders}
        ref_npf = cplx(g["npf_columns"]).T
    else:
        modes = reference_modes(s)
        refP = {M: oracle.sym(s, M, modes=modes)["P"] for M in s.orders}
        zeta = s.delta * s.U[modes, :]
        ref_npf = s.V[:, modes] * (zeta + sum(refP.values())).T
    log(f"[bench] oracle reference ({len(modes)} modes) in {time.perf_counter() - t0:.1f} s")

    def errors(r):
        e = {f"P{M}": rel(r["P"][M][modes], refP[M]) for M in s.orders}
        e["npf"] = rel(r["npf"][:, modes], ref_npf)
        return e

    progress = s.n > 128
    res = time_path(sysm, s, args.precision, args.steps, args.warmup, device,
                    not args.no_profile, budget_for(args.workload, args.precision), progress)
    plan = res["plan"]
    entries = plan.modal_entries
    value = entries / (res["ms_per_step"] * 1e-3)
    err = errors(res)
    log(f"[bench] {args.precision}: {res['ms_per_step']:.3f} ms/step, {value:.3e} entries/s, err {err}")

    fp64 = None
    if args.precision != "fp64" and not args.no_fp64:
        torch.cuda.empty_cache()
        st64 = args.steps if args.fp64_steps is None else args.fp64_steps
        wu64 = args.warmup if args.fp64_warmup is None else args.fp64_warmup
        r64 = time_path(sysm, s, "fp64", st64, wu64, device, False,
                        budget_for(args.workload, "fp64"), progress)
        v64 = entries / (r64["ms_per_step"] * 1e-3)
        e64 = errors(r64)
        fp64 = {"value": v64, "ms_per_step": r64["ms_per_step"], "rel_err": e64,
                "speedup_of_selected": v64 and value / v64, "steps": st64, "warmup": wu64,
                "budget_bytes": budget_for(args.workload, "fp64")}
        log(f"[bench] fp64: {r64['ms_per_step']:.3f} ms/step, {v64:.3e} entries/s, err {e64}")

    roof = None
    if res["kernels"]:
        name, (cnt, tot) = max(res["kernels"].items(), key=lambda kv: kv[1][1])
        flops, byts, bound, mfma = kernel_work(name, sysm, plan)
        avg_s = tot / cnt * 1e-3
        if bound == "hbm":
            achieved, peak, unit = byts / avg_s / 1e9, HBM_GBPS, "GB/s"
        else:
            achieved = flops / avg_s / 1e12
            peak = (PEAK_TFLOPS if mfma else PEAK_VALU_TFLOPS)[args.precision]
            unit = "TFLOP/s"
        roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak,
                "traffic": measured_traffic(args.workload, args.precision, name),
                "algorithmic_bytes": byts, "kernel": name,
                "avg_launch_ms": tot / cnt, "launches_per_step": cnt / args.steps,
                "share_of_step": tot / args.steps / res["ms_per_step"],
                "timing": "HIP events around every launch, eager pass of the same steps"}
        if mfma:
            roof["executed_mfma_frac"] = achieved * SPLIT_PRODUCTS[args.precision] / peak
        log(f"[bench] kernels: " + ", ".join(f"{k}={v[1] / args.steps:.3f}ms"
                                             for k, v in sorted(res['kernels'].items())))

    cpu = None if args.no_cpu_baseline else cpu_baseline(s, entries)

    line = {
        "metric": METRIC, "value": value, "unit": "modal entries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.precision], "data": "synthetic",
        "config": {"workload": args.workload, "n": s.n, "orders": s.orders,
                   "precision": args.precision, "modal_entries_per_step": entries,
                   "block_modes": plan.block_modes, "blocks": plan.n_blocks,
                   "workspace_bytes": plan.workspace_bytes, "oracle_checked_modes": modes},
        "eager_ms_per_step": res.get("eager_ms_per_step"),
        "rel_err_vs_oracle": err,
        "fp64_gpu": fp64,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
